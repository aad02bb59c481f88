"""FP64 CPU oracle for the GSRF hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package.  See
``oracle.gsrf_oracle`` for the definition it implements and the paper
passages it follows.
"""
from .gsrf_oracle import *  # noqa: F401,F403
from .gsrf_oracle import Params, Bands  # noqa: F401
