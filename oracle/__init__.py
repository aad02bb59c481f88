"""FP64 CPU oracle for the GSRF hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package.  See
``oracle.gsrf_oracle`` (render, binning, gradients) and ``oracle.train_oracle``
(losses, attribute update) for the definitions they implement and the paper
passages they follow.
"""
from .gsrf_oracle import *  # noqa: F401,F403
from .gsrf_oracle import Params, Bands  # noqa: F401
from . import train_oracle  # noqa: F401
