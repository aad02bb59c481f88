"""MI355X (gfx950) implementation of GSRF's data-parallel hot path (arXiv 2502.01826).

The work happens in libgsrf.so (HIP): splatting of complex 3D Gaussians onto a
receiver's ray grid, per-tile depth sorting and complex front-to-back ray
accumulation, forward and adjoint.  This package is the thin Python binding.
"""
from .render import GSRFRender, GridSpec, Problem, pack_pairs, render  # noqa: F401
