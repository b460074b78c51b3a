"""MI355X (gfx950) implementation of the Newton-step linear solve of a fully
implicit two-phase reservoir simulator: CPR-preconditioned flexible GMRES
with Quasi-IMPES/ABF decoupling, local potential reordering, block
ILU(0)/RAS and aggregation AMG (Liu et al., arXiv 1701.06254).

The numerical work lives in libr2p.so (HIP kernels behind the C ABI of
include/r2p.h); `r2p` is its Python binding and `build` compiles it.
"""
from . import r2p  # noqa: F401

__all__ = ["r2p"]
