"""MI355X (gfx950) implementation of the double-distribution cascaded
central-moment lattice Boltzmann method for 3D thermal convection
(Hajabdollahi & Premnath, arXiv:1710.04751).

The method runs in the HIP library liblbm.so (C ABI in include/lbm.h);
`capi` binds it under the same names and `solver.Cavity` manages device
memory and streams through PyTorch.
"""
from . import capi  # noqa: F401

__all__ = ["capi"]
