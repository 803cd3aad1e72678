"""MI355X (gfx950) D2Q9 lattice Boltzmann hot path with half-way bounce-back on
moving solids, newborn-node refill and the conventional (Eq. 4) and
Galilean-invariant (Eq. 5) momentum-exchange force of Wen et al.,
arXiv:1303.0625.

The arithmetic lives in HIP kernels behind the C ABI of include/lbm.h
(liblbm.so); ``paper_1303_0625_amd.lbm`` is its ctypes binding.
"""
from . import lbm  # noqa: F401
from .lbm import Lattice, Lattice3D, LatticeBatch, WarmStartNet  # noqa: F401
