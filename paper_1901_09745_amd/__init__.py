"""MI355X (gfx950) partially-saturated-cell lattice Boltzmann hot path of
Liu & Wu (arXiv 1901.09745).

The compute path lives in ``libpsclbm.so`` (HIP kernels behind the C ABI of
include/psclbm.h); ``paper_1901_09745_amd.psclbm`` is its ctypes binding and
``paper_1901_09745_amd.autograd`` the adjoint's torch.autograd.Function.
Importing this package does not load the library; the binding does, and
raises if it is missing.
"""
__all__ = ["psclbm"]
