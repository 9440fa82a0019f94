"""MI355X-native adjoint lattice-Boltzmann hot path (gfx950 HIP kernels behind a C ABI).

Importing the package loads nothing; the HIP library is opened on first use of
``paper_1501_04741_amd.lbm`` (and fails loudly if it has not been built).
"""
__all__ = ["inputs", "lbm", "autograd", "serve"]
