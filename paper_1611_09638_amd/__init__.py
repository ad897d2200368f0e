"""MI355X-native nonlinear reconstruction (Zhu, Yu, Pen, Chen & Yu, arXiv:1611.09638).

The displacement potential phi (x = xi + grad phi, positive-definite map) and
the reconstructed density delta_r = -laplacian phi are computed by hand-written
HIP kernels for gfx950 behind a C ABI (``include/recon.h``).  ``binding`` holds
the thin Python wrapper; ``inputs`` the seeded synthetic workloads.  Importing
the package loads nothing; ``binding`` loads the HIP library on first use.
"""
__all__ = ["binding", "inputs"]
