"""MI355X (gfx950) library for the SU(3) adjoint-Laplacian hot path of RMHMC tooling.

``api`` binds the HIP library librmh.so (C ABI in include/rmh.h); ``autograd`` wraps
the kinetic energy as a torch.autograd.Function; ``inputs`` draws the seeded synthetic
links and fields.  Importing the package does not load the library; the first call
does, and raises if it has not been built.
"""
__all__ = ["api", "autograd", "inputs"]
