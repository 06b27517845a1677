"""MI355X (gfx950) regularised spiral-MRI reconstruction.

Hot path (HIP, behind the C ABI in include/recon.h): exact NUDFT adjoint and
forward on the matrix cores, FP64 Gram kernel, LDS-staged Stockham FFT
Toeplitz apply and fused pseudo-conjugate-gradient kernels.  ``recon`` is the
ctypes binding; ``build`` compiles the library.
"""
__all__ = ["recon", "build"]
