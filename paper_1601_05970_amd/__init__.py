"""Galerkin-FFT Newton--CG micromechanics solver for AMD MI355X (gfx950).

The product is libfftg.so (HIP kernels + C ABI, include/fftg.h); the
``fftg`` module is its thin ctypes binding.  Importing the package does not
load the library; ``fftg.lib()`` does, and raises if it is missing.
"""
__all__ = ["fftg", "build"]
