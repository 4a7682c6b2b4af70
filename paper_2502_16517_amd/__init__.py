"""MI355X-native temporary AoS-to-SoA views around SPH particle-interaction
kernels (arxiv 2502.16517).  The product is libsphview.so (HIP for gfx950,
C-ABI in include/sphview.h); ``sphview`` is its ctypes binding and ``inputs``
the seeded synthetic particle sets."""
__all__ = ["sphview", "inputs"]
