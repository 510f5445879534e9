"""MI355X-native iterative Fourier-transform hologram generation.

Gerchberg-Saxton and One-Step Phase-Retrieval holograms (Fourier or Fresnel;
phase-only, multi-level or binary SLMs) computed by hand-written HIP kernels
for gfx950 behind the C ABI in include/hologen.h.  ``hologen`` is the ctypes
binding; ``workloads`` holds the seeded synthetic inputs; ``build`` compiles
libhologen.so in-tree.  Importing the package loads nothing: the library is
opened on first use.
"""
__all__ = ["hologen", "workloads", "build"]
