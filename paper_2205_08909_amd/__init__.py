"""MI355X-native fused matrix-free conjugate gradient (arXiv 2205.08909).

The solver lives in a C-ABI shared library (include/mfcg.h) built from HIP
sources for gfx950; `paper_2205_08909_amd.mfcg` is its thin ctypes binding.
Importing this package does not load the library.
"""
__all__ = ["mfcg", "inputs"]
