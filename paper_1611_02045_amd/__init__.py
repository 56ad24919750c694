"""MI355X (gfx950) implementation of the hot path of the preconditioned nonlinear conjugate
gradient ground-state solver for the rotating Gross-Pitaevskii energy (arXiv:1611.02045).

The compute lives in libgpe.so (HIP kernels behind the C ABI of include/gpe.h); ``gpe`` is the
ctypes binding.  Import ``paper_1611_02045_amd.gpe`` explicitly to load the library.
"""

__all__ = ["gpe", "build"]
