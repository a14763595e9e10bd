"""MI355X-native coupled Yee-FDTD / quantum-emitter engine.

The compute path is ``libmlk.so`` (hand-written HIP kernels for gfx950 behind
a C ABI, declared in ``include/mlk.h``); ``paper_2512_06173_amd.mlk`` is its
ctypes binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""

__all__ = ["mlk", "workloads"]
