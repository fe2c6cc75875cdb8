"""MI355X-native Yee/UPML FDTD for PCB power/ground-plane stacks.

``fdtd`` is the ctypes binding of ``libfdtd.so`` (the C-ABI declared in
``include/fdtd.h``; HIP kernels for gfx950 under ``csrc/``), ``build`` compiles it.
Batching, the autotuner and the serving loop sit on top of the binding.
"""
__all__ = ["fdtd", "build"]
