"""MI355X-native axion-coupled Yee/FDTD step (An et al., arXiv 2406.16796).

The compute path is the HIP library ``libaxf.so`` (kernels for gfx950 behind a
C ABI, declared in include/axf.h); ``paper_2406_16796_amd.axf`` is its thin
ctypes binding.  Importing this package does not load the library.
"""
__all__ = ["axf", "workloads"]
