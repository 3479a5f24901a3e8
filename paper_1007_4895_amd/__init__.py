"""MI355X-native multiscale lattice Boltzmann hot path (Meng, Zhang & Shan).

The computation lives in liblb.so (HIP kernels for gfx950 behind the C ABI
of include/lb.h); ``lb`` is its ctypes binding, ``workloads`` the seeded
synthetic input recipes.  Importing this package loads nothing.
"""
__all__ = ["lb", "workloads", "build"]
