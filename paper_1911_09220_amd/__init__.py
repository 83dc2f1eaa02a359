"""MI355X-native partial-assembly H1 diffusion/mass operators and PCG.

The compute path lives in libpafem.so (hand-written HIP for gfx950) behind the C
ABI of include/pafem.h; ``paper_1911_09220_amd.pafem`` is its ctypes binding.
Importing the binding fails if the library has not been built.
"""
__all__ = ["pafem"]
