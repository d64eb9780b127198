"""MI355X-native butterfly-compressed multifrontal solver (HIP for gfx950).

The computation lives in libbfmf.so (C ABI in include/bfmf.h); ``bfmf`` is
its ctypes binding.
"""
