"""MI355X-native application of a local potential to plane-wave wave functions.

The compute path is libvloc.so (HIP kernels for gfx950 behind the C ABI in
include/vloc.h); ``paper_1601_07378_amd.vloc`` is its ctypes binding.
"""
