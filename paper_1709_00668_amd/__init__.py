"""MI355X (gfx950) implementation of the SamBaTen batch update.

The compute path is the HIP library libsambaten.so (csrc/, C ABI in
include/sambaten.h); `sambaten` is its ctypes binding.
"""
