"""MI355X-native contracting-grid event reconstruction (ANTS2, arXiv:1602.07247).

The hot path is the HIP library libants.so (sources in csrc/, C ABI in
include/ants.h); `ants` is its ctypes binding.
"""
