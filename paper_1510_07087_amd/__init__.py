"""MI355X-native directional H2-matrix compression.

The computation lives in the native library libdh2.so (C ABI in
include/dh2.h; host plan in C++, hot path in gfx950 HIP kernels).  The
module ``dh2`` is its thin Python binding.
"""
