"""MI355X-native RK4 solver for the Higgs boson equation in de Sitter spacetime.

The compute path is libhb.so (HIP kernels for gfx950 behind the C ABI in
include/hb.h); ``paper_1803_01291_amd.hb`` is its ctypes binding.
"""
