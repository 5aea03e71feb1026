"""MI355X-native LLOID filtering path: gfx950 HIP kernels behind the C ABI in
include/lloid.h, with a thin ctypes binding (paper_2410_16416_amd.lloid)."""
