"""MI355X-native nested-grid particle-mesh field solve (HIP kernels for gfx950).

The C ABI is declared in include/sbx.h; `paper_1210_1736_amd.sbx` is its
ctypes binding (importing it loads libsbx.so and fails if it is not built).
"""
__all__ = ["sbx"]
