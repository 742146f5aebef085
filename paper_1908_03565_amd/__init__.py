"""MI355X-native JPEG XL VarDCT reconstruction (coefficients -> RGB).

The compute path is the HIP library libjxlr.so (C ABI in include/jxlr.h);
`paper_1908_03565_amd.jxlr` is its ctypes binding.  The package import itself
is light: the binding loads the library on first use and raises if it is
missing.
"""
