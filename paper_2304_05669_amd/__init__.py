"""MI355X-native hot path of Factorized Inverse Path Tracing (ICCV 2023).

The computation lives in libfipt.so (HIP kernels for gfx950 behind the C ABI
of include/fipt.h); ``paper_2304_05669_amd.fipt`` is its Python binding.
Importing this package loads nothing; import ``.fipt`` to use the library.
"""
__version__ = "1.0.0"
