"""MI355X-native probing / multi-shift Krylov log-determinant library.

The computation lives in libldq.so (HIP kernels for gfx950 behind the C ABI
of include/ldq.h); ``paper_1105_5256_amd.ldq`` is its ctypes binding and
``paper_1105_5256_amd.workloads`` draws the seeded synthetic inputs.
Importing this package loads nothing; the shared library is opened by the
first binding call.
"""
