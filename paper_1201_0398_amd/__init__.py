"""MI355X (gfx950) AES block encryption: T-table rounds in hand-written HIP
kernels behind a C ABI (``include/aesgpu.h``).

``paper_1201_0398_amd.aesgpu`` is the ctypes binding (loads ``libaesgpu.so``,
needs torch and a built library); ``workloads`` holds the seeded synthetic
inputs; ``build`` compiles the library.  The binding is imported lazily so
that the input generators work without a GPU.
"""
