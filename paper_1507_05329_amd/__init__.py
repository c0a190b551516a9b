"""libcola: the COLA particle-mesh step on AMD MI355X (HIP, gfx950).

The compute runs in libcola.so (C ABI in include/cola.h); this package holds
its ctypes binding, the torch-facing wrapper and the seeded input generators.
"""
