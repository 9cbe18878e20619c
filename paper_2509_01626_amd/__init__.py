"""MI355X-native STZ streaming compressor hot path (HIP, gfx950).

The compute path lives in the HIP shared library built from ``csrc/`` and is
reached through ``stz`` (ctypes binding of the C ABI declared in
``include/stz.h``).
"""
