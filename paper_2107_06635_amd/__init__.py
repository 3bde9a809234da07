"""MI355X-native hot path of the neighbourhood tensor update (NTU).

The compute lives in ``libntu.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/ntu.h``).  Import :mod:`paper_2107_06635_amd.ntu` for the
binding; importing the package itself loads nothing.
"""
