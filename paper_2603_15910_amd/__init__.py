"""MI355X-native CQK / simplex / l1 projection library (HIP, gfx950).

The compute path lives in the HIP shared library ``libcqk.so`` (built from
``csrc/``); this package is a thin ctypes binding over its C ABI.  The library
is loaded on first use and a missing build raises an error: there is no CPU
fallback.
"""
