"""MI355X-native Euler-characteristic curves of 2D/3D fields (vertex contributions).

The compute path is the HIP library ``libecc.so`` behind the C ABI declared in
``include/ecc.h``; :mod:`paper_2311_11740_amd.ecc` is its ctypes binding.
Importing this package loads nothing; the library is opened on first use.
"""
__all__ = ["ecc", "synth"]
