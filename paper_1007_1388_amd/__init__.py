"""MI355X-native patch-and-block D3Q19 lattice Boltzmann library.

The compute path lives in the HIP library ``liblbm_hip.so`` (built from
``csrc/``) behind the C ABI declared in ``include/lbm.h``; ``lbm`` is the thin
ctypes binding with the same names.  Importing this package loads nothing;
``paper_1007_1388_amd.lbm`` loads the library on first use and raises if it
is missing.
"""
__all__ = ["inputs", "lbm"]
