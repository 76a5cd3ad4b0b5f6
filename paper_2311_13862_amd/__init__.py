"""MI355X-native reduced-basis warm-start solver (Hou, Chen, Xia).

The compute path is the HIP library ``librbws.so`` (C ABI, ``include/rbws.h``);
``rbws`` is its thin ctypes binding.  Importing the package loads nothing;
importing ``paper_2311_13862_amd.rbws`` imports torch, then loads the library
against torch's HIP runtime, and raises if it is missing.
"""
__all__ = ["workloads", "rbws"]
