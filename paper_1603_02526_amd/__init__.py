"""MI355X-native factor-graph ADMM (message-passing ADMM of arXiv 1603.02526).

The compute path is the HIP library ``libadmm_hip.so`` (C ABI:
``include/admm.h``); ``paper_1603_02526_amd.admm`` is its thin ctypes
binding.  Importing this package loads nothing; the library is loaded on
first use and its absence is an error.
"""
__all__ = ["admm", "build"]
