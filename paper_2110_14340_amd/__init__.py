"""MI355X-native runtime for K-partitioned OpenACC-style parallel loop nests.

The compute path is the C-ABI library ``libjacc.so`` (hand-written HIP for
gfx950 plus a C++ runtime); ``paper_2110_14340_amd.jacc`` is its thin ctypes
binding.  Importing this package loads nothing; ``jacc`` loads the library
on first use and raises if it is missing.
"""
__all__ = ["jacc", "inputs"]
