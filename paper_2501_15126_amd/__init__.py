"""MI355X-native sparse matrix permanent (Gray-code Nijenhuis-Wilf / Ryser).

The compute path lives in the C-ABI library ``libperm_mi355x.so`` (HIP host
code, hipRTC-generated gfx950 kernels and a precompiled reduction kernel).
``paper_2501_15126_amd.perm`` is its thin ctypes binding.  Nothing is loaded
at import time of this package.
"""
__all__ = ["perm", "workloads"]
