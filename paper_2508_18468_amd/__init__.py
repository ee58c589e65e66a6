"""Monitored free-fermion quantum trajectories on AMD MI355X (gfx950).

The compute path is the HIP library ``libmfq.so`` (C ABI in include/mfq.h),
built in-tree by ``__graft_entry__.build()``.  ``paper_2508_18468_amd.mfq`` is
its ctypes binding; nothing is loaded at import time.
"""

__all__ = ["mfq", "workloads"]
