"""Acc-Sinkhorn for entropy-regularized optimal transport on AMD MI355X (gfx950).

The solver lives in the HIP library ``libaccsk.so`` (sources under ``csrc/``,
C-ABI in ``include/accsk.h``).  ``paper_2605_30267_amd.accsk`` is the thin
ctypes binding; it loads the library on first use and raises if it is missing.
"""
__all__ = ["accsk", "workloads"]
