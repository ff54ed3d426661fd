"""MI355X (gfx950) implementation of the per-solution-interval Jones-chain
gain solver of QuartiCal (Kenyon et al., arXiv 2412.10072).

The solver runs in hand-written HIP kernels in ``libqc.so`` behind the C-ABI
of ``include/qc.h``; ``qc`` is the ctypes binding (argument marshalling only).
"""
__all__ = ["qc", "build"]
