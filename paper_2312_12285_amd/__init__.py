"""ptalm -- direct point-to-harmonic transform (a_lm = sum_i w_i Y*_lm) on MI355X.

The compute path is the C-ABI library ``libptalm.so`` (hand-written HIP for
gfx950), reached from Python through :mod:`paper_2312_12285_amd.ptalm`.
Importing this package loads nothing; submodules are imported on demand.
"""
__all__ = ["ptalm", "synth"]
