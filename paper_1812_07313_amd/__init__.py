"""Barnes-Hut tree forces with monopole and traceless-quadrupole cell terms
over per-group interaction lists, on AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library ``libbhq.so`` (HIP kernels plus a
host list builder), reached through the thin ctypes binding in
``paper_1812_07313_amd.bhq``.  Importing this package loads nothing; the
library is loaded on first use of the binding.
"""
__all__ = ["bhq", "synth", "tune"]
