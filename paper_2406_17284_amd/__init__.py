"""MI355X-native Larger-than-Life stepping with banded MFMA products (CAT, arXiv 2406.17284).

The compute path is the C-ABI library ``libltl.so`` built from ``csrc/`` (HIP for
gfx950); :mod:`paper_2406_17284_amd.ltl` is its thin ctypes binding and
:mod:`paper_2406_17284_amd.inputs` holds the seeded synthetic workloads.
Importing the package loads nothing native.
"""
__all__ = ["inputs", "ltl"]
