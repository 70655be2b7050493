"""libscitv: GAP-TV / ADMM-TV reconstruction for snapshot video compressive
imaging on AMD Instinct MI355X (gfx950).

The compute path is the C-ABI shared library ``libscitv.so`` (hand-written
HIP kernels); :mod:`paper_2005_08028_amd.scitv` is its thin Python binding.
Importing the package does not load the library; the binding does, and it
raises if the library is missing.
"""
__all__ = ["scitv", "synth"]
