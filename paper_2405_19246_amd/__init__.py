"""MI355X-native entropic multi-marginal optimal transport with L1 cost.

The O(N)-per-marginal Sinkhorn of arXiv:2405.19246 as hand-written HIP kernels
for gfx950 behind a C ABI (include/mmot.h); `paper_2405_19246_amd.mmot` is the
ctypes binding and `paper_2405_19246_amd.inputs` the seeded synthetic
marginals.  Importing the package loads nothing; the binding loads libmmot.so
on first use and raises if it is not built.
"""
__version__ = "0.1.0"
