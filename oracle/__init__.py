"""CPU oracle for entropic multi-marginal optimal transport with L1 cost.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this folder; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.

Contents
  dense.py       the plain definition: the full N^l cost tensor, the Gibbs
                 kernel and generalised (Gauss-Seidel) Sinkhorn, FP64, in the
                 log domain (Sec. 2, Alg. 1; Sec. 4.2 for l marginals).
  paper_ftvp.py  the paper's own O(N) recurrences for l = 3 written from its
                 equations (Sec. 3.1 FTVP-1, Sec. 3.2 FTVP-2), linear domain,
                 with the two printed mistakes corrected (see that file).
  fastcheck.c    an O(N) FP64 log-domain checker for any l (a subset-lattice
                 dynamic program, derived in the file header), used where the
                 dense tensor does not fit; pinned against dense.py by tests.
  fastcheck.py   ctypes loader for fastcheck.c.
"""
