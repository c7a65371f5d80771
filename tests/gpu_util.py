"""Helpers for the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


# Bar for one FP32-scan product or one FP32 sweep against the FP64 oracle (relative
# error of J, or of the potentials).  The products round in FP32 (unit roundoff
# 2^-24 = 6.0e-8) through a few dozen operations whose errors decay with the
# discount factors; measured: 1.6e-7 .. 7.7e-7 over every FP32 product and
# one-sweep test (l = 3..10, uniform and graded grids, one wavefront, teams and
# tiles).  The bar is 4e-6, about 67 roundings: a five-fold margin over the
# largest error seen, so a regression of ten times fails.
FP32_TOL = 4e-6


def say(msg: str) -> None:
    """Name the case before a GPU step, flushed, so a failing run shows where it was."""
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def to_dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev())


def log_rel_err(got_log: np.ndarray, ref_log: np.ndarray, mag_ulps: float = 0.0) -> float:
    """Largest relative error of exp(got) vs exp(ref), pointwise, from logs.

    Entries where both are -inf (exact zeros) agree; one -inf alone is an error.
    mag_ulps > 0 discounts the part an FP64 log of that size cannot resolve:
    a log of magnitude |x| is itself only known to |x| * 2^-53 absolute, so
    each difference is reduced by mag_ulps * |x| * 2^-53 before it is compared.
    """
    got_log = np.asarray(got_log, dtype=np.float64)
    ref_log = np.asarray(ref_log, dtype=np.float64)
    both = np.isneginf(got_log) & np.isneginf(ref_log)
    if np.any(np.isneginf(got_log) != np.isneginf(ref_log)):
        return np.inf
    d = np.abs(got_log[~both] - ref_log[~both])
    if mag_ulps > 0:
        d = np.maximum(0.0, d - mag_ulps * np.abs(ref_log[~both]) * 2.0 ** -53)
    return float(np.max(np.expm1(d))) if d.size else 0.0


def gauge_fix(a: np.ndarray) -> np.ndarray:
    """Representative of the potentials modulo the gauge of the Gibbs form.

    Adding constants c_q with sum_q c_q = 0 to the rows a_q leaves the plan
    K * prod_q exp(a_q) unchanged, so only this class is determined by the
    plan: shift rows 0..l-2 to mean zero over their finite entries and move
    the sum of the shifts into the last row.
    """
    a = np.array(a, dtype=np.float64)
    tot = 0.0
    for q in range(a.shape[0] - 1):
        fin = np.isfinite(a[q])
        c = float(np.mean(a[q][fin])) if fin.any() else 0.0
        a[q] -= c
        tot += c
    a[-1] += tot
    return a


def potentials_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max |a_got - a_ref| / max(1, |a_ref|) after fixing the gauge of both."""
    got, ref = gauge_fix(got), gauge_fix(ref)
    fin = np.isfinite(ref)
    if np.any(np.isfinite(got) != fin):
        return np.inf
    return float(np.max(np.abs(got[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin])))) if fin.any() else 0.0
