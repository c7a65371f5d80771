"""Three marginals on a 2-D grid with separable L1 cost (Sec. 4.1).  TEST
INFRASTRUCTURE ONLY (see oracle/__init__.py).

Marginal q is an N x M array stored as a[q, i2, i1] (i1 = 0..N-1 along the first
axis with spacing h1, i2 = 0..M-1 along the second with spacing h2), i.e. the
paper's column-major flattening phi = (phi_1, ..., phi_M) with phi_{i2} in R^N.
The cost of a triple of points is
    c = h1 (|i1 - j1| + |i1 - k1| + |j1 - k1|) + h2 (|i2 - j2| + |i2 - k2| + |j2 - k2|),
so K = K_1 (x) K_2 with K_1 = lambda_1^{...}, lambda_1 = exp(-h1/eps), and the
same along the second axis (Sec. 4.1, kernel of the 2-D problem).

Two references:
  * dense2d_*: the (NM)^3 tensors written out (plain definition);
  * product / objective: the paper's reduction of the 2-D product to 1-D ones,
    J_{k2} = sum_{i2, j2} K_2(i2, j2, k2) (K_N x_{i1} phi_{i2} x_{j1} psi_{j2})
    (Sec. 4.1), with the sums over the second-axis indices written out
    (O(M^3) 1-D products of length N, from oracle/fastcheck.c) -- slow, but
    each term is the definition.  The objective splits the same way:
    <C, T> = sum over second-axis triples of K_2 times (h1 <phi_j, FTVP-2 along
    the first axis> + h2 E_2 <phi_j, FTVP along the first axis>).
Everything is in the log domain.  Pinned in tests/test_oracle_twod.py.
"""
from __future__ import annotations

import itertools

import numpy as np

from oracle import fastcheck


def _lse(x):
    x = np.asarray(x, dtype=np.float64)
    m = np.max(x)
    if not np.isfinite(m):
        return m
    return m + np.log(np.sum(np.exp(x - m)))


def _lse0(T):
    """log sum exp over axis 0 of a 2-D array, column by column, with a max shift."""
    m = np.max(T, axis=0)
    ms = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        return np.log(np.sum(np.exp(T - ms), axis=0)) + ms


def _e3(i, j, k):
    return abs(i - j) + abs(i - k) + abs(j - k)


# ---- dense definition -------------------------------------------------------------

def dense2d_log_kernel(N: int, M: int, h1: float, h2: float, eps: float) -> np.ndarray:
    """log K over points p = (i2, i1) of the three marginals: shape (M, N, M, N, M, N)."""
    i1 = np.arange(N)
    i2 = np.arange(M)
    E1 = (np.abs(i1[:, None, None] - i1[None, :, None]) + np.abs(i1[:, None, None] - i1[None, None, :]) +
          np.abs(i1[None, :, None] - i1[None, None, :]))
    E2 = (np.abs(i2[:, None, None] - i2[None, :, None]) + np.abs(i2[:, None, None] - i2[None, None, :]) +
          np.abs(i2[None, :, None] - i2[None, None, :]))
    # axes (a2, a1, b2, b1, c2, c1)
    L = -(h1 / eps) * E1[None, :, None, :, None, :] - (h2 / eps) * E2[:, None, :, None, :, None]
    return L


def dense2d_cost(N: int, M: int, h1: float, h2: float) -> np.ndarray:
    i1 = np.arange(N)
    i2 = np.arange(M)
    E1 = (np.abs(i1[:, None, None] - i1[None, :, None]) + np.abs(i1[:, None, None] - i1[None, None, :]) +
          np.abs(i1[None, :, None] - i1[None, None, :]))
    E2 = (np.abs(i2[:, None, None] - i2[None, :, None]) + np.abs(i2[:, None, None] - i2[None, None, :]) +
          np.abs(i2[None, :, None] - i2[None, None, :]))
    return h1 * E1[None, :, None, :, None, :] + h2 * E2[:, None, :, None, :, None]


def _log_plan(logK, a):
    return (logK + a[0][:, :, None, None, None, None] + a[1][None, None, :, :, None, None] +
            a[2][None, None, None, None, :, :])


def dense2d_product(logK: np.ndarray, a: np.ndarray, j: int) -> np.ndarray:
    """log (K x_{q != j} phi_q), shape (M, N), from the dense tensor (row j of a ignored)."""
    b = np.array(a, dtype=np.float64)
    b[j] = 0.0
    T = _log_plan(logK, b)
    axes = tuple(ax for q in range(3) if q != j for ax in (2 * q, 2 * q + 1))
    m = np.max(T, axis=axes, keepdims=True)
    ms = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        s = np.log(np.sum(np.exp(T - ms), axis=axes, keepdims=True)) + ms
    return np.squeeze(s, axis=axes)


def dense2d_sinkhorn(u: np.ndarray, h1: float, h2: float, eps: float, itmax: int) -> dict:
    """Gauss-Seidel updates phi_j <- u_j / (K x_{q != j} phi_q), j = 0, 1, 2 (Sec. 4.1 update
    formulas), from phi = 1/(NM); Res = errors of marginals 0 and 1 after the last sweep."""
    _, M, N = u.shape
    logK = dense2d_log_kernel(N, M, h1, h2, eps)
    with np.errstate(divide="ignore"):
        lu = np.log(u)
    a = np.full(u.shape, -np.log(N * M))
    for _ in range(itmax):
        for j in range(3):
            a[j] = lu[j] - dense2d_product(logK, a, j)
    res = sum(float(np.sum(np.abs(np.exp(a[j] + dense2d_product(logK, a, j)) - u[j]))) for j in range(2))
    T = np.exp(_log_plan(logK, a))
    W = float(np.sum(dense2d_cost(N, M, h1, h2) * T))
    return dict(log_phi=a, res=res, W=W, plan=T)


# ---- reduction to 1-D products (Sec. 4.1) ---------------------------------------

def ftvp(log_u: np.ndarray, log_v: np.ndarray, h1: float, eps: float) -> np.ndarray:
    """log (K_N x_{i1} u x_{j1} v): the 1-D three-marginal product along the first axis."""
    N = log_u.shape[0]
    rows = np.stack([log_u, log_v, np.zeros(N)])
    return fastcheck.marginal_product_log(rows, 2, h1, eps)


def _others(j):
    return [q for q in range(3) if q != j]


def product(a: np.ndarray, j: int, h1: float, h2: float, eps: float) -> np.ndarray:
    """log J_j, shape (M, N): J_{k2} = sum_{i2, j2} lambda_2^{E_2(i2, j2, k2)} FTVP(phi_{i2}, psi_{j2})."""
    _, M, N = a.shape
    p, q = _others(j)
    lam2 = -h2 / eps
    F = {}
    for i2, j2 in itertools.product(range(M), repeat=2):
        F[i2, j2] = ftvp(a[p, i2], a[q, j2], h1, eps)
    out = np.empty((M, N))
    for k2 in range(M):
        terms = np.stack([lam2 * _e3(i2, j2, k2) + F[i2, j2] for i2, j2 in itertools.product(range(M), repeat=2)])
        out[k2] = _lse0(terms)
    return out


def objective(a: np.ndarray, h1: float, h2: float, eps: float) -> float:
    """W = <C, T> (Sec. 4.1, 2-D distance): over second-axis triples (i2, j2, k2), the
    weight lambda_2^{E_2} times h1 <phi_{k2}, FTVP-2 along the first axis> plus h2 E_2
    <phi_{k2}, FTVP along the first axis>; the first-axis parts are the 1-D objective
    and product of oracle/fastcheck.c."""
    _, M, N = a.shape
    total = 0.0
    for i2, j2, k2 in itertools.product(range(M), repeat=3):
        e2 = _e3(i2, j2, k2)
        w2 = np.exp(-(h2 / eps) * e2)
        rows = np.stack([a[0, i2], a[1, j2], a[2, k2]])
        wx = fastcheck.objective(rows, h1, eps)                 # h1 <phi_2, (E_1 K_1) x phi_0 x phi_1>
        px = np.exp(_lse(a[2, k2] + fastcheck.marginal_product_log(rows, 2, h1, eps)))
        total += w2 * (wx + h2 * e2 * px)
    return total


def marginal_errors(u: np.ndarray, a: np.ndarray, h1: float, h2: float, eps: float) -> np.ndarray:
    return np.array([float(np.sum(np.abs(np.exp(a[j] + product(a, j, h1, h2, eps)) - u[j]))) for j in range(3)])


def sinkhorn(u: np.ndarray, h1: float, h2: float, eps: float, itmax: int) -> dict:
    """Gauss-Seidel sweeps (Sec. 4.1 update formulas) with the products above, from
    phi = 1/(NM); Res = errors of marginals 0 and 1 after the last sweep."""
    _, M, N = u.shape
    with np.errstate(divide="ignore"):
        lu = np.log(u)
    a = np.full(u.shape, -np.log(N * M))
    for _ in range(itmax):
        for j in range(3):
            a[j] = lu[j] - product(a, j, h1, h2, eps)
    err = marginal_errors(u, a, h1, h2, eps)
    return dict(log_phi=a, res=float(err[:2].sum()), W=objective(a, h1, h2, eps))
