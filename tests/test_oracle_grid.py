"""Pins of the oracle on non-uniform grids and unequal supports.

Every marginal lives on the same non-decreasing coordinates x[0..N-1]; a
marginal with a smaller support carries zeros elsewhere.  The dense oracle forms
c = sum_{p<q} |x[i_p] - x[i_q]| directly; the C checker walks the gaps with
per-gap factors exp(-(x_{k+1} - x_k) m (l - m) / eps).  The pins:
  * the gap identity on coordinates, by enumeration;
  * an affine grid equals the uniform grid of its step;
  * checker == dense for products, objective, errors and Sinkhorn, l = 2..8,
    with zero scaling factors, large potentials and repeated coordinates;
  * the eps -> 0 limit: the 1-D pairwise-L1 problem is solved by the quantile
    (comonotone) coupling, so W_eps >= sum_{p<q} int |F_p - F_q| dx and tends to it.
"""
import itertools

import numpy as np
import pytest

from oracle import dense, fastcheck
from paper_2405_19246_amd import inputs


def _grid(N, seed, repeat=False):
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.uniform(0.2, 1.8, N)) / N
    if repeat and N > 3:
        x[2] = x[1]  # a zero-length gap
    return x - x[0]


def test_gap_identity_on_coordinates():
    # sum_{p<q} |x_{i_p} - x_{i_q}| = sum_k (x_{k+1} - x_k) m_k (l - m_k), m_k = #{q : i_q <= k}
    for l, N in [(2, 5), (3, 5), (4, 4), (5, 3)]:
        x = _grid(N, 10 * l + N)
        C = dense.cost_tensor_grid(l, x)
        for idx in itertools.product(range(N), repeat=l):
            g = 0.0
            for k in range(N - 1):
                m = sum(1 for i in idx if i <= k)
                g += (x[k + 1] - x[k]) * m * (l - m)
            assert abs(C[idx] - g) <= 1e-14 * max(1.0, g)


def test_affine_grid_equals_uniform_grid():
    l, N, eps = 4, 9, 0.05
    h = 0.125
    x = 3.0 + h * np.arange(N)
    np.testing.assert_allclose(dense.log_kernel(l, N, 0.0, eps, x), dense.log_kernel(l, N, h, eps),
                               rtol=1e-13, atol=1e-13)
    rng = np.random.default_rng(4)
    a = rng.normal(size=(l, N))
    for j in range(l):
        np.testing.assert_allclose(fastcheck.marginal_product_log(a, j, 0.0, eps, x),
                                   fastcheck.marginal_product_log(a, j, h, eps), rtol=1e-13)
    assert abs(fastcheck.objective(a, 0.0, eps, x) - fastcheck.objective(a, h, eps)) <= \
        1e-13 * abs(fastcheck.objective(a, h, eps))


_LN = [(2, 12), (3, 10), (4, 8), (5, 6), (6, 5), (7, 4), (8, 3)]


@pytest.mark.parametrize("l,N", _LN)
def test_checker_matches_dense_on_grid(l, N):
    x = _grid(N, 7 * l + N, repeat=(l <= 5))
    eps = 0.07
    rng = np.random.default_rng(l * 100 + N)
    a = rng.normal(size=(l, N)) * 3.0
    a[0, min(1, N - 1)] = -np.inf
    a[l - 1, N - 1] += 800.0  # large potentials stay exact in the log domain
    logK = dense.log_kernel(l, N, 0.0, eps, x)
    for j in range(l):
        ref = dense.marginal_product_log(logK, a, j)
        got = fastcheck.marginal_product_log(a, j, 0.0, eps, x)
        fin = np.isfinite(ref)
        assert np.array_equal(fin, np.isfinite(got))
        np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-13, atol=1e-12)
    b = rng.normal(size=(l, N))
    Wd = dense.objective(l, N, 0.0, eps, b, x)
    assert abs(fastcheck.objective(b, 0.0, eps, x) - Wd) <= 1e-12 * abs(Wd)
    u = rng.uniform(0.1, 1.0, size=(l, N))
    u /= u.sum(axis=1, keepdims=True)
    ed = np.array([np.sum(np.abs(np.exp(b[j] + dense.marginal_product_log(logK, b, j)) - u[j])) for j in range(l)])
    np.testing.assert_allclose(fastcheck.marginal_errors(u, b, 0.0, eps, x), ed, rtol=1e-12)


@pytest.mark.parametrize("l,N,its", [(3, 9, 30), (5, 5, 12), (7, 3, 8)])
def test_checker_sinkhorn_matches_dense_on_grid(l, N, its):
    x = _grid(N, l + 3 * N)
    eps = 0.05
    rng = np.random.default_rng(its)
    u = rng.uniform(0.1, 1.0, size=(l, N))
    u[1, 0] = 0.0  # a point outside marginal 1's support
    u /= u.sum(axis=1, keepdims=True)
    rd = dense.sinkhorn(u, 0.0, eps, itmax=its, x=x)
    rf = fastcheck.sinkhorn(u, 0.0, eps, itmax=its, check_every=its, x=x)
    fin = np.isfinite(rd["log_phi"])
    assert np.array_equal(fin, np.isfinite(rf["log_phi"]))
    assert not fin[1, 0]
    np.testing.assert_allclose(rf["log_phi"][fin], rd["log_phi"][fin], rtol=1e-11, atol=1e-11)
    assert abs(rf["W"] - rd["W"]) <= 1e-12 * abs(rd["W"])
    assert abs(rf["res"] - rd["res"]) <= 1e-10 * max(rd["res"], 1e-300)


def test_unequal_supports_converge_to_the_given_marginals():
    # three marginals on different supports, merged onto one sorted grid
    rng = np.random.default_rng(9)
    supports = [np.sort(rng.uniform(0, 1, n)) for n in (7, 11, 5)]
    weights = [rng.uniform(0.2, 1.0, len(s)) for s in supports]
    x, u = inputs.merge_supports(supports, weights)
    l, N = u.shape
    assert N == 23 and np.all(np.diff(x) > 0)
    r = fastcheck.sinkhorn(u, 0.0, 0.05, itmax=20000, tol=1e-12, check_every=10, x=x)
    assert r["res"] <= 1e-12
    logK = dense.log_kernel(l, N, 0.0, 0.05, x)
    M = dense.plan_marginals(logK, r["log_phi"])
    np.testing.assert_allclose(M, u, atol=1e-12)
    assert np.all(np.isneginf(r["log_phi"][u == 0.0]))


@pytest.mark.parametrize("l", [2, 3])
def test_small_eps_tends_to_the_quantile_coupling_cost(l):
    N = 25
    x = _grid(N, 50 + l)
    rng = np.random.default_rng(l)
    u = rng.uniform(0.1, 1.0, size=(l, N))
    u /= u.sum(axis=1, keepdims=True)
    F = np.cumsum(u, axis=1)
    W0 = sum(float(np.sum(np.abs(F[p, :-1] - F[q, :-1]) * np.diff(x)))
             for p in range(l) for q in range(p + 1, l))
    Ws = []
    for eps in (0.02, 0.005, 0.001):
        r = fastcheck.sinkhorn(u, 0.0, eps, itmax=400000, tol=1e-11, check_every=50, x=x)
        assert r["res"] <= 1e-11
        Ws.append(r["W"])
    assert all(w >= W0 * (1 - 1e-12) for w in Ws)
    assert Ws[0] > Ws[1] > Ws[2]
    assert (Ws[2] - W0) / W0 < 2e-3
