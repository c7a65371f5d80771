"""Pins of the 2-D (three marginals, separable L1 cost) oracle, oracle/twod.py.

* the dense log-kernel equals the cost written from point coordinates;
* one point along an axis reduces the problem to the 1-D one along the other;
* the reduction to 1-D products (Sec. 4.1) equals the dense definition for
  products, objective and Gauss-Seidel sweeps, with zero scaling factors;
* Table 3's comparison (U[0,1] marginals, eps = 0.1, 100 sweeps): the plan of the
  reduced iteration and the dense one agree to rounding.
"""
import itertools

import numpy as np
import pytest

from oracle import dense, twod


def test_dense_kernel_is_the_coordinate_cost():
    N, M, h1, h2, eps = 3, 2, 0.3, 0.7, 0.5
    L = twod.dense2d_log_kernel(N, M, h1, h2, eps)
    pts = [(i2, i1) for i2 in range(M) for i1 in range(N)]
    for pa, pb, pc in itertools.product(pts, repeat=3):
        P = [pa, pb, pc]
        c = 0.0
        for s in range(3):
            for t in range(s + 1, 3):
                c += abs(P[s][1] - P[t][1]) * h1 + abs(P[s][0] - P[t][0]) * h2
        assert abs(L[pa[0], pa[1], pb[0], pb[1], pc[0], pc[1]] + c / eps) < 1e-13


def test_one_point_along_an_axis_is_the_1d_problem():
    rng = np.random.default_rng(0)
    eps = 0.2
    a = rng.normal(size=(3, 1, 7))          # M = 1: the first axis alone, step h1
    L2 = twod.dense2d_log_kernel(7, 1, 0.1, 0.9, eps)
    L1 = dense.log_kernel(3, 7, 0.1, eps)
    for j in range(3):
        np.testing.assert_allclose(twod.dense2d_product(L2, a, j)[0], dense.marginal_product_log(L1, a[:, 0, :], j),
                                   rtol=1e-13)
    b = rng.normal(size=(3, 6, 1))          # N = 1: the second axis alone, step h2
    L2 = twod.dense2d_log_kernel(1, 6, 0.1, 0.9, eps)
    L1 = dense.log_kernel(3, 6, 0.9, eps)
    for j in range(3):
        np.testing.assert_allclose(twod.dense2d_product(L2, b, j)[:, 0], dense.marginal_product_log(L1, b[:, :, 0], j),
                                   rtol=1e-13)


@pytest.mark.parametrize("N,M", [(4, 3), (3, 4), (5, 2), (2, 5)])
def test_reduction_matches_dense(N, M):
    rng = np.random.default_rng(N * 10 + M)
    h1, h2, eps = 0.25, 0.4, 0.15
    a = rng.normal(size=(3, M, N)) * 2.0
    a[0, 1, 1] = -np.inf
    a[2, M - 1, 0] = -np.inf
    L = twod.dense2d_log_kernel(N, M, h1, h2, eps)
    for j in range(3):
        ref = twod.dense2d_product(L, a, j)
        got = twod.product(a, j, h1, h2, eps)
        fin = np.isfinite(ref)
        assert np.array_equal(fin, np.isfinite(got))
        np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-12, atol=1e-12)
    T = np.exp(twod._log_plan(L, a))
    W = float(np.sum(twod.dense2d_cost(N, M, h1, h2) * T))
    assert abs(twod.objective(a, h1, h2, eps) - W) <= 1e-12 * abs(W)


def test_reduced_sweeps_match_dense_and_table3_plans_agree():
    # Sec. 5.3: U[0,1] entries, eps = 0.1, here N = M = 4 and 100 sweeps
    N = M = 4
    rng = np.random.default_rng(5)
    u = rng.uniform(0.0, 1.0, size=(3, M, N))
    u /= u.reshape(3, -1).sum(axis=1)[:, None, None]
    h1 = h2 = 1.0 / (N - 1)
    rd = twod.dense2d_sinkhorn(u, h1, h2, 0.1, itmax=100)
    rr = twod.sinkhorn(u, h1, h2, 0.1, itmax=100)
    L = twod.dense2d_log_kernel(N, M, h1, h2, 0.1)
    P = np.exp(twod._log_plan(L, rr["log_phi"]))
    assert np.linalg.norm((P - rd["plan"]).ravel()) < 1e-14
    assert abs(rr["W"] - rd["W"]) <= 1e-12 * rd["W"]
    assert abs(rr["res"] - rd["res"]) <= 1e-8 * max(rd["res"], 1e-300)
