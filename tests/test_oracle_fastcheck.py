"""Pin the O(N) C checker (oracle/fastcheck.c) to the dense oracle."""
import numpy as np
import pytest

from oracle import dense, fastcheck
from paper_2405_19246_amd import inputs


# every l the checker serves, with N small enough that the dense N^l tensor
# stays below ~7e4 entries (l = 6: N <= 6, l = 7, 8: N <= 4, l = 16: N = 2)
_LN = [(l, N) for l in (2, 3, 4, 5) for N in (1, 2, 3, 6, 11)] + \
      [(6, 1), (6, 2), (6, 4), (6, 6), (7, 2), (7, 3), (7, 4), (8, 2), (8, 3), (8, 4)] + \
      [(9, 3), (10, 3), (12, 2), (16, 2)]   # the wide l of the l = 10 and serving shapes


@pytest.mark.parametrize("l,N", _LN)
def test_product_and_objective_match_dense(l, N):
    rng = np.random.default_rng(100 * l + N)
    a = rng.normal(size=(l, N)) * 3.0
    h, eps = 0.21, 0.33
    logK = dense.log_kernel(l, N, h, eps)
    # the checker chains about l 2^(l-2) log-sum-exps per position, so its own
    # rounding grows with l: 1e-13 up to l = 8, 1e-11 beyond (l = 16: 2^14 steps)
    tol = 1e-13 if l <= 8 else 1e-11
    for j in range(l):
        np.testing.assert_allclose(fastcheck.marginal_product_log(a, j, h, eps),
                                   dense.marginal_product_log(logK, a, j), rtol=tol, atol=tol)
    W_d = dense.objective(l, N, h, eps, a)
    assert abs(fastcheck.objective(a, h, eps) - W_d) <= 100 * tol * max(abs(W_d), 1e-300)


@pytest.mark.parametrize("l,N", [(4, 6), (6, 4), (7, 3), (8, 3)])
def test_large_potentials_and_zero_entries(l, N):
    # |a| of order C_max / eps and u = 0 entries (a = -inf) stay finite / exact
    rng = np.random.default_rng(9 + l)
    a = rng.normal(size=(l, N)) * 800.0
    a[1, 2] = -np.inf
    a[3, 0] = -np.inf
    a[l - 1, N - 1] = -np.inf
    h, eps = 0.2, 0.01
    logK = dense.log_kernel(l, N, h, eps)
    for j in range(l):
        d = dense.marginal_product_log(logK, a, j)
        f = fastcheck.marginal_product_log(a, j, h, eps)
        np.testing.assert_allclose(f, d, rtol=1e-13)


def test_sinkhorn_matches_dense():
    u = inputs.marginals(4, 9, K=3, master_seed=1)
    h = inputs.grid_step(9)
    rd = dense.sinkhorn(u, h, 0.05, itmax=40)
    rf = fastcheck.sinkhorn(u, h, 0.05, itmax=40)
    np.testing.assert_allclose(rf["log_phi"], rd["log_phi"], rtol=1e-12, atol=1e-11)
    assert abs(rf["W"] - rd["W"]) < 1e-13
    assert abs(rf["res"] - rd["res"]) < 1e-13
    err = fastcheck.marginal_errors(u, rf["log_phi"], h, 0.05)
    logK = dense.log_kernel(4, 9, h, 0.05)
    err_d = np.abs(dense.plan_marginals(logK, rd["log_phi"]) - u).sum(axis=1)
    np.testing.assert_allclose(err, err_d, rtol=1e-6, atol=1e-15)


@pytest.mark.parametrize("l,N,eps,its", [(6, 5, 0.1, 12), (7, 3, 0.2, 8), (8, 3, 0.3, 6)])
def test_sinkhorn_matches_dense_wide(l, N, eps, its):
    # the checker's whole iteration (updates, residual, objective) at the l the
    # GPU tests use it for, against the dense definition
    u = inputs.marginals(l, N, K=2, master_seed=3)
    h = inputs.grid_step(N)
    rd = dense.sinkhorn(u, h, eps, itmax=its)
    rf = fastcheck.sinkhorn(u, h, eps, itmax=its)
    np.testing.assert_allclose(rf["log_phi"], rd["log_phi"], rtol=1e-12, atol=1e-11)
    assert abs(rf["W"] - rd["W"]) <= 1e-12 * abs(rd["W"])
    assert abs(rf["res"] - rd["res"]) <= 1e-12 + 1e-10 * abs(rd["res"])
    logK = dense.log_kernel(l, N, h, eps)
    err_d = np.abs(dense.plan_marginals(logK, rd["log_phi"]) - u).sum(axis=1)
    err = fastcheck.marginal_errors(u, rf["log_phi"], h, eps)
    np.testing.assert_allclose(err, err_d, rtol=1e-8, atol=1e-15)


@pytest.mark.parametrize("l,N,its", [(3, 8, 12), (5, 5, 7)])
def test_jacobi_matches_dense(l, N, its):
    u = inputs.marginals(l, N, K=2, master_seed=l, instance=N)
    u[1, 2] = 0.0
    u /= u.sum(axis=1, keepdims=True)
    h, eps = inputs.grid_step(N), 0.1
    rd = dense.sinkhorn_jacobi(u, h, eps, itmax=its)
    rf = fastcheck.sinkhorn_jacobi(u, h, eps, itmax=its, check_every=its)
    fin = np.isfinite(rd["log_phi"])
    assert np.array_equal(fin, np.isfinite(rf["log_phi"]))
    np.testing.assert_allclose(rf["log_phi"][fin], rd["log_phi"][fin], rtol=1e-12, atol=1e-12)
    assert abs(rf["W"] - rd["W"]) <= 1e-12 * abs(rd["W"])
    assert abs(rf["res"] - rd["res"]) <= 1e-10 * rd["res"]
