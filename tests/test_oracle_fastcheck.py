"""Pin the O(N) C checker (oracle/fastcheck.c) to the dense oracle."""
import numpy as np
import pytest

from oracle import dense, fastcheck
from paper_2405_19246_amd import inputs


@pytest.mark.parametrize("l", [2, 3, 4, 5])
@pytest.mark.parametrize("N", [1, 2, 3, 6])
def test_product_and_objective_match_dense(l, N):
    rng = np.random.default_rng(100 * l + N)
    a = rng.normal(size=(l, N)) * 3.0
    h, eps = 0.21, 0.33
    logK = dense.log_kernel(l, N, h, eps)
    for j in range(l):
        np.testing.assert_allclose(fastcheck.marginal_product_log(a, j, h, eps),
                                   dense.marginal_product_log(logK, a, j), rtol=1e-13, atol=1e-13)
    W_d = dense.objective(l, N, h, eps, a)
    assert abs(fastcheck.objective(a, h, eps) - W_d) <= 1e-12 * max(abs(W_d), 1e-300)


def test_large_potentials_and_zero_entries():
    # |a| of order C_max / eps and u = 0 entries (a = -inf) stay finite / exact
    l, N = 4, 6
    rng = np.random.default_rng(9)
    a = rng.normal(size=(l, N)) * 800.0
    a[1, 2] = -np.inf
    a[3, 0] = -np.inf
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
