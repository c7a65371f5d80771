"""Pins of the dense oracle against facts it does not compute itself.

Each test fixes a part of oracle/dense.py that a plausible mistake would break:
explicit enumeration (a wrong axis or a dropped term), closed forms at
lambda = 1 and lambda = 0, the l = 2 Toeplitz matrix (a library routine), the
symmetries of the cost, the mass identity, the marginal constraints at
convergence, and the comonotone lower bound of the objective.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle import dense
from paper_2405_19246_amd import inputs


def _enumerate_product(a, j, h, eps):
    """J_j(y) by explicit loops over every index tuple (pure Python)."""
    l, N = a.shape
    lam = np.exp(-h / eps)
    out = np.zeros(N)
    for idx in itertools.product(range(N), repeat=l):
        E = sum(abs(idx[p] - idx[q]) for p in range(l) for q in range(p + 1, l))
        w = lam ** E
        for q in range(l):
            if q != j:
                w *= np.exp(a[q, idx[q]])
        out[idx[j]] += w
    return out


@pytest.mark.parametrize("l", [2, 3, 4, 5])
def test_cost_gap_and_rank_forms(l):
    # sum_{p<q}|i_p-i_q| = sum_r (2r-l-1) x_(r) = sum_x m_x (l - m_x)
    N = 4
    E = dense.cost_exponent(l, N)
    for idx in itertools.product(range(N), repeat=l):
        xs = sorted(idx)
        rank = sum((2 * (r + 1) - l - 1) * xs[r] for r in range(l))
        gap = sum(m * (l - m) for m in (sum(1 for i in idx if i <= x) for x in range(N - 1)))
        assert E[idx] == rank == gap


@pytest.mark.parametrize("l,N", [(2, 4), (3, 3), (3, 4), (4, 3)])
def test_product_matches_enumeration(l, N):
    rng = np.random.default_rng(l * 10 + N)
    a = rng.normal(size=(l, N))
    h, eps = 0.3, 0.45
    logK = dense.log_kernel(l, N, h, eps)
    for j in range(l):
        got = np.exp(dense.marginal_product_log(logK, a, j))
        ref = _enumerate_product(a, j, h, eps)
        np.testing.assert_allclose(got, ref, rtol=1e-13)
        lin = dense.marginal_product_lin(np.exp(logK), np.exp(a), j)
        np.testing.assert_allclose(lin, ref, rtol=1e-13)


@pytest.mark.parametrize("l", [2, 3, 4])
def test_lambda_one_closed_form(l):
    # h = 0: K = 1 and J_j(y) = prod_{q != j} sum_x phi_q(x) for every y
    N = 5
    rng = np.random.default_rng(1)
    a = rng.normal(size=(l, N))
    logK = dense.log_kernel(l, N, 0.0, 1.0)
    for j in range(l):
        got = np.exp(dense.marginal_product_log(logK, a, j))
        ref = np.prod([np.exp(a[q]).sum() for q in range(l) if q != j])
        np.testing.assert_allclose(got, np.full(N, ref), rtol=1e-13)


@pytest.mark.parametrize("l", [2, 3, 4])
def test_lambda_zero_closed_form(l):
    # lambda -> 0: only the diagonal i_1 = .. = i_l survives, J_j(y) = prod phi_q(y)
    N = 5
    rng = np.random.default_rng(2)
    a = rng.normal(size=(l, N))
    logK = np.where(dense.cost_exponent(l, N) == 0, 0.0, -np.inf)
    for j in range(l):
        got = dense.marginal_product_log(logK, a, j)
        ref = sum(a[q] for q in range(l) if q != j)
        np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_two_marginals_is_toeplitz_matvec():
    N = 7
    h, eps = 0.2, 0.3
    lam = np.exp(-h / eps)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(2, N))
    T = scipy.linalg.toeplitz(lam ** np.arange(N))
    logK = dense.log_kernel(2, N, h, eps)
    np.testing.assert_allclose(np.exp(dense.marginal_product_log(logK, a, 0)), T @ np.exp(a[1]), rtol=1e-13)
    np.testing.assert_allclose(np.exp(dense.marginal_product_log(logK, a, 1)), T @ np.exp(a[0]), rtol=1e-13)


def test_permutation_and_reflection_symmetry():
    l, N = 4, 5
    rng = np.random.default_rng(4)
    a = rng.normal(size=(l, N))
    logK = dense.log_kernel(l, N, 0.25, 0.4)
    j = 1
    base = dense.marginal_product_log(logK, a, j)
    others = [q for q in range(l) if q != j]
    for perm in itertools.permutations(others):
        b = a.copy()
        for q, p in zip(others, perm):
            b[q] = a[p]
        np.testing.assert_allclose(dense.marginal_product_log(logK, b, j), base, rtol=1e-13)
    np.testing.assert_allclose(dense.marginal_product_log(logK, a[:, ::-1], j), base[::-1], rtol=1e-13)


def test_mass_identity():
    # <phi_j, J_j> is the total mass of the plan, the same for every j
    l, N = 4, 6
    rng = np.random.default_rng(5)
    a = rng.normal(size=(l, N))
    logK = dense.log_kernel(l, N, 0.15, 0.2)
    Z = [np.sum(np.exp(a[j] + dense.marginal_product_log(logK, a, j))) for j in range(l)]
    np.testing.assert_allclose(Z, np.full(l, Z[0]), rtol=1e-13)


def test_sinkhorn_meets_marginals():
    u = inputs.marginals(3, 20, K=2, master_seed=7)
    h = inputs.grid_step(20)
    r = dense.sinkhorn(u, h, 0.1, itmax=2000, tol=1e-13)
    assert r["res"] <= 1e-13
    logK = dense.log_kernel(3, 20, h, 0.1)
    np.testing.assert_allclose(dense.plan_marginals(logK, r["log_phi"]), u, atol=1e-13)


def test_gauge_invariance_of_plan():
    # shifting the potentials by constants c_q with sum c_q = 0 leaves the plan
    # unchanged, so every later iterate gives the same plan and objective
    u = inputs.marginals(3, 12, K=2, master_seed=8)
    h = inputs.grid_step(12)
    a0 = np.full((3, 12), -np.log(12))
    r1 = dense.sinkhorn(u, h, 0.2, itmax=30, log_phi0=a0)
    r2 = dense.sinkhorn(u, h, 0.2, itmax=30, log_phi0=a0 + np.array([[1.5], [-0.5], [-1.0]]))
    logK = dense.log_kernel(3, 12, h, 0.2)
    np.testing.assert_allclose(dense.log_plan(logK, r1["log_phi"]), dense.log_plan(logK, r2["log_phi"]), atol=1e-12)
    assert abs(r1["W"] - r2["W"]) <= 1e-13


def _comonotone_cost(u):
    """W0 = sum_{p<q} int_0^1 |F_p^-1(s) - F_q^-1(s)| ds on the grid x_i = i h."""
    l, N = u.shape
    h = inputs.grid_step(N)
    cdf = np.cumsum(u, axis=1)
    cdf[:, -1] = 1.0
    br = np.unique(np.concatenate([[0.0], cdf.ravel()]))
    br = br[(br >= 0.0) & (br <= 1.0)]
    W0 = 0.0
    for s0, s1 in zip(br[:-1], br[1:]):
        s = 0.5 * (s0 + s1)
        xs = [h * int(np.searchsorted(cdf[p], s)) for p in range(l)]
        W0 += (s1 - s0) * sum(abs(xs[p] - xs[q]) for p in range(l) for q in range(p + 1, l))
    return W0


def test_objective_above_comonotone_bound_and_monotone_in_eps():
    # For a pairwise convex cost on the line the comonotone (quantile) coupling
    # is optimal, so W_eps >= W0; W_eps decreases to W0 as eps decreases.
    u = inputs.marginals(3, 24, K=2, master_seed=0)
    h = inputs.grid_step(24)
    W0 = _comonotone_cost(u)
    Ws = []
    for eps in (0.2, 0.1, 0.05, 0.02):
        r = dense.sinkhorn(u, h, eps, itmax=5000, tol=1e-12)
        Ws.append(r["W"])
    assert all(w >= W0 - 1e-12 for w in Ws)
    assert all(Ws[i] > Ws[i + 1] for i in range(len(Ws) - 1))
    assert Ws[-1] - W0 < 0.25 * (Ws[0] - W0)


def test_linear_domain_breaks_where_log_domain_does_not():
    # The paper's unstabilised run stops on Ricker wavelets at N = 100,
    # eps = 1e-3 (Sec. 5.2, at its 89th iteration; the exact count depends on the
    # overflow test and is not pinned); the log-domain iteration stays finite.
    N = 100
    u = inputs.ricker_marginals(N)
    _, h = inputs.ricker_grid(N)
    lin = dense.sinkhorn_linear(u, h, 1e-3, itmax=200)
    assert lin["failed_at"] is not None
    r = dense.sinkhorn(u, h, 1e-3, itmax=lin["failed_at"] + 5, check_every=1000)
    assert np.all(np.isfinite(r["log_phi"])) and np.isfinite(r["res"])


def test_jacobi_ascends_the_dual_and_reaches_the_gauss_seidel_plan():
    # the damped all-marginals sweep is the mean of the l block updates, so the
    # concave dual never decreases; its limit is the unique entropic plan
    l, N, eps = 3, 7, 0.2
    u = inputs.marginals(l, N, K=2, master_seed=3, instance=1)
    h = inputs.grid_step(N)
    logK = dense.log_kernel(l, N, h, eps)
    vals = []
    for its in range(1, 30):
        r = dense.sinkhorn_jacobi(u, h, eps, itmax=its)
        vals.append(dense.dual_value(u, logK, r["log_phi"]))
    assert all(b >= a - 1e-15 for a, b in zip(vals, vals[1:]))
    gs = dense.sinkhorn(u, h, eps, itmax=5000, tol=1e-14)
    jc = dense.sinkhorn_jacobi(u, h, eps, itmax=20000, tol=1e-13)
    assert jc["res"] <= 1e-13
    Pg = np.exp(dense.log_plan(logK, gs["log_phi"]))
    Pj = np.exp(dense.log_plan(logK, jc["log_phi"]))
    assert np.abs(Pg - Pj).sum() < 1e-12
    assert abs(gs["W"] - jc["W"]) < 1e-12


def test_undamped_jacobi_is_not_a_fixed_point_iteration_that_settles():
    # without the 1/l damping the all-marginals update overshoots: at l = 3 the
    # plan's mass is multiplied by the product of the three corrections, so the
    # iterates cycle instead of settling (why the variant takes the mean)
    l, N, eps = 3, 6, 0.2
    u = inputs.marginals(l, N, K=2, master_seed=4, instance=0)
    h = inputs.grid_step(N)
    logK = dense.log_kernel(l, N, h, eps)
    a = np.full((l, N), -np.log(N))
    hist = []
    for _ in range(60):
        J = np.stack([dense.marginal_product_log(logK, a, j) for j in range(l)])
        a = np.log(u) - J
        hist.append(dense.residual(logK, a, u))
    assert min(hist[-10:]) > 1e-3
