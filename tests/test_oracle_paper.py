"""Pins of the paper's own l = 3 recurrences (oracle/paper_ftvp.py)."""
import itertools

import numpy as np
import pytest

from oracle import dense, paper_ftvp
from paper_2405_19246_amd import inputs


def _brute(phi, psi, lam, h):
    N = phi.shape[0]
    J = np.zeros(N)
    Jh = np.zeros(N)
    for i, j, k in itertools.product(range(N), repeat=3):
        E = abs(i - j) + abs(i - k) + abs(j - k)
        J[k] += phi[i] * psi[j] * lam ** E
        Jh[k] += h * E * phi[i] * psi[j] * lam ** E
    return J, Jh


def test_ordering_sets_partition_and_exponents():
    # D_1..D_6 (Sec. 3, Eq. D_p) partition [N]^3 and on D_p the exponent of
    # lambda is a_p i + b_p j + c_p k (Eq. a_p b_p c_p)
    N = 5
    rng1 = range(1, N + 1)
    sets = {
        1: lambda i, j, k: i <= j <= k, 2: lambda i, j, k: j < i <= k,
        3: lambda i, j, k: i <= k < j, 4: lambda i, j, k: j <= k < i,
        5: lambda i, j, k: k < i <= j, 6: lambda i, j, k: k < j < i,
    }
    for i, j, k in itertools.product(rng1, repeat=3):
        member = [p for p in sets if sets[p](i, j, k)]
        assert len(member) == 1
        p = member[0]
        assert abs(i - j) + abs(i - k) + abs(j - k) == paper_ftvp.A[p] * i + paper_ftvp.B[p] * j + paper_ftvp.C[p] * k


@pytest.mark.parametrize("N", [1, 2, 3, 4, 7, 9])
@pytest.mark.parametrize("lam", [0.0, 0.35, 0.9, 1.0])
def test_ftvp1_and_ftvp2_match_brute_force(N, lam):
    rng = np.random.default_rng(N)
    phi = rng.uniform(0.1, 1.0, N)
    psi = rng.uniform(0.1, 1.0, N)
    h = 0.25
    J, Jh = _brute(phi, psi, lam, h)
    np.testing.assert_allclose(paper_ftvp.ftvp1(phi, psi, lam), J, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(paper_ftvp.ftvp2(phi, psi, lam, h), Jh, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("N", [2, 3, 6])
def test_printed_ftvp2_initial_values_are_wrong(N):
    # the printed R_{N,5}, R_{N,6} (without the factor N) disagree with brute force
    rng = np.random.default_rng(10 + N)
    phi = rng.uniform(0.1, 1.0, N)
    psi = rng.uniform(0.1, 1.0, N)
    _, Jh = _brute(phi, psi, 0.6, 0.3)
    bad = paper_ftvp.ftvp2_printed_init(phi, psi, 0.6, 0.3)
    assert np.max(np.abs(bad - Jh) / Jh.max()) > 1e-2


def test_ftvp1_equals_dense_product():
    N = 11
    rng = np.random.default_rng(3)
    a = rng.normal(size=(3, N))
    h, eps = inputs.grid_step(N), 0.1
    lam = np.exp(-h / eps)
    logK = dense.log_kernel(3, N, h, eps)
    np.testing.assert_allclose(paper_ftvp.ftvp1(np.exp(a[0]), np.exp(a[1]), lam),
                               np.exp(dense.marginal_product_log(logK, a, 2)), rtol=1e-13)


@pytest.mark.parametrize("N", [10, 20])
def test_fast_and_dense_plans_agree_like_the_paper(N):
    # Table 1 (Sec. 5.1) prints ||P_O - P_S||_F between 3.6e-17 and 1.1e-16 after
    # 100 iterations at eps = 0.1 on U[0,1] marginals; the two iterations are the
    # same arithmetic up to rounding, so their plans agree to ~1e-15 here too.
    u = inputs.uniform_random_marginals(3, N, seed=N)
    h, eps = inputs.grid_step(N), 0.1
    lam = np.exp(-h / eps)
    phi, psi, vphi, W_fast = paper_ftvp.fs3_sinkhorn(u[0], u[1], u[2], lam, h, 100)
    r = dense.sinkhorn(u, h, eps, itmax=100)
    logK = dense.log_kernel(3, N, h, eps)
    P_S = np.exp(dense.log_plan(logK, r["log_phi"]))
    P_O = np.exp(logK) * phi[:, None, None] * psi[None, :, None] * vphi[None, None, :]
    assert np.linalg.norm((P_O - P_S).ravel()) < 1e-14
    # one factor h in the objective: <varphi, FTVP-2(phi, psi)> is <C, T>
    assert abs(W_fast - r["W"]) < 1e-13


def test_ricker_inputs_follow_sec_5_2():
    # R(0) = A; R vanishes at t = +-1 / (sqrt(2) pi F0); each marginal sums to 1,
    # sits at or above its floor delta / (1 + N delta) and peaks at the grid
    # point nearest its shift tau once the grid resolves the main lobe (|R| is 1
    # there, 2 e^{-3/2} on the side lobes)
    assert inputs.ricker(np.array([0.0]))[0] == 1.0
    r0 = 1.0 / (np.sqrt(2.0) * np.pi)
    assert np.all(np.abs(inputs.ricker(np.array([-r0, r0]))) < 1e-15)
    assert abs(inputs.ricker(np.array([np.sqrt(1.5) / np.pi]))[0] + 2 * np.exp(-1.5)) < 1e-15
    for N in (97, 161, 401):
        t, h = inputs.ricker_grid(N)
        assert t[0] == -2.0 and t[-1] == 2.0 and abs(h - (t[1] - t[0])) < 1e-15
        u = inputs.ricker_marginals(N)
        assert u.shape == (3, N)
        np.testing.assert_allclose(u.sum(axis=1), 1.0, rtol=1e-14)
        assert np.all(u >= 1e-3 / (1 + N * 1e-3) * (1 - 1e-14))
        for q, tau in enumerate((0.0, 0.75, 1.5)):
            assert abs(t[np.argmax(u[q])] - tau) < 1e-12
