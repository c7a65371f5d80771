"""Three marginals on a 2-D grid (separable L1 cost, Sec. 4.1) through the C ABI
against the oracle (oracle/twod.py: the dense (NM)^3 definition at small sizes,
the reduction to 1-D products over second-axis triples beyond).  FP64 only;
tolerances 1e-12 relative (products pointwise, objective, potentials).
"""
import numpy as np
import pytest

from gpu_util import log_rel_err, potentials_err, say, to_dev
from oracle import twod
from paper_2405_19246_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _mmot():
    from paper_2405_19246_amd import mmot
    return mmot


def _pots(N, M, seed, scale=2.0):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(3, M, N)) * scale
    a[0, 0, min(1, N - 1)] = -np.inf
    a[2, M - 1, N - 1] = -np.inf
    return a


@pytest.mark.parametrize("N,M", [(4, 3), (5, 5), (3, 6), (1, 5), (6, 1)])
def test_product_matches_dense_definition(N, M):
    mmot = _mmot()
    h1, h2, eps = 0.3, 0.2, 0.15
    a = _pots(N, M, N * 7 + M)
    L = twod.dense2d_log_kernel(N, M, h1, h2, eps)
    plan = mmot.Plan2D(N, M, h1, h2, eps)
    for j in range(3):
        say("2-D product vs dense N=%d M=%d j=%d" % (N, M, j))
        got = plan.marginal_product(j, to_dev(a)).cpu().numpy()
        assert log_rel_err(got, twod.dense2d_product(L, a, j)) < TOL
    W = plan.objective(to_dev(a))
    T = np.exp(twod._log_plan(L, a))
    Wd = float(np.sum(twod.dense2d_cost(N, M, h1, h2) * T))
    assert abs(W - Wd) <= TOL * abs(Wd), (W, Wd)


@pytest.mark.parametrize("N,M", [(300, 6), (40, 12), (7, 30)])
def test_product_and_objective_match_reduction(N, M):
    mmot = _mmot()
    h1, h2, eps = 1.0 / N, 1.0 / M, 0.05
    a = _pots(N, M, N + M, scale=3.0)
    plan = mmot.Plan2D(N, M, h1, h2, eps)
    for j in range(3):
        say("2-D product vs reduction N=%d M=%d j=%d" % (N, M, j))
        got = plan.marginal_product(j, to_dev(a)).cpu().numpy()
        assert log_rel_err(got, twod.product(a, j, h1, h2, eps)) < TOL
    say("2-D objective N=%d M=%d" % (N, M))
    W = plan.objective(to_dev(a))
    Wr = twod.objective(a, h1, h2, eps)
    assert abs(W - Wr) <= TOL * abs(Wr), (W, Wr)


def test_table3_plans_match_dense():
    # Sec. 5.3: U[0,1] entries, eps = 0.1, 100 sweeps; N = M = 4 here (dense (NM)^3)
    mmot = _mmot()
    N = M = 4
    u = inputs.random_2d_marginals(N, M, seed=3)
    h = 1.0 / (N - 1)
    say("2-D 100 sweeps N=M=4 vs dense")
    plan = mmot.Plan2D(N, M, h, h, 0.1, tol=-1.0, itr_max=100)
    lp, res = plan.solve(to_dev(np.log(u)))
    rd = twod.dense2d_sinkhorn(u, h, h, 0.1, itmax=100)
    L = twod.dense2d_log_kernel(N, M, h, h, 0.1)
    P = np.exp(twod._log_plan(L, lp.cpu().numpy()))
    d = float(np.linalg.norm((P - rd["plan"]).ravel()))
    print("||P_gpu - P_dense||_F = %.3e" % d)
    assert res["iters"] == 100 and d < 1e-14
    assert abs(res["W"] - rd["W"]) <= TOL * rd["W"]
    assert abs(res["marg_err"] - rd["res"]) <= 1e-9 * max(rd["res"], 1e-300)


def test_fixed_sweeps_match_reduction():
    mmot = _mmot()
    N, M, eps, its = 12, 10, 0.05, 8
    u = inputs.random_2d_marginals(N, M, seed=4)
    say("2-D %d sweeps N=%d M=%d vs reduction" % (its, N, M))
    plan = mmot.Plan2D(N, M, 1.0 / (N - 1), 1.0 / (M - 1), eps, tol=-1.0, itr_max=its)
    lp, res = plan.solve(to_dev(np.log(u)))
    ref = twod.sinkhorn(u, 1.0 / (N - 1), 1.0 / (M - 1), eps, itmax=its)
    assert potentials_err(lp.cpu().numpy().reshape(3, -1), ref["log_phi"].reshape(3, -1)) < TOL
    assert abs(res["W"] - ref["W"]) <= TOL * ref["W"]
    assert abs(res["marg_err"] - ref["res"]) <= 1e-9 * ref["res"]


def test_solve_to_tolerance_certified():
    mmot = _mmot()
    N = M = 20
    u = inputs.random_2d_marginals(N, M, seed=5)
    h = 1.0 / (N - 1)
    say("2-D solve N=M=20 eps=0.1 to 1e-9")
    plan = mmot.Plan2D(N, M, h, h, 0.1, tol=1e-9, itr_max=20000, check_every=10)
    lp, res = plan.solve(to_dev(np.log(u)))
    a = lp.cpu().numpy()
    err = twod.marginal_errors(u, a, h, h, 0.1)
    print("2-D N=M=20: %d sweeps, Res %.3e, certified %.3e, W %.12f" % (res["iters"], res["marg_err"], err[:2].sum(),
                                                                       res["W"]))
    assert res["status"] == 0 and err[:2].sum() <= 1e-9
    np.testing.assert_allclose(plan.marginal_errors(to_dev(np.log(u)), lp), err, rtol=1e-9, atol=1e-15)
