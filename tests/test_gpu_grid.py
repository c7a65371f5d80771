"""Non-uniform grids and unequal supports through the C ABI against the oracle.

A problem on coordinates x (mmot_problem.x / mmot_instance.x) runs on the tiled
kernels at every N, with the gap factors exp(-(x_{k+1} - x_k) m (l - m) / eps)
staged per position.  References: the C checker on the same coordinates
(pinned to the dense coordinate cost at l = 2..8) and, at small sizes, the dense
oracle itself.

Tolerances: FP64 1e-12 relative (products pointwise, potentials gauge-fixed,
objective); FP32 products: measured error printed, asserted below FP32_TOL (4e-6); FP32
solves certified by the oracle's FP64 marginal errors.
"""
import numpy as np
import pytest

from gpu_util import FP32_TOL, log_rel_err, potentials_err, say, to_dev
from oracle import dense, fastcheck
from paper_2405_19246_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
SHAPES = [(2, 50), (3, 70), (4, 130), (5, 100), (6, 64), (7, 70), (8, 40), (9, 30), (10, 19)]


def _mmot():
    from paper_2405_19246_amd import mmot
    return mmot


def _pots(l, N, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(l, N)) * scale
    if N > 2:
        a[0, 1] = -np.inf
        a[l - 1, N - 1] = -np.inf
    return a


@pytest.mark.parametrize("l,N", SHAPES)
def test_grid_product_fp64_matches_oracle(l, N):
    mmot = _mmot()
    x = inputs.graded_grid(N, seed=l)
    eps = 0.05
    a = _pots(l, N, 13 * l + N)
    plan = mmot.Plan(l, N, 0.0, eps, precision=mmot.FP64, x=x)
    ta = to_dev(a)
    for j in range(l):
        say("grid product fp64 l=%d N=%d j=%d" % (l, N, j))
        got = plan.marginal_product(j, ta).cpu().numpy()
        ref = fastcheck.marginal_product_log(a, j, 0.0, eps, x)
        assert log_rel_err(got, ref) < FP64_TOL, (l, N, j, log_rel_err(got, ref))


@pytest.mark.parametrize("l,N", [(3, 12), (5, 6)])
def test_grid_product_matches_dense_coordinate_cost(l, N):
    mmot = _mmot()
    x = inputs.graded_grid(N, seed=100 + l)
    x[3] = x[2]  # a repeated coordinate: a gap of length 0
    eps = 0.04
    a = _pots(l, N, 5 * l, scale=2.0)
    logK = dense.log_kernel(l, N, 0.0, eps, x)
    plan = mmot.Plan(l, N, 0.0, eps, precision=mmot.FP64, x=x)
    for j in range(l):
        say("grid product vs dense l=%d N=%d j=%d" % (l, N, j))
        got = plan.marginal_product(j, to_dev(a)).cpu().numpy()
        assert log_rel_err(got, dense.marginal_product_log(logK, a, j)) < FP64_TOL


@pytest.mark.parametrize("l,N", [(3, 70), (7, 70)])
def test_grid_product_fp32_error_is_small(l, N):
    mmot = _mmot()
    x = inputs.graded_grid(N, seed=2 * l)
    eps = 0.02
    a = _pots(l, N, 7 * l + N, scale=10.0)
    plan = mmot.Plan(l, N, 0.0, eps, precision=mmot.FP32, x=x)
    worst = 0.0
    for j in range(l):
        say("grid product fp32 l=%d N=%d j=%d" % (l, N, j))
        got = plan.marginal_product(j, to_dev(a)).cpu().numpy()
        worst = max(worst, log_rel_err(got, fastcheck.marginal_product_log(a, j, 0.0, eps, x)))
    print("grid fp32 product l=%d N=%d: max relative error %.3e" % (l, N, worst))
    assert worst < FP32_TOL


@pytest.mark.parametrize("l,N", [(3, 80), (4, 50), (6, 40), (8, 30), (10, 19)])
def test_grid_solve_fp64_fixed_sweeps_match_oracle(l, N):
    mmot = _mmot()
    x = inputs.graded_grid(N, seed=3 * l)
    u = inputs.grid_marginals(x, l, K=3, master_seed=41, instance=N)
    eps = 0.05
    say("grid solve fp64 l=%d N=%d, 15 sweeps" % (l, N))
    plan = mmot.Plan(l, N, 0.0, eps, precision=mmot.FP64, tol=-1.0, itr_max=15, check_every=0, x=x)
    log_phi, res = plan.solve(to_dev(np.log(u)))
    ref = fastcheck.sinkhorn(u, 0.0, eps, itmax=15, check_every=15, x=x)
    assert res["iters"] == 15
    assert potentials_err(log_phi.cpu().numpy(), ref["log_phi"]) < FP64_TOL
    assert abs(res["W"] - ref["W"]) <= FP64_TOL * abs(ref["W"])
    assert abs(res["marg_err"] - ref["res"]) <= 1e-10 * ref["res"]


@pytest.mark.parametrize("l,N", [(4, 45), (9, 21)])
def test_grid_objective_and_marginal_errors(l, N):
    mmot = _mmot()
    x = inputs.graded_grid(N, seed=l + N)
    eps = 0.07
    a = _pots(l, N, 3 * l + N, scale=2.0)
    u = inputs.grid_marginals(x, l, K=2, master_seed=5, instance=N)
    plan = mmot.Plan(l, N, 0.0, eps, precision=mmot.FP64, x=x)
    say("grid objective l=%d N=%d" % (l, N))
    W = plan.objective(to_dev(a))
    Wr = fastcheck.objective(a, 0.0, eps, x)
    assert abs(W - Wr) <= FP64_TOL * abs(Wr), (W, Wr)
    say("grid marginal errors l=%d N=%d" % (l, N))
    err = plan.marginal_errors(to_dev(np.log(u)), to_dev(a))
    np.testing.assert_allclose(err, fastcheck.marginal_errors(u, a, 0.0, eps, x), rtol=1e-10)


def test_grid_long_product_eps_1e3():
    mmot = _mmot()
    l, N, eps = 4, 65536, 1e-3
    x = inputs.graded_grid(N, seed=9)
    u = inputs.grid_marginals(x, l, K=3, master_seed=3, instance=0)
    a = np.log(u) + np.random.default_rng(4).normal(size=(l, N)) * 2.0
    plan = mmot.Plan(l, N, 0.0, eps, precision=mmot.FP64, x=x)
    for j in (0, l - 1):
        say("grid long product l=4 N=65536 j=%d" % j)
        got = plan.marginal_product(j, to_dev(a)).cpu().numpy()
        ref = fastcheck.marginal_product_log(a, j, 0.0, eps, x)
        assert log_rel_err(got, ref) < FP64_TOL, log_rel_err(got, ref)


def test_unequal_supports_solve_certified():
    # three marginals on their own supports, merged onto one grid; off-support
    # points get zero mass and -inf potentials
    mmot = _mmot()
    rng = np.random.default_rng(21)
    supports = [np.sort(rng.uniform(0, 1, n)) for n in (300, 450, 200)]
    weights = [np.exp(-((s - c) / 0.15) ** 2) + 1e-3 for s, c in zip(supports, (0.3, 0.5, 0.7))]
    x, u = inputs.merge_supports(supports, weights)
    l, N = u.shape
    eps = 0.02
    with np.errstate(divide="ignore"):
        lu = np.log(u)
    plan = mmot.Plan(l, N, 0.0, eps, precision=mmot.FP64, tol=1e-9, itr_max=20000, check_every=0, x=x)
    say("unequal supports solve l=3 N=%d" % N)
    log_phi, res = plan.solve(to_dev(lu))
    a = log_phi.cpu().numpy()
    print("unequal supports: N=%d sweeps=%d Res=%.3e W=%.12f" % (N, res["iters"], res["marg_err"], res["W"]))
    assert res["status"] == 0
    assert np.all(np.isneginf(a[u == 0.0])) and np.all(np.isfinite(a[u > 0.0]))
    err = fastcheck.marginal_errors(u, a, 0.0, eps, x)
    assert err[:-1].sum() <= 1e-9
    assert abs(res["W"] - fastcheck.objective(a, 0.0, eps, x)) <= 1e-12 * res["W"]


def test_batch_mixes_grids_and_uniform_fp32_certified():
    mmot = _mmot()
    import torch
    cases = [(3, 500, 0.05, True), (4, 300, 0.1, False), (7, 200, 0.1, True), (5, 20000, 0.05, True),
             (3, 800, 0.02, False)]
    insts = []
    for s, (l, N, eps, grid) in enumerate(cases):
        x = inputs.graded_grid(N, seed=s) if grid else None
        u = inputs.grid_marginals(x, l, K=3, master_seed=8, instance=s) if grid else \
            inputs.marginals(l, N, K=3, master_seed=8, instance=s)
        d = dict(l=l, N=N, h=inputs.grid_step(N), eps=eps, u=u, xs=x, log_u=to_dev(np.log(u)),
                 log_phi=to_dev(np.zeros((l, N))))
        if grid:
            d["x"] = torch.tensor(x, dtype=torch.float64, device="cuda:0")
        insts.append(d)
    say("grid/uniform batch fp32 to 1e-6")
    res = mmot.solve_batch(insts, precision=mmot.FP32, tol=1e-6, itr_max=20000, check_every=0)
    for d, r in zip(insts, res):
        a = d["log_phi"].cpu().numpy()
        h = 0.0 if d["xs"] is not None else d["h"]
        err = fastcheck.marginal_errors(d["u"], a, h, d["eps"], d["xs"])
        print("l=%d N=%d grid=%s status=%d sweeps=%d Res=%.3e certified=%.3e" %
              (d["l"], d["N"], d["xs"] is not None, r["status"], r["iters"], r["marg_err"], err[:-1].sum()))
        assert r["status"] == 0
        assert err[:-1].sum() <= 1e-6
        W = fastcheck.objective(a, h, d["eps"], d["xs"])
        assert abs(r["W"] - W) <= 1e-10 * abs(W)


def test_batch_rejects_a_bad_grid():
    mmot = _mmot()
    import torch
    l, N = 3, 100
    x = inputs.graded_grid(N, seed=1)
    x[50] = x[49] - 1e-3  # decreasing
    u = inputs.grid_marginals(x, l)
    d = dict(l=l, N=N, h=0.0, eps=0.1, log_u=to_dev(np.log(u)), log_phi=to_dev(np.zeros((l, N))),
             x=torch.tensor(x, dtype=torch.float64, device="cuda:0"))
    say("batch with a decreasing grid")
    with pytest.raises(mmot.MmotError) as e:
        mmot.solve_batch([d], precision=mmot.FP64)
    assert e.value.code == mmot.ERR_INVALID
