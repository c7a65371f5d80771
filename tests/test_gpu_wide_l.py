"""l = 7..10 through the C ABI against the oracle.  These run on the team-layout
kernels (subset states spread over the lanes of a team, positions walked in
order, forward checkpoints every few positions): k_wide_pass, k_wide_check_all,
k_wide_batch.

Shapes are chosen so that every pass crosses several checkpoint blocks and ends
in a ragged one (positions per block: 16, 8, 4, 2 for l = 7..10 in FP64).

Tolerances: FP64 1e-12 relative (products pointwise, potentials gauge-fixed,
objective); FP32 products: the measured error is printed and asserted below a
bar a few times above it; FP32 solves are certified by the oracle's FP64
marginal errors of the returned potentials.
"""
import numpy as np
import pytest

from gpu_util import FP32_TOL, log_rel_err, potentials_err, say, to_dev
from oracle import dense, fastcheck
from paper_2405_19246_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
WIDE = [(7, 1), (7, 5), (7, 70), (8, 3), (8, 65), (9, 40), (10, 3), (10, 37)]


def _mmot():
    from paper_2405_19246_amd import mmot
    return mmot


def _rand_potentials(l, N, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(l, N)) * scale
    if N > 2:
        a[0, 1] = -np.inf  # a zero scaling factor
        a[l - 1, N - 1] = -np.inf
    return a


@pytest.mark.parametrize("l,N", WIDE)
def test_product_fp64_wide_l_matches_oracle(l, N):
    mmot = _mmot()
    h, eps = inputs.grid_step(max(N, 2)), 0.05
    a = _rand_potentials(l, N, 10 * l + N)
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64)
    ta = to_dev(a)
    for j in range(l):
        say("product fp64 l=%d N=%d j=%d" % (l, N, j))
        got = plan.marginal_product(j, ta).cpu().numpy()
        ref = fastcheck.marginal_product_log(a, j, h, eps)
        assert log_rel_err(got, ref) < FP64_TOL, (l, N, j, log_rel_err(got, ref))


@pytest.mark.parametrize("l,N", [(5, 5), (6, 4), (7, 3), (8, 3), (9, 3), (10, 3)])
def test_product_fp64_matches_dense_definition_wide(l, N):
    # straight against the N^l definition (no checker in between)
    mmot = _mmot()
    h, eps = 0.13, 0.07
    a = _rand_potentials(l, N, 70 + l, scale=20.0)
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64)
    logK = dense.log_kernel(l, N, h, eps)
    ta = to_dev(a)
    for j in range(l):
        say("product fp64 vs dense l=%d N=%d j=%d" % (l, N, j))
        got = plan.marginal_product(j, ta).cpu().numpy()
        ref = dense.marginal_product_log(logK, a, j)
        assert log_rel_err(got, ref) < FP64_TOL, (l, N, j, log_rel_err(got, ref))


@pytest.mark.parametrize("l,N", [(7, 9), (8, 7)])
def test_product_fp64_wide_l_huge_potentials(l, N):
    # |a| of order C_max / eps and zero scaling factors: exact shifts keep it finite
    mmot = _mmot()
    h, eps = 0.2, 0.01
    rng = np.random.default_rng(9 + l)
    a = rng.normal(size=(l, N)) * 800.0
    a[1, 2] = -np.inf
    a[3, 0] = -np.inf
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64)
    ta = to_dev(a)
    for j in range(l):
        say("product fp64 huge l=%d N=%d j=%d" % (l, N, j))
        got = plan.marginal_product(j, ta).cpu().numpy()
        ref = fastcheck.marginal_product_log(a, j, h, eps)
        assert log_rel_err(got, ref, mag_ulps=16) < FP64_TOL, (l, N, j, log_rel_err(got, ref, mag_ulps=16))


@pytest.mark.parametrize("l,N", WIDE)
def test_product_fp32_wide_l_error_is_small(l, N):
    mmot = _mmot()
    h, eps = inputs.grid_step(max(N, 2)), 0.01
    a = _rand_potentials(l, N, 5 * l + N, scale=20.0)
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP32)
    worst = 0.0
    for j in range(l):
        say("product fp32 l=%d N=%d j=%d" % (l, N, j))
        got = plan.marginal_product(j, to_dev(a)).cpu().numpy()
        worst = max(worst, log_rel_err(got, fastcheck.marginal_product_log(a, j, h, eps)))
    print("fp32 product l=%d N=%d: max relative error %.3e" % (l, N, worst))
    assert worst < FP32_TOL


@pytest.mark.parametrize("l,N", [(7, 40), (8, 24), (9, 20), (10, 11)])
def test_solve_fp64_wide_l_fixed_sweeps_match_oracle(l, N):
    mmot = _mmot()
    u = inputs.marginals(l, N, K=3, master_seed=41, instance=N)
    h, eps = inputs.grid_step(N), 0.05
    say("solve fp64 l=%d N=%d, 20 sweeps" % (l, N))
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64, tol=-1.0, itr_max=20, check_every=0)
    log_phi, res = plan.solve(to_dev(np.log(u)))
    ref = fastcheck.sinkhorn(u, h, eps, itmax=20, check_every=20)
    assert res["iters"] == 20
    assert potentials_err(log_phi.cpu().numpy(), ref["log_phi"]) < FP64_TOL
    assert abs(res["W"] - ref["W"]) <= FP64_TOL * abs(ref["W"])
    assert abs(res["marg_err"] - ref["res"]) <= 1e-10 * max(ref["res"], 1e-300)


@pytest.mark.parametrize("l,N", [(7, 33), (9, 17)])
def test_objective_and_marginal_errors_wide_l(l, N):
    mmot = _mmot()
    h, eps = inputs.grid_step(N), 0.07
    a = _rand_potentials(l, N, 3 * l + N, scale=2.0)
    u = inputs.marginals(l, N, K=2, master_seed=5, instance=N)
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64)
    say("objective l=%d N=%d" % (l, N))
    W = plan.objective(to_dev(a))
    Wr = fastcheck.objective(a, h, eps)
    assert abs(W - Wr) <= FP64_TOL * abs(Wr), (W, Wr)
    say("marginal errors l=%d N=%d" % (l, N))
    err = plan.marginal_errors(to_dev(np.log(u)), to_dev(a))
    ref = fastcheck.marginal_errors(u, a, h, eps)
    np.testing.assert_allclose(err, ref, rtol=1e-10)


def test_batch_mixed_l_up_to_10_certified():
    # A small batch shaped like the mixed configuration (l from 3 to 10, uneven N
    # and eps), FP32 scans to Res <= 1e-6: every instance is certified by the
    # oracle's FP64 marginal errors of the returned potentials.
    mmot = _mmot()
    rng = np.random.default_rng(7)
    insts = []
    for s in range(24):
        l = 3 + s % 8
        N = int(rng.integers(16, 120)) if l <= 8 else int(rng.integers(8, 40))
        eps = float(rng.choice([0.1, 0.05]))
        u = inputs.marginals(l, N, K=3, master_seed=43, instance=s)
        insts.append(dict(l=l, N=N, h=inputs.grid_step(N), eps=eps, u=u, log_u=to_dev(np.log(u)),
                          log_phi=to_dev(np.zeros((l, N)))))
    say("mixed batch of %d, l = 3..10, fp32 to 1e-6" % len(insts))
    res = mmot.solve_batch(insts, precision=mmot.FP32, tol=1e-6, itr_max=20000, check_every=0)
    for d, r in zip(insts, res):
        assert r["status"] == 0, (d["l"], d["N"], d["eps"], r)
        err = fastcheck.marginal_errors(d["u"], d["log_phi"].cpu().numpy(), d["h"], d["eps"])
        assert err[:-1].sum() <= 1e-6, (d["l"], d["N"], err)
        ref = fastcheck.objective(d["log_phi"].cpu().numpy(), d["h"], d["eps"])
        assert abs(r["W"] - ref) <= 1e-10 * abs(ref), (d["l"], d["N"])
