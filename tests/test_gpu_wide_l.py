"""l = 7 and 8 (the batch configuration's widest instances) through the C ABI,
against the oracle.  These run on the extended-range solver only, one
wavefront per instance (k_solve_batch_l, k_pass, k_check_all).

Tolerances as in test_gpu_parity: FP64 1e-12 relative; FP32 products 2e-5;
FP32 solves certified by the oracle's FP64 marginal errors.
"""
import numpy as np
import pytest

from gpu_util import log_rel_err, potentials_err, say, to_dev
from oracle import fastcheck
from paper_2405_19246_amd import inputs

# Switched off: in the first GPU run of an l = 7 build, the FP64 product at
# l = 7, N = 5 (one chunk) passed and the one at N = 70 (two chunks, the
# forward-checkpoint path) left the GPU faulted.  The same case emulated on the
# CPU, with AddressSanitizer, is clean and matches the oracle to 2e-14, and no
# cause has been found in the code, so l > 6 returns MMOT_ERR_UNSUPPORTED again
# and these tests stay skipped until a cause is shown.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="l = 7, 8 switched off: GPU fault at l=7 N=70 (two chunks), cause not found")]

FP64_TOL = 1e-12
WIDE = [(7, 5), (7, 70), (8, 3), (8, 65)]


def _mmot():
    from paper_2405_19246_amd import mmot
    return mmot


def _rand_potentials(l, N, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(l, N)) * scale
    if N > 2:
        a[0, 1] = -np.inf  # a zero scaling factor
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
    assert worst < 2e-5


@pytest.mark.parametrize("l,N", [(7, 40), (8, 24)])
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


def test_batch_mixed_l_up_to_8_certified():
    # A small batch shaped like the mixed configuration (l from 3 to 8, uneven N
    # and eps), FP32 scans to Res <= 1e-6: every instance is certified by the
    # oracle's FP64 marginal errors of the returned potentials.
    mmot = _mmot()
    rng = np.random.default_rng(7)
    insts = []
    for s in range(18):
        l = 3 + s % 6
        N = int(rng.integers(16, 120))
        eps = float(rng.choice([0.1, 0.05]))
        u = inputs.marginals(l, N, K=3, master_seed=43, instance=s)
        insts.append(dict(l=l, N=N, h=inputs.grid_step(N), eps=eps, u=u, log_u=to_dev(np.log(u)),
                          log_phi=to_dev(np.zeros((l, N)))))
    say("mixed batch of %d, l = 3..8, fp32 to 1e-6" % len(insts))
    res = mmot.solve_batch(insts, precision=mmot.FP32, tol=1e-6, itr_max=20000, check_every=0)
    for d, r in zip(insts, res):
        assert r["status"] == 0, (d["l"], d["N"], d["eps"], r)
        err = fastcheck.marginal_errors(d["u"], d["log_phi"].cpu().numpy(), d["h"], d["eps"])
        assert err[:-1].sum() <= 1e-6, (d["l"], d["N"], err)
        ref = fastcheck.objective(d["log_phi"].cpu().numpy(), d["h"], d["eps"])
        assert abs(r["W"] - ref) <= 1e-10 * abs(ref), (d["l"], d["N"])
