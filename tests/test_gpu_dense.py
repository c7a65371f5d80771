"""The dense (O(N^l)) product and sweeps on the device, the comparison point of the
scans (mmot_dense_marginal_product, mmot_dense_sinkhorn_iter), against the
oracle's dense definition and against the O(N) path.

Tolerance: FP64, 1e-12 relative (products pointwise, potentials gauge-fixed).
"""
import numpy as np
import pytest

from gpu_util import log_rel_err, potentials_err, say, to_dev
from oracle import dense, fastcheck
from paper_2405_19246_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def _mmot():
    from paper_2405_19246_amd import mmot
    return mmot


@pytest.mark.parametrize("l,N", [(2, 9), (3, 7), (4, 6), (5, 4), (6, 3)])
def test_dense_product_matches_oracle_definition(l, N):
    mmot = _mmot()
    h, eps = 0.13, 0.07
    rng = np.random.default_rng(l * 10 + N)
    a = rng.normal(size=(l, N)) * 20.0
    a[0, 1] = -np.inf
    logK = dense.log_kernel(l, N, h, eps)
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64)
    for j in range(l):
        say("dense product l=%d N=%d j=%d" % (l, N, j))
        got = plan.dense_marginal_product(j, to_dev(a)).cpu().numpy()
        ref = dense.marginal_product_log(logK, a, j)
        assert np.array_equal(np.isfinite(got), np.isfinite(ref))
        assert log_rel_err(got, ref) < FP64_TOL, (l, N, j, log_rel_err(got, ref))


def test_dense_product_on_coordinates_matches_oracle():
    mmot = _mmot()
    l, N, eps = 3, 8, 0.05
    x = inputs.graded_grid(N, seed=3)
    rng = np.random.default_rng(5)
    a = rng.normal(size=(l, N)) * 5.0
    logK = dense.log_kernel(l, N, 1.0, eps, x=x)
    plan = mmot.Plan(l, N, inputs.grid_step(N), eps, precision=mmot.FP64, x=x)
    for j in range(l):
        say("dense product on coordinates j=%d" % j)
        got = plan.dense_marginal_product(j, to_dev(a)).cpu().numpy()
        assert log_rel_err(got, dense.marginal_product_log(logK, a, j)) < FP64_TOL


def test_dense_product_equals_the_scans_at_n100():
    # the comparison workload: l = 4, N = 100, eps = 1e-2
    mmot = _mmot()
    l, N, eps = 4, 100, 0.01
    u = inputs.marginals(l, N, K=3, master_seed=0, instance=0)
    h = inputs.grid_step(N)
    a = fastcheck.sinkhorn(u, h, eps, itmax=20, check_every=10**9)["log_phi"]
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64)
    ta = to_dev(a)
    for j in range(l):
        say("dense vs scans l=4 N=100 j=%d" % j)
        d = plan.dense_marginal_product(j, ta).cpu().numpy()
        f = plan.marginal_product(j, ta).cpu().numpy()
        assert log_rel_err(d, f) < FP64_TOL


def test_dense_sweeps_equal_scan_sweeps():
    mmot = _mmot()
    l, N, eps = 4, 60, 0.05
    u = inputs.marginals(l, N, K=3, master_seed=2, instance=1)
    h = inputs.grid_step(N)
    lu = to_dev(np.log(u))
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64, tol=-1.0, itr_max=8, check_every=0)
    a0 = np.full((l, N), -np.log(N))
    ad, af = to_dev(a0), to_dev(a0)
    say("dense sweeps")
    plan.dense_sinkhorn_iter(lu, ad, 8)
    say("scan sweeps")
    plan.sinkhorn_iter(lu, af, 8, want_err=False)
    ref = fastcheck.sinkhorn(u, h, eps, itmax=8, check_every=10**9, log_phi0=a0)["log_phi"]
    assert potentials_err(ad.cpu().numpy(), ref) < FP64_TOL
    assert potentials_err(ad.cpu().numpy(), af.cpu().numpy()) < FP64_TOL


def test_dense_rejects_sizes_beyond_its_limits():
    mmot = _mmot()
    plan = mmot.Plan(4, 2000, inputs.grid_step(2000), 0.01, precision=mmot.FP64)
    a = to_dev(np.zeros((4, 2000)))
    with pytest.raises(mmot.MmotError) as e:
        plan.dense_marginal_product(0, a)
    assert e.value.code == mmot.ERR_UNSUPPORTED
