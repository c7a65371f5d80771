"""Batched persistent solves and the serving loop, against the oracle."""
import time

import numpy as np
import pytest

from gpu_util import potentials_err, say, to_dev
from oracle import fastcheck
from paper_2405_19246_amd import inputs

pytestmark = pytest.mark.gpu


def _mmot():
    from paper_2405_19246_amd import mmot
    return mmot


def _mixed(count, seed, l_choices=(2, 3, 4, 5, 6), n_choices=(1, 17, 64, 300, 1000, 2100),
           eps_choices=(0.1, 0.02)):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        l = int(rng.choice(l_choices))
        N = int(rng.choice(n_choices))
        eps = float(rng.choice(eps_choices))
        u = inputs.marginals(l, N, K=2, master_seed=seed, instance=s)
        out.append(dict(l=l, N=N, h=inputs.grid_step(max(N, 2)), eps=eps, u=u))
    return out


def _device_instances(insts):
    for d in insts:
        d["log_u"] = to_dev(np.log(d["u"]))
        d["log_phi"] = to_dev(np.zeros((d["l"], d["N"])))
    return insts


def test_batch_fp64_fixed_sweeps_matches_oracle():
    mmot = _mmot()
    insts = _device_instances(_mixed(24, seed=11))
    say("batch fp64 24 mixed instances, 25 sweeps")
    res = mmot.solve_batch(insts, precision=mmot.FP64, tol=-1.0, itr_max=25, check_every=0)
    for d, r in zip(insts, res):
        ref = fastcheck.sinkhorn(d["u"], d["h"], d["eps"], itmax=25, check_every=25)
        assert r["iters"] == 25 and r["status"] == 0
        assert potentials_err(d["log_phi"].cpu().numpy(), ref["log_phi"]) < 1e-12, (d["l"], d["N"], d["eps"])
        assert abs(r["W"] - ref["W"]) <= 1e-12 * abs(ref["W"]) + 1e-300


def test_batch_fp32_to_tolerance_certified():
    mmot = _mmot()
    insts = _device_instances(_mixed(40, seed=12, l_choices=(3, 4, 5), n_choices=(64, 256, 1000, 3000)))
    say("batch fp32 40 instances to tol 1e-6")
    res = mmot.solve_batch(insts, precision=mmot.FP32, tol=1e-6, itr_max=20000, check_every=10)
    worst = 0.0
    for d, r in zip(insts, res):
        assert r["status"] == 0, r
        err = fastcheck.marginal_errors(d["u"], d["log_phi"].cpu().numpy(), d["h"], d["eps"])
        worst = max(worst, err.max())
        assert err[:-1].sum() <= 1.5e-6 and err.max() <= 2e-6, (d["l"], d["N"], d["eps"], err)
    print("fp32 batch: worst FP64-recomputed marginal error %.3e" % worst)


def test_batch_equals_single_solve_bitwise():
    mmot = _mmot()
    insts = _device_instances(_mixed(12, seed=13, n_choices=(100, 700)))
    say("batch vs single")
    res = mmot.solve_batch(insts, precision=mmot.FP32, tol=1e-6, itr_max=5000, check_every=10)
    for d, r in list(zip(insts, res))[:4]:
        plan = mmot.Plan(d["l"], d["N"], d["h"], d["eps"], precision=mmot.FP32, tol=1e-6, itr_max=5000,
                         check_every=10)
        a, rs = plan.solve(d["log_u"])
        assert rs["iters"] == r["iters"]
        assert np.array_equal(a.cpu().numpy(), d["log_phi"].cpu().numpy())
        assert rs["W"] == r["W"]


@pytest.mark.parametrize("prec", ["FP32", "FP64"])
def test_fast_path_instance_alone_equals_sharing_rounds_with_a_longer_one(prec):
    # the register-resident kernels size a group's workgroups for its longest
    # instance: an N = 64 solve alone runs on one wavefront, beside an N = 1000
    # one on four (padding positions carry zero mass); its iterates, sweep count
    # and objective must not change
    mmot = _mmot()
    pr = getattr(mmot, prec)
    small = dict(l=4, N=64, h=inputs.grid_step(64), eps=0.05, u=inputs.marginals(4, 64, K=2, master_seed=31))
    big = dict(l=4, N=1000, h=inputs.grid_step(1000), eps=0.01, u=inputs.marginals(4, 1000, K=3, master_seed=32))
    say("fast path alone vs shared rounds, %s" % prec)
    alone = _device_instances([dict(small)])
    ra = mmot.solve_batch(alone, precision=pr, tol=1e-6 if prec == "FP32" else 1e-9, itr_max=20000, check_every=0)
    mix = _device_instances([dict(big), dict(small), dict(big)])
    rm = mmot.solve_batch(mix, precision=pr, tol=1e-6 if prec == "FP32" else 1e-9, itr_max=20000, check_every=0)
    t = mmot.last_batch_timing()
    assert t["sweep_launches"] > 0  # the register-resident path ran
    assert rm[1]["iters"] == ra[0]["iters"] and rm[1]["W"] == ra[0]["W"]
    assert np.array_equal(mix[1]["log_phi"].cpu().numpy(), alone[0]["log_phi"].cpu().numpy())


def test_server_mix_equals_alone():
    # a request gives the same result alone and while sharing rounds with others
    mmot = _mmot()
    reqs = _mixed(10, seed=14, l_choices=(3, 4, 5), n_choices=(64, 500, 1500))
    say("server alone")
    srv = mmot.Server(precision=mmot.FP32, tol=1e-6, itr_max=20000, check_every=10, max_slots=4,
                      block_sweeps=40, hbm_budget_bytes=256 << 20)
    alone = []
    for d in reqs[:3]:
        t = srv.submit(d["u"], d["h"], d["eps"])
        while True:
            r = srv.poll(t, want_potentials=True)
            if r is not None:
                break
            time.sleep(0.001)
        alone.append(r)
    srv.stop()
    say("server mix")
    srv = mmot.Server(precision=mmot.FP32, tol=1e-6, itr_max=20000, check_every=10, max_slots=4,
                      block_sweeps=40, hbm_budget_bytes=256 << 20)
    tickets = [srv.submit(d["u"], d["h"], d["eps"]) for d in reqs]
    out = {}
    deadline = time.time() + 120
    while len(out) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t not in out:
                r = srv.poll(t, want_potentials=True)
                if r is not None:
                    out[t] = r
        time.sleep(0.002)
    srv.stop()
    assert len(out) == len(tickets)
    for k in range(3):
        m = out[tickets[k]]
        assert m["iters"] == alone[k]["iters"]
        assert np.array_equal(m["log_phi"], alone[k]["log_phi"])
        assert m["W"] == alone[k]["W"]
    for d, t in zip(reqs, tickets):
        r = out[t]
        assert r["status"] == 0 and r["t_done"] >= r["t_admit"] >= r["t_submit"]
        err = fastcheck.marginal_errors(d["u"], r["log_phi"], d["h"], d["eps"])
        assert err[:-1].sum() <= 1.5e-6


def test_blocking_serve_reports_latency_and_throughput():
    mmot = _mmot()
    reqs = _mixed(16, seed=15, l_choices=(3, 4), n_choices=(64, 256, 1000))

    def gen(i):
        if i >= len(reqs):
            return None
        d = reqs[i]
        return d["u"], d["h"], d["eps"], 0.002 * i

    say("blocking serve 16 requests")
    st = mmot.serve(gen, precision=mmot.FP32, tol=1e-6, itr_max=20000, check_every=10, max_slots=8,
                    block_sweeps=20, hbm_budget_bytes=256 << 20, max_records=16)
    assert st["completed"] == 16 and st["rejected"] == 0
    assert 0 < st["p50_latency"] <= st["p99_latency"] <= st["wall_seconds"] + 1e-6
    assert st["units_per_second"] > 0
    assert all(r["status"] == 0 for r in st["records"])
    print(st["p50_latency"], st["p99_latency"], st["units_per_second"])
