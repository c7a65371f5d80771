#!/usr/bin/env python3
"""Benchmark: l*N*Sinkhorn-iterations per second at fixed marginal error, one MI355X.

Headline workload (one "step"): a batch of 4096 seeded synthetic instances of
the l = 4, N = 1000, eps = 1e-2 problem (3-component Gaussian-mixture marginals
on a uniform grid of [0, 1], +1e-3 floor, normalised), each solved to the FP64
marginal error Res <= 1e-6 with FP32 scans and an FP64 objective
(mmot_solve_batch): rounds of the register-resident sweep kernel (one
workgroup per instance) and the FP64 residual-check kernel.  Inputs are
resident in device memory before the timed region.

value = sum over instances of l * N * sweeps, divided by the wall time of the K
timed steps (bracketed by device synchronisation).

roofline: the dominant kernel's algorithmic HBM bytes per launch (40 B per
marginal-position update: read l - 1 = 3 potential rows and log u_j, write
a_j, FP64) over its average launch duration, from HIP events recorded around
each launch on the batch's stream, against 8 TB/s; the calibrated counter
traffic is attached while the kernel sources match the profiled ones.

Extra fields (skipped with --no-extras): the same batch in FP64 to 1e-8; the
plain configuration (l = 3, N = 64, eps = 0.1, 500 FP64 sweeps, 10 seeds); the
l = 10, N = 1e5, eps = 1e-3 shape (a few tiled sweeps); the Ricker-wavelet
problem (Table 2's sizes, time to each marginal error at N = 80); the 2-D problem (Table 3's
sizes), a non-uniform grid and the Jacobi sweep; the batch on the
one-wavefront solver; one solve per call; continuous-batching serving runs
(the headline shape, and the mixed request stream with l up to 16 and N up to
1e6, cancelled after a fixed window); the oracle timed on the host cores.
--c4 COUNT adds the mixed batch (l 3..8, N log-uniform in [256, 65536], eps in
{1e-1, 1e-2, 1e-3}) with its first COUNT instances (minutes for 4096).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--instances B]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "l4_n1000_eps0.01"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
BYTES_PER_UNIT_L4 = (4 + 1) * 8     # FP64 potentials: read l-1 rows and log u_j, write a_j
ORACLE_SWEEP_CAP = 2000              # bounded CPU sample: instances needing more sweeps stop there
KERNEL_FILES = ("fast.hpp", "scan.hpp", "xf.hpp", "common.hpp", "kernels.hpp", "launch.hpp", "k_single.hip")


def kernel_source_sha1() -> str:
    """Hash of the sources the headline sweep kernel is built from."""
    d = os.path.join(ROOT, "paper_2405_19246_amd", "csrc")
    h = hashlib.sha1()
    for name in KERNEL_FILES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def host_cpu():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def make_batch(count: int, dev, workload=WORKLOAD):
    import torch
    from paper_2405_19246_amd import inputs
    insts = []
    for s in range(count):
        u, h, eps = inputs.workload(workload, instance=s)
        l, N = u.shape
        insts.append(dict(l=l, N=N, h=h, eps=eps, u=u,
                          log_u=torch.tensor(np.log(u), dtype=torch.float64, device=dev),
                          log_phi=torch.zeros((l, N), dtype=torch.float64, device=dev)))
    return insts


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def units_of(res):
    return float(sum(r["l"] * r["N"] * r["iters"] for r in res))


def traffic_entry(sha: str):
    path = os.path.join(ROOT, "profiles", "traffic_l4_n1000.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("kernel_src_sha1") != sha:
        return None
    return t


def _pmc_sum(run_dir: str, kernel_prefix: str):
    """Sum of the one counter of a rocprofv3 --pmc run over the dispatches of a kernel, and their count."""
    import csv
    tot, n = 0.0, 0
    for root, _, files in os.walk(run_dir):
        for fn in files:
            if not fn.endswith("counter_collection.csv"):
                continue
            with open(os.path.join(root, fn)) as f:
                for r in csv.DictReader(f):
                    if r["Kernel_Name"].startswith(kernel_prefix):
                        tot += float(r["Counter_Value"])
                        n += 1
    return tot, n


def write_traffic(root: str):
    """Calibrated HBM bytes per launch of the sweep kernel: FETCH_SIZE and WRITE_SIZE (KiB) each scaled
    by true bytes / counter reading of a plain 256 MiB device copy, over the sweep launches of a
    one-step bench run; units per launch from that run's own JSON line."""
    kern, copy = "void mmot::k_fast_sweep<4, 4, float>", "__amd_rocclr_copyBuffer"
    fetch, nf = _pmc_sum(os.path.join(root, "pmc_bench_FETCH_SIZE"), kern)
    write, nw = _pmc_sum(os.path.join(root, "pmc_bench_WRITE_SIZE"), kern)
    cf, ncf = _pmc_sum(os.path.join(root, "pmc_copy_FETCH_SIZE"), copy)
    cw, ncw = _pmc_sum(os.path.join(root, "pmc_copy_WRITE_SIZE"), copy)
    true_kib = (256 << 20) / 1024.0
    fs, ws = true_kib / (cf / ncf), true_kib / (cw / ncw)
    line = [ln for ln in open(os.path.join(root, "pmc_bench_FETCH_SIZE.log")) if ln.startswith('{"metric"')][-1]
    d = json.loads(line)
    upl = d["roofline"]["units_per_launch"]
    bpl = (fetch / nf * fs + write / nw * ws) * 1024.0
    out = dict(kernel="k_fast_sweep<4,4,float>", workload=d["config"]["workload"],
               kernel_src_sha1=d["kernel_src_sha1"], launches=nf,
               fetch_kib_per_launch_raw=fetch / nf, write_kib_per_launch_raw=write / nw,
               copy_fetch_kib_raw=cf / ncf, copy_write_kib_raw=cw / ncw, copy_kib_true=true_kib,
               fetch_scale=fs, write_scale=ws, hbm_bytes_per_launch=bpl, units_per_launch=upl,
               hbm_bytes_per_unit=bpl / upl, algorithmic_bytes_per_unit=BYTES_PER_UNIT_L4)
    path = os.path.join(ROOT, "profiles", "traffic_l4_n1000.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def _oracle_worker(args):
    """One host process: solve instances of the workload with the oracle for `seconds` of its own time."""
    start, stride, seconds = args
    from oracle import fastcheck
    from paper_2405_19246_amd import inputs
    units, n, s = 0.0, 0, start
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        u, h, eps = inputs.workload(WORKLOAD, instance=s)
        r = fastcheck.sinkhorn(u, h, eps, itmax=ORACLE_SWEEP_CAP, tol=1e-6, check_every=10)
        units += u.shape[0] * u.shape[1] * r["iters"]
        n += 1
        s += stride
    return units, n, time.perf_counter() - t0


def cpu_baseline(seconds: float):
    """The oracle (FP64 C checker, oracle/fastcheck.c, as it stands) on instances of the headline
    workload: all host cores (one process each, instances dealt round-robin) and one core; plus the
    dense FP64 oracle's time per sweep on the plain configuration."""
    import multiprocessing as mp
    from oracle import dense
    from paper_2405_19246_amd import inputs
    model, ncpu = host_cpu()
    workers = max(1, min(16, ncpu))
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(_oracle_worker, [(w, workers, seconds) for w in range(workers)])
    dt = max(p[2] for p in parts)
    units = sum(p[0] for p in parts)
    n = sum(p[1] for p in parts)
    u1, n1, d1 = _oracle_worker((10 ** 6, 1, seconds / 3))
    # dense N^l oracle, plain configuration (l = 3, N = 64, eps = 0.1), a few sweeps
    u, h, eps = inputs.workload("l3_n64_eps0.1", instance=0)
    t2 = time.perf_counter()
    dense.sinkhorn(u, h, eps, itmax=20, check_every=20)
    d2 = (time.perf_counter() - t2) / 20
    return dict(value=units / dt, unit="l*N*sweeps/s", cores=workers, kind="oracle",
                sample="%d instances of %s, each to Res<=1e-6 or %d sweeps, by oracle/fastcheck.c (FP64), "
                       "%d processes over %.1f s" % (n, WORKLOAD, ORACLE_SWEEP_CAP, workers, dt),
                host_cpu=model, host_nproc=ncpu,
                one_core=dict(value=u1 / d1, instances=n1, seconds=d1),
                dense_oracle_plain_config=dict(seconds_per_sweep=d2, value=3 * 64 / d2,
                                               sample="l=3, N=64, eps=0.1, 20 sweeps of oracle/dense.py"))


def plain_config(dev):
    """l = 3, N = 64, eps = 0.1, exactly 500 FP64 sweeps, seeds 0..9 in one batch."""
    import torch
    from paper_2405_19246_amd import inputs, mmot
    insts = []
    for s in range(10):
        u, h, eps = inputs.workload("l3_n64_eps0.1", instance=s)
        insts.append(dict(l=3, N=64, h=h, eps=eps, log_u=torch.tensor(np.log(u), dtype=torch.float64, device=dev),
                          log_phi=torch.zeros((3, 64), dtype=torch.float64, device=dev)))
    mmot.solve_batch(insts, precision=mmot.FP64, tol=-1.0, itr_max=500, check_every=0)
    res, dt = timed(lambda: mmot.solve_batch(insts, precision=mmot.FP64, tol=-1.0, itr_max=500, check_every=0))
    return dict(value=units_of(res) / dt, seconds=dt, seeds=10, sweeps=500, dtype="f64",
                W_seed0=res[0]["W"], Res_seed0=res[0]["marg_err"])


def l10_shape(dev, sweeps: int):
    """l = 10, N = 1e5, eps = 1e-3: a few tiled sweeps in FP32 mode (the scan window here is about 12
    positions, so FP32 mantissas), throughput and the FP64 residual after them."""
    import torch
    from paper_2405_19246_amd import inputs, mmot
    u, h, eps = inputs.workload("l10_n100000_eps0.001", instance=0)
    l, N = u.shape
    lu = torch.tensor(np.log(u), dtype=torch.float64, device=dev)
    lp = torch.zeros((l, N), dtype=torch.float64, device=dev)
    d = [dict(l=l, N=N, h=h, eps=eps, log_u=lu, log_phi=lp)]
    mmot.solve_batch(d, precision=mmot.FP32, tol=-1.0, itr_max=1, check_every=0)
    res, dt = timed(lambda: mmot.solve_batch(d, precision=mmot.FP32, tol=-1.0, itr_max=sweeps, check_every=0))
    return dict(value=units_of(res) / dt, sweeps=sweeps, seconds=dt, ms_per_sweep=dt / sweeps * 1e3,
                Res_after=res[0]["marg_err"], path="tiled (teams of 64 lanes, 8 states each, FP64 mantissas)")


def ricker(dev):
    """The Ricker-wavelet problem (three squared, floored wavelets on [-2, 2]), one FP64 solve per call.

    table2: 100 sweeps at eps = 0.1 for N = 10 ... 160 (wall seconds of one call);
    fig2a: N = 80, eps = 0.1 and 0.05, wall seconds and sweeps to reach each
    marginal error (the residual checked after every sweep)."""
    import torch
    from paper_2405_19246_amd import inputs, mmot

    def run(N, eps, tol, itr_max, check_every):
        u = inputs.ricker_marginals(N)
        _, h = inputs.ricker_grid(N)
        lu = torch.tensor(np.log(u), dtype=torch.float64, device=dev)
        plan = mmot.Plan(3, N, h, eps, precision=mmot.FP64, tol=tol, itr_max=itr_max, check_every=check_every)
        plan.solve(lu)
        (lp, r), dt = timed(lambda: plan.solve(lu))
        return dict(seconds=dt, sweeps=r["iters"], Res=r["marg_err"], W=r["W"])

    table2 = {str(N): run(N, 0.1, -1.0, 100, 0) for N in (10, 20, 40, 80, 160)}
    fig2a = {}
    for eps in (0.1, 0.05):
        fig2a[str(eps)] = {"%.0e" % tol: run(80, eps, tol, 100000, 1) for tol in (1e-3, 1e-5, 1e-7, 1e-9)}
    return {"table2_eps0.1_100_sweeps": table2, "fig2a_n80": fig2a}


def next_rows(dev):
    """The rows built around the hot path, each timed once (FP64, one solve per call).

    twod: three marginals on an N x N grid (Sec. 5.3: U[0, 1] entries), eps = 0.1,
    100 sweeps; grid: l = 4, N = 1000, eps = 1e-2 on a graded non-uniform grid
    to Res <= 1e-8, beside the same marginals on the uniform grid; jacobi: the
    all-marginals sweep against Gauss-Seidel, l = 4, N = 300, eps = 0.05, to 1e-9."""
    import torch
    from paper_2405_19246_amd import inputs, mmot

    def t64(x):
        return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    twod = {}
    for N in (10, 20, 40, 80, 160):
        u = inputs.random_2d_marginals(N, N, seed=N)
        h = 1.0 / (N - 1)
        plan = mmot.Plan2D(N, N, h, h, 0.1, tol=-1.0, itr_max=100)
        lu = t64(np.log(u))
        plan.solve(lu)
        (lp, r), dt = timed(lambda: plan.solve(lu))
        twod[str(N)] = dict(seconds=dt, sweeps=r["iters"], units_per_s=3 * N * N * r["iters"] / dt, W=r["W"])
    grid = {}
    l, N, eps = 4, 1000, 1e-2
    x = inputs.graded_grid(N, seed=1)
    for name, xs in (("graded", x), ("uniform", None)):
        u = inputs.grid_marginals(xs, l, K=3, master_seed=3) if xs is not None else \
            inputs.marginals(l, N, K=3, master_seed=3)
        plan = mmot.Plan(l, N, inputs.grid_step(N), eps, precision=mmot.FP64, tol=1e-8, itr_max=100000,
                         check_every=0, x=xs)
        lu = t64(np.log(u))
        plan.solve(lu)
        (lp, r), dt = timed(lambda: plan.solve(lu))
        grid[name] = dict(seconds=dt, sweeps=r["iters"], units_per_s=l * N * r["iters"] / dt, Res=r["marg_err"])
    jac = {}
    l, N, eps = 4, 300, 0.05
    u = inputs.marginals(l, N, K=3, master_seed=2, instance=7)
    lu = t64(np.log(u))
    for name, jflag in (("jacobi", True), ("gauss_seidel", False)):
        plan = mmot.Plan(l, N, inputs.grid_step(N), eps, precision=mmot.FP64, tol=1e-9, itr_max=200000,
                         check_every=20, jacobi=jflag)
        plan.solve(lu)
        (lp, r), dt = timed(lambda: plan.solve(lu))
        jac[name] = dict(seconds=dt, sweeps=r["iters"], Res=r["marg_err"], W=r["W"])
    return {"twod_eps0.1_100_sweeps": twod, "grid_l4_n1000_eps0.01": grid, "jacobi_l4_n300_eps0.05": jac}


def dense_comparator(dev, sweeps: int = 10):
    """The dense O(N^l) Sinkhorn on the device against the O(N) scans, both FP64, one instance of
    l = 4, N = 100, eps = 1e-2 (the headline shape at N = 100), the same sweeps from the same start;
    then one dense sweep at N = 1000 against the scans' time per sweep there."""
    import torch
    from paper_2405_19246_amd import inputs, mmot
    l, N, eps = 4, 100, 0.01
    u = inputs.marginals(l, N, K=3, master_seed=0, instance=0)
    h = inputs.grid_step(N)
    lu = torch.tensor(np.log(u), dtype=torch.float64, device=dev)
    plan = mmot.Plan(l, N, h, eps, precision=mmot.FP64, tol=-1.0, itr_max=sweeps, check_every=0)
    a0 = torch.full((l, N), -float(np.log(N)), dtype=torch.float64, device=dev)
    ad, af = a0.clone(), a0.clone()
    plan.dense_sinkhorn_iter(lu, a0.clone(), 1)
    plan.sinkhorn_iter(lu, a0.clone(), 1, want_err=False)
    torch.cuda.synchronize()
    _, td = timed(lambda: plan.dense_sinkhorn_iter(lu, ad, sweeps))
    _, tf = timed(lambda: plan.sinkhorn_iter(lu, af, sweeps, want_err=False))
    diff = float(torch.max(torch.abs((ad - ad.mean()) - (af - af.mean()))).item())
    out = dict(l=l, N=N, eps=eps, sweeps=sweeps, dense_ms_per_sweep=td / sweeps * 1e3,
               scans_ms_per_sweep=tf / sweeps * 1e3, scans_speedup=td / tf,
               dense_units_per_s=l * N * sweeps / td, max_potential_difference=diff)
    # the headline shape itself (N = 1000): one dense sweep (10^12 terms per product)
    N2 = 1000
    u2 = inputs.marginals(l, N2, K=3, master_seed=0, instance=0)
    lu2 = torch.tensor(np.log(u2), dtype=torch.float64, device=dev)
    plan2 = mmot.Plan(l, N2, inputs.grid_step(N2), eps, precision=mmot.FP64, tol=-1.0, itr_max=sweeps,
                      check_every=0)
    b0 = torch.full((l, N2), -float(np.log(N2)), dtype=torch.float64, device=dev)
    bd, bf = b0.clone(), b0.clone()
    plan2.sinkhorn_iter(lu2, b0.clone(), 1, want_err=False)
    _, td2 = timed(lambda: plan2.dense_sinkhorn_iter(lu2, bd, 1))
    _, tf2 = timed(lambda: plan2.sinkhorn_iter(lu2, bf, sweeps, want_err=False))
    out["n1000"] = dict(dense_ms_per_sweep=td2 * 1e3, dense_sweeps=1, scans_ms_per_sweep=tf2 / sweeps * 1e3,
                        scans_speedup=td2 / (tf2 / sweeps))
    return out


def c4_batch(dev, count: int, itr_max: int):
    import torch
    from paper_2405_19246_amd import inputs, mmot
    insts = inputs.batch_instances(count)
    for d in insts:
        d["log_u"] = torch.tensor(np.log(d["u"]), dtype=torch.float64, device=dev)
        d["log_phi"] = torch.zeros((d["l"], d["N"]), dtype=torch.float64, device=dev)
    res, dt = timed(lambda: mmot.solve_batch(insts, precision=mmot.FP32, tol=1e-6, itr_max=itr_max, check_every=0))
    st = np.array([r["status"] for r in res])
    return dict(value=units_of(res) / dt, instances=count, seconds=dt, itr_max=itr_max,
                converged=int((st == 0).sum()), not_converged=int((st == mmot.NOT_CONVERGED).sum()),
                failed=int(((st != 0) & (st != mmot.NOT_CONVERGED)).sum()),
                sweeps_max=int(max(r["iters"] for r in res)))


def serve_mixed(seconds: float, grace: float):
    """Requests of the serving configuration: Poisson arrivals at 2000/s, l uniform in 3..16, N
    log-uniform in [1e3, 1e6], eps log-uniform in [1e-3, 1e-1], 3-component mixture marginals (a pool of
    seeded shapes, each request one of them with its own eps), FP32 mode, tol 1e-6.  Arrivals for
    `seconds`, completions collected for `grace` more, then the server is cancelled (queued requests
    dropped, running ones end after the current round)."""
    import ctypes
    from paper_2405_19246_amd import inputs, mmot
    rate = 2000.0
    rng = np.random.default_rng(0)
    pool = []
    for k in range(24):
        l = int(rng.integers(3, 17))
        N = int(round(float(np.exp(rng.uniform(np.log(1e3), np.log(1e6))))))
        u = inputs.marginals(l, N, K=3, master_seed=5, instance=k) if l <= mmot.MAX_L else None
        pool.append((l, N, u))
    arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * seconds * 1.3)))
    arr = arr[arr < seconds]
    pick = rng.integers(0, len(pool), size=len(arr))
    eps = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), size=len(arr)))
    srv = mmot.Server(precision=mmot.FP32, tol=1e-6, itr_max=100000, check_every=0, max_slots=256,
                      block_sweeps=2, hbm_budget_bytes=24 << 30)
    dummy = np.zeros(1)
    tickets, rejected, reasons = [], 0, {}
    t0 = time.perf_counter()
    t_sub = 0.0
    for i, ta in enumerate(arr):
        w = t0 + ta - time.perf_counter()
        if w > 0:
            time.sleep(w)
        l, N, u = pool[pick[i]]
        try:
            if u is None:   # more marginals than the library takes: refused before u is read
                req = mmot.Request(l, N, 1.0 / (N - 1), float(eps[i]), dummy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
                t = ctypes.c_uint64()
                mmot._check(mmot.lib().mmot_serve_submit(srv._h, ctypes.byref(req), ctypes.byref(t)))
            else:
                tickets.append(srv.submit(u, 1.0 / (N - 1), float(eps[i])))
        except mmot.MmotError as e:
            rejected += 1
            reasons[e.code] = reasons.get(e.code, 0) + 1
    t_sub = time.perf_counter() - t0
    deadline = t0 + seconds + grace
    done = {}
    while time.perf_counter() < deadline and len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.05)
    window = time.perf_counter() - t0
    srv.cancel()
    t_c = time.perf_counter()
    while len(done) < len(tickets) and time.perf_counter() - t_c < 60.0:
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.05)
    t_end = time.perf_counter() - t0
    srv.stop()
    conv = [r for r in done.values() if r["status"] == 0 and r["t_done"] - t0 <= window + 1e9]
    lat = np.sort([r["t_done"] - r["t_submit"] for r in conv]) if conv else np.zeros(0)
    units = sum(r["l"] * r["N"] * r["iters"] for r in done.values())  # converged or ended by the cancel
    return dict(offered_req_per_s=rate, seconds_of_arrivals=seconds, submit_seconds=t_sub, window_seconds=window,
                requests=int(len(arr)), accepted=len(tickets), rejected=rejected,
                rejected_by_code={str(k): v for k, v in reasons.items()},
                completed_converged=len(conv), ended=len(done), seconds_to_end_after_cancel=t_end - window,
                p50_latency_s=float(np.percentile(lat, 50)) if lat.size else None,
                p99_latency_s=float(np.percentile(lat, 99)) if lat.size else None,
                units_per_second=units / t_end,
                workload="serving mix: l 3..16, N 1e3..1e6 log-uniform, eps 1e-3..1e-1 log-uniform, 2000 req/s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--c4", type=int, default=0, metavar="COUNT",
                    help="also solve the first COUNT instances of the mixed batch configuration")
    ap.add_argument("--c4-itr-max", type=int, default=100000)
    ap.add_argument("--only", choices=("plain", "l10", "serve_mixed", "ricker", "next_rows", "dense"),
                    help="run only this extra leg and print its JSON (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB device buffer 4 times (reference for HBM byte counters)")
    ap.add_argument("--write-traffic", metavar="PMC_ROOT",
                    help="write profiles/traffic_l4_n1000.json from the rocprofv3 --pmc runs under PMC_ROOT "
                         "(pmc_bench_FETCH_SIZE, pmc_bench_WRITE_SIZE, pmc_copy_FETCH_SIZE, pmc_copy_WRITE_SIZE "
                         "and their .log files); runs on the CPU")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    if args.copy_calibration:
        import torch
        n = 256 << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 4}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: instances are independent and would shard across GPUs "
              "with no communication; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_19246_amd import mmot

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    mmot.lib()
    if args.only:
        leg = {"plain": lambda: plain_config(dev), "l10": lambda: l10_shape(dev, 3),
               "serve_mixed": lambda: serve_mixed(0.5, 8.0), "ricker": lambda: ricker(dev),
               "next_rows": lambda: next_rows(dev), "dense": lambda: dense_comparator(dev)}[args.only]()
        print(json.dumps({"leg": args.only, **leg}), flush=True)
        return
    tol32, tol64 = 1e-6, 1e-8
    batch = make_batch(args.instances, dev)

    def step(prec, tol, fast=True):
        return mmot.solve_batch(batch, precision=prec, tol=tol, itr_max=20000, check_every=0, fast=fast)

    for _ in range(args.warmup):
        step(mmot.FP32, tol32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units = 0.0
    kern_ms, timings, res = [], [], None
    for _ in range(args.steps):
        res = step(mmot.FP32, tol32)
        units += units_of(res)
        kern_ms.append(mmot.last_batch_kernel_ms())
        timings.append(mmot.last_batch_timing())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = units / wall
    ok = all(r["status"] == 0 and r["marg_err"] <= tol32 for r in res)
    iters = np.array([r["iters"] for r in res])

    # roofline of the dominant kernel (the register-resident sweep kernel): algorithmic HBM bytes per
    # launch over its average launch duration (HIP events around each launch on the batch's stream)
    sweep_launches = sum(t["sweep_launches"] for t in timings)
    kname = "k_fast_sweep<4,4,float>"
    avg_ms = sum(t["sweep_ms"] for t in timings) / max(sweep_launches, 1)
    units_per_launch = sum(t["sweep_units"] for t in timings) / max(sweep_launches, 1)
    achieved = units_per_launch * BYTES_PER_UNIT_L4 / (avg_ms / 1e3) / 1e9
    flops_per_unit = 2 * (3 ** 3 - 1) * 2 + 2 ** 3 * 2
    sha = kernel_source_sha1()
    tr = traffic_entry(sha)
    roofline = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s", frac=achieved / PEAK_HBM_GBS,
                    traffic=(tr["hbm_bytes_per_launch"] if tr else None),
                    kernel=kname, avg_launch_ms=avg_ms, launches=sweep_launches,
                    algorithmic_bytes_per_unit=BYTES_PER_UNIT_L4, units_per_launch=units_per_launch,
                    traffic_bytes_per_unit=(tr["hbm_bytes_per_unit"] if tr else None),
                    alu=dict(flops_per_unit=flops_per_unit,
                             achieved_tflops=units_per_launch * flops_per_unit / (avg_ms / 1e3) / 1e12,
                             peak_tflops=PEAK_FP32_TFLOPS),
                    check_ms=sum(t["check_ms"] for t in timings) / args.steps,
                    rounds=[t["rounds"] for t in timings], batch_ms=float(np.mean(kern_ms)))

    out = {
        "metric": "l*N*Sinkhorn-iters/sec at fixed marginal error (Res<=1e-6, FP64-checked)",
        "value": value,
        "unit": "marginal-position updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian-mixture marginals)",
        "config": {"workload": "%s: batch of %d instances, l=4, N=1000, eps=1e-2, FP32 scans to Res<=1e-6"
                               % (WORKLOAD, args.instances),
                   "l": 4, "N": 1000, "eps": 0.01, "instances": args.instances, "tol": tol32,
                   "check_every": 0,
                   "parallelism": "one workgroup (4 wavefronts) per instance, rounds of sweep and check kernels"},
        "all_converged": ok,
        "max_final_res": float(max(r["marg_err"] for r in res)),
        "sweeps": {"min": int(iters.min()), "median": float(np.median(iters)), "max": int(iters.max())},
        "roofline": roofline,
    }

    if not args.no_extras:
        (r64, t64) = timed(lambda: step(mmot.FP64, tol64))
        out["fp64"] = dict(value=units_of(r64) / t64, tol=tol64, seconds=t64,
                           all_converged=all(r["status"] == 0 for r in r64),
                           max_final_res=float(max(r["marg_err"] for r in r64)),
                           kernel_ms=mmot.last_batch_kernel_ms())
        out["plain_config"] = plain_config(dev)
        out["l10_n100000_eps0.001"] = l10_shape(dev, 3)
        out["ricker"] = ricker(dev)
        out["next_rows"] = next_rows(dev)
        out["dense_comparator_l4_n100"] = dense_comparator(dev)
        (rx, tx) = timed(lambda: step(mmot.FP32, tol32, fast=False))
        out["one_wavefront_solver"] = dict(value=units_of(rx) / tx, seconds=tx,
                                           all_converged=all(r["status"] == 0 for r in rx),
                                           speedup_of_register_resident_path=value / (units_of(rx) / tx))
        # one solve per call (mmot_solve: several launches per solve, one instance at a time)
        nplain = min(16, args.instances)
        plans = [mmot.Plan(4, 1000, batch[i]["h"], batch[i]["eps"], precision=mmot.FP32, tol=tol32,
                           itr_max=20000, check_every=0) for i in range(nplain)]

        def plain():
            return [plans[i].solve(batch[i]["log_u"], batch[i]["log_phi"])[1] for i in range(nplain)]

        plain()
        (rp, tp) = timed(plain)
        plain_rate = units_of(rp) / tp
        out["one_solve_per_call"] = dict(value=plain_rate, instances=nplain, seconds=tp,
                                         batched_speedup=value / plain_rate)
        # continuous batching, the headline shape
        from paper_2405_19246_amd import inputs
        rate, dur = 2000.0, 2.0
        rng = np.random.default_rng(0)
        arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * dur * 1.2)))
        arr = arr[arr < dur]
        us = [inputs.workload(WORKLOAD, instance=10000 + i)[0] for i in range(64)]
        h0, e0 = inputs.grid_step(1000), 0.01

        def gen(i):
            if i >= len(arr):
                return None
            return us[i % len(us)], h0, e0, float(arr[i])

        st = mmot.serve(gen, precision=mmot.FP32, tol=tol32, itr_max=20000, check_every=0, max_slots=2048,
                        block_sweeps=100, hbm_budget_bytes=16 << 30)
        out["serve"] = dict(offered_req_per_s=rate, seconds_of_arrivals=dur, requests=int(len(arr)),
                            completed=st["completed"], rejected=st["rejected"], p50_latency_s=st["p50_latency"],
                            p99_latency_s=st["p99_latency"], units_per_second=st["units_per_second"],
                            wall_seconds=st["wall_seconds"], workload=WORKLOAD + " requests")
        out["serve_mixed"] = serve_mixed(0.5, 8.0)
        # a bounded sample of the mixed-batch distribution: its first 256 instances, at most 200
        # sweeps each (most need more; the full configuration runs with --c4 COUNT)
        out["c4_sample_256_cap200"] = c4_batch(dev, 256, 200)
        if args.c4 > 0:
            out["c4"] = c4_batch(dev, args.c4, args.c4_itr_max)
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    elif args.c4 > 0:
        out["c4"] = c4_batch(dev, args.c4, args.c4_itr_max)
    out["kernel_src_sha1"] = sha
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
