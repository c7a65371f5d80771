#!/usr/bin/env python3
"""Benchmark: l*N*Sinkhorn-iterations per second at fixed marginal error, 1 MI355X.

Workload (one "step"): a batch of seeded synthetic instances of the l = 4,
N = 1000, eps = 1e-2 problem (3-component Gaussian-mixture marginals on a
uniform grid of [0, 1], +1e-3 floor, normalised), each solved to the FP64
marginal error Res <= 1e-6 with FP32 scans and an FP64 objective
(mmot_solve_batch): rounds of the register-resident sweep kernel (one
workgroup per instance) and the FP64 residual-check kernel, checks taken when
the sweeps' own error estimate asks for one.  Inputs are resident in device
memory before the timed region.

value = sum over instances of l * N * sweeps, divided by the wall time of the
K timed steps (bracketed by device synchronisation).

Extra fields: the same batch in FP64 to Res <= 1e-8; the same batch on the
extended-range solver (one wavefront per instance); the plain
one-solve-per-call form and the batched speed-up; a short continuous-batching
serving run with p50/p99 latency; the roofline of the sweep kernel; and the
oracle timed on host cores on a bounded sample.

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


def kernel_source_sha1() -> str:
    d = os.path.join(ROOT, "paper_2405_19246_amd", "csrc")
    h = hashlib.sha1()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hpp", ".hip", ".cpp")):
            with open(os.path.join(d, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def make_batch(count: int, dev):
    import torch
    from paper_2405_19246_amd import inputs
    insts = []
    for s in range(count):
        u, h, eps = inputs.workload(WORKLOAD, instance=s)
        l, N = u.shape
        insts.append(dict(l=l, N=N, h=h, eps=eps, u=u,
                          log_u=torch.tensor(np.log(u), dtype=torch.float64, device=dev),
                          log_phi=torch.zeros((l, N), dtype=torch.float64, device=dev)))
    return insts


def timed(fn):
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    out = fn()
    e1.record(s)
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1) / 1e3


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
    with open(os.path.join(run_dir, "run_counter_collection.csv")) as f:
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
               hbm_bytes_per_unit=bpl / upl, algorithmic_bytes_per_unit=24)
    path = os.path.join(ROOT, "profiles", "traffic_l4_n1000.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def cpu_baseline(seconds: float):
    """The oracle (FP64 C checker, one thread) on instances of the same workload."""
    from oracle import fastcheck
    from paper_2405_19246_amd import inputs
    t0 = time.perf_counter()
    units = 0.0
    n = 0
    while time.perf_counter() - t0 < seconds:
        u, h, eps = inputs.workload(WORKLOAD, instance=n)
        r = fastcheck.sinkhorn(u, h, eps, itmax=20000, tol=1e-6, check_every=10)
        units += u.shape[0] * u.shape[1] * r["iters"]
        n += 1
    dt = time.perf_counter() - t0
    return dict(value=units / dt, unit="l*N*sweeps/s", cores=1, kind="oracle",
                sample="%d instances of %s solved to Res<=1e-6 by oracle/fastcheck.c (FP64, 1 thread), %.1f s"
                       % (n, WORKLOAD, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true")
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
    tol32, tol64 = 1e-6, 1e-8
    batch = make_batch(args.instances, dev)

    def step(prec, tol, fast=True):
        return mmot.solve_batch(batch, precision=prec, tol=tol, itr_max=20000, check_every=0, fast=fast)

    for _ in range(args.warmup):
        step(mmot.FP32, tol32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units = 0.0
    kern_ms = []
    timings = []
    res = None
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

    # roofline of the dominant kernel: algorithmic FP32 flops of the gap-form
    # recurrences per marginal-position update (l = 4: 2 * (3^3 - 1) + 2^3 = 60
    # multiply-adds = 120 flops) over its average launch duration (HIP events
    # around each launch on the batch's stream).  The register-resident sweep
    # kernel dominates when it runs; otherwise the extended-range batch kernel
    # (one launch per step) does.
    flops_per_unit = 2 * (3 ** 3 - 1) * 2 + 2 ** 3 * 2
    sweep_launches = sum(t["sweep_launches"] for t in timings)
    if sweep_launches > 0:
        kname = "k_fast_sweep<4,4,float>"
        avg_ms = sum(t["sweep_ms"] for t in timings) / sweep_launches
        units_per_launch = sum(t["sweep_units"] for t in timings) / sweep_launches
        launches = sweep_launches
    else:
        kname = "k_solve_batch<float>"
        avg_ms = sum(t["other_ms"] for t in timings) / args.steps
        units_per_launch = units / args.steps
        launches = args.steps
    achieved = units_per_launch * flops_per_unit / (avg_ms / 1e3) / 1e12
    sha = kernel_source_sha1()
    tr = traffic_entry(sha)
    roofline = dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                    frac=achieved / PEAK_FP32_TFLOPS,
                    traffic=(tr["hbm_bytes_per_launch"] if tr else None),
                    kernel=kname, avg_launch_ms=avg_ms, launches=launches,
                    flops_per_unit=flops_per_unit, units_per_launch=units_per_launch,
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
                   "parallelism": ("one workgroup (4 wavefronts) per instance, rounds of sweep and check kernels"
                                   if sweep_launches > 0 else "one wavefront per instance, persistent launch")},
        "all_converged": ok,
        "sweeps": {"min": int(iters.min()), "median": float(np.median(iters)), "max": int(iters.max())},
        "roofline": roofline,
    }

    if not args.no_extras:
        # FP64 scans to Res <= 1e-8
        (r64, t64) = timed(lambda: step(mmot.FP64, tol64))
        out["fp64"] = dict(value=units_of(r64) / t64, tol=tol64, seconds=t64,
                           all_converged=all(r["status"] == 0 for r in r64),
                           kernel_ms=mmot.last_batch_kernel_ms())
        if sweep_launches > 0:
            # the extended-range solver on the same batch (one wavefront per instance)
            (rx, tx) = timed(lambda: step(mmot.FP32, tol32, fast=False))
            out["extended_range_solver"] = dict(value=units_of(rx) / tx, seconds=tx,
                                                all_converged=all(r["status"] == 0 for r in rx),
                                                speedup_of_fast_path=value / (units_of(rx) / tx))
        # plain form: one solve per call, same accuracy, a subset of the batch
        nplain = min(16, args.instances)
        plans = [mmot.Plan(4, 1000, batch[i]["h"], batch[i]["eps"], precision=mmot.FP32, tol=tol32,
                           itr_max=20000, check_every=0) for i in range(nplain)]

        def plain():
            return [plans[i].solve(batch[i]["log_u"], batch[i]["log_phi"])[1] for i in range(nplain)]

        plain()
        (rp, tp) = timed(plain)
        plain_rate = units_of(rp) / tp
        out["plain_one_solve_per_launch"] = dict(value=plain_rate, instances=nplain, seconds=tp,
                                                 batched_speedup=value / plain_rate)
        # continuous-batching serving: Poisson arrivals of the same problem shape
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
                            completed=st["completed"], p50_latency_s=st["p50_latency"],
                            p99_latency_s=st["p99_latency"], units_per_second=st["units_per_second"],
                            wall_seconds=st["wall_seconds"], workload=WORKLOAD + " requests")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    out["kernel_src_sha1"] = sha
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
