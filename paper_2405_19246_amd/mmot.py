"""ctypes binding of libmmot (include/mmot.h).  Argument marshalling only.

Every call goes to the HIP library; there is no CPU fallback.  If libmmot.so is
not built, loading raises.  Device buffers are torch CUDA (HIP) tensors of
dtype float64, contiguous, shape [l, N] (marginal logs, log potentials) or [N]
(product output); torch supplies device memory and the current stream only.
"""
from __future__ import annotations

import ctypes
import os
from typing import Callable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmot.so")

OK, ERR_INVALID, ERR_NOMEM, ERR_NUMERIC, NOT_CONVERGED, ERR_UNSUPPORTED, ERR_HIP, ERR_STATE = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32 = 0, 1
FLAG_WARM_START = 1
FLAG_NO_FAST = 2
FLAG_TILES = 4
FLAG_NO_GRAPH = 8
FLAG_JACOBI = 16
MAX_L = 10

_c_d, _c_i32, _c_i64, _c_p = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p


class Problem(ctypes.Structure):
    _fields_ = [("l", _c_i32), ("N", _c_i64), ("h", _c_d), ("eps", _c_d), ("precision", _c_i32),
                ("x", ctypes.POINTER(_c_d))]


class Problem2D(ctypes.Structure):
    _fields_ = [("N", _c_i64), ("M", _c_i64), ("h1", _c_d), ("h2", _c_d), ("eps", _c_d)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", _c_d), ("itr_max", _c_i64), ("check_every", _c_i32), ("flags", _c_i32)]


class Result(ctypes.Structure):
    _fields_ = [("W", _c_d), ("marg_err", _c_d), ("iters", _c_i64), ("status", _c_i32), ("l", _c_i32),
                ("N", _c_i64)]

    def as_dict(self):
        return dict(W=self.W, marg_err=self.marg_err, iters=self.iters, status=self.status, l=self.l, N=self.N)


class Instance(ctypes.Structure):
    _fields_ = [("l", _c_i32), ("N", _c_i64), ("h", _c_d), ("eps", _c_d), ("log_u", _c_p), ("log_phi", _c_p),
                ("x", _c_p)]


class ServeCfg(ctypes.Structure):
    _fields_ = [("precision", _c_i32), ("opts", Opts), ("max_slots", _c_i32), ("block_sweeps", _c_i64),
                ("hbm_budget_bytes", ctypes.c_size_t)]


class Request(ctypes.Structure):
    _fields_ = [("l", _c_i32), ("N", _c_i64), ("h", _c_d), ("eps", _c_d), ("u", ctypes.POINTER(_c_d))]


class RequestRecord(ctypes.Structure):
    _fields_ = [("result", Result), ("t_submit", _c_d), ("t_admit", _c_d), ("t_done", _c_d)]


class ServeStats(ctypes.Structure):
    _fields_ = [("completed", _c_i64), ("rejected", _c_i64), ("wall_seconds", _c_d), ("p50_latency", _c_d),
                ("p99_latency", _c_d), ("units_per_second", _c_d)]


class BatchTiming(ctypes.Structure):
    _fields_ = [("total_ms", _c_d), ("sweep_ms", _c_d), ("check_ms", _c_d), ("other_ms", _c_d),
                ("sweep_units", _c_d), ("sweep_launches", _c_i32), ("rounds", _c_i32)]


REQUEST_FN = ctypes.CFUNCTYPE(ctypes.c_int, _c_p, _c_i64, ctypes.POINTER(Request), ctypes.POINTER(_c_d))

EXPORTS = ["mmot_plan", "mmot_plan_footprint", "mmot_plan_destroy", "mmot_marginal_product", "mmot_sinkhorn_iter",
           "mmot_solve", "mmot_objective", "mmot_marginal_errors", "mmot_solve_batch", "mmot_serve_start",
           "mmot_serve_submit", "mmot_serve_poll", "mmot_serve_stop", "mmot_serve_cancel", "mmot_serve", "mmot_last_batch_kernel_ms",
           "mmot_last_batch_timing", "mmot_marginal_product_noalloc", "mmot_plan_2d", "mmot_plan_2d_destroy",
           "mmot_marginal_product_2d", "mmot_solve_2d", "mmot_objective_2d", "mmot_marginal_errors_2d",
           "mmot_dense_marginal_product", "mmot_dense_sinkhorn_iter", "mmot_last_error"]


class MmotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("mmot error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmmot.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmmot.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2405_19246_amd.csrc.build)")
        # torch's HIP runtime (a separate copy from the one the library links)
        # has to hold the device before the library is loaded: loaded first, the
        # library's first allocation found no device
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        L = ctypes.CDLL(LIB_PATH)
        PP = ctypes.POINTER
        L.mmot_plan.argtypes = [PP(Problem), PP(Opts), _c_p, PP(_c_p)]
        L.mmot_plan_footprint.argtypes = [_c_p, PP(ctypes.c_size_t)]
        L.mmot_plan_destroy.argtypes = [_c_p]
        L.mmot_marginal_product.argtypes = [_c_p, _c_i32, _c_p, _c_p]
        L.mmot_sinkhorn_iter.argtypes = [_c_p, _c_p, _c_p, _c_i64, PP(_c_d)]
        L.mmot_dense_marginal_product.argtypes = [_c_p, _c_i32, _c_p, _c_p]
        L.mmot_dense_sinkhorn_iter.argtypes = [_c_p, _c_p, _c_p, _c_i64]
        L.mmot_solve.argtypes = [_c_p, _c_p, _c_p, PP(Result)]
        L.mmot_objective.argtypes = [_c_p, _c_p, PP(_c_d)]
        L.mmot_marginal_errors.argtypes = [_c_p, _c_p, _c_p, PP(_c_d)]
        L.mmot_solve_batch.argtypes = [PP(Instance), _c_i32, _c_i32, PP(Opts), _c_p, PP(Result)]
        L.mmot_serve_start.argtypes = [PP(ServeCfg), PP(_c_p)]
        L.mmot_serve_submit.argtypes = [_c_p, PP(Request), PP(ctypes.c_uint64)]
        L.mmot_serve_poll.argtypes = [_c_p, ctypes.c_uint64, PP(RequestRecord), _c_p]
        L.mmot_serve_stop.argtypes = [_c_p]
        L.mmot_serve_cancel.argtypes = [_c_p]
        L.mmot_serve.argtypes = [PP(ServeCfg), REQUEST_FN, _c_p, PP(ServeStats), PP(RequestRecord), _c_i64]
        L.mmot_last_batch_kernel_ms.argtypes = [PP(_c_d)]
        L.mmot_last_batch_timing.argtypes = [PP(BatchTiming)]
        L.mmot_marginal_product_noalloc.argtypes = [PP(Problem), _c_i32, _c_p, _c_p, _c_p]
        L.mmot_plan_2d.argtypes = [PP(Problem2D), PP(Opts), _c_p, PP(_c_p)]
        L.mmot_plan_2d_destroy.argtypes = [_c_p]
        L.mmot_marginal_product_2d.argtypes = [_c_p, _c_i32, _c_p, _c_p]
        L.mmot_solve_2d.argtypes = [_c_p, _c_p, _c_p, PP(Result)]
        L.mmot_objective_2d.argtypes = [_c_p, _c_p, PP(_c_d)]
        L.mmot_marginal_errors_2d.argtypes = [_c_p, _c_p, _c_p, PP(_c_d)]
        L.mmot_last_error.argtypes = []
        L.mmot_last_error.restype = ctypes.c_char_p
        for name in EXPORTS[:-1]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().mmot_last_error().decode()


def _check(rc: int, allow=(OK,)) -> int:
    if rc not in allow:
        raise MmotError(rc, last_error())
    return rc


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _flags(warm_start: bool, fast: bool, tiles: bool = False, graph: bool = True, jacobi: bool = False) -> int:
    return ((FLAG_WARM_START if warm_start else 0) | (0 if fast else FLAG_NO_FAST) | (FLAG_TILES if tiles else 0) |
            (0 if graph else FLAG_NO_GRAPH) | (FLAG_JACOBI if jacobi else 0))


def _dev_f64(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("%s must be contiguous float64" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t.data_ptr()


def _host_grid(x, N):
    """Host float64 copy of grid coordinates and a pointer to it (None: uniform grid)."""
    if x is None:
        return None, None
    g = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if g.shape != (N,):
        raise ValueError("x has shape %s, expected (%d,)" % (g.shape, N))
    return g, g.ctypes.data_as(ctypes.POINTER(_c_d))


class Plan:
    """Execution plan for one problem shape (mmot_plan).  x: optional host array of N
    non-decreasing grid coordinates (non-uniform grid; h is then ignored).  jacobi: the
    damped all-marginals sweep (MMOT_FLAG_JACOBI) in solve and sinkhorn_iter."""

    def __init__(self, l: int, N: int, h: float, eps: float, precision: int = FP64, tol: float = 1e-8,
                 itr_max: int = 1000, check_every: int = 10, warm_start: bool = False, stream=None,
                 fast: bool = True, tiles: bool = False, graph: bool = True, x=None, jacobi: bool = False):
        self.l, self.N, self.h, self.eps, self.precision = int(l), int(N), float(h), float(eps), int(precision)
        self.stream = stream
        gx, px = _host_grid(x, self.N)
        p = Problem(self.l, self.N, self.h, self.eps, self.precision, px)
        o = Opts(float(tol), int(itr_max), int(check_every), _flags(warm_start, fast, tiles, graph, jacobi))
        h_ = _c_p()
        _check(lib().mmot_plan(ctypes.byref(p), ctypes.byref(o), _c_p(_stream_handle(stream)), ctypes.byref(h_)))
        self._h = h_

    def close(self):
        if getattr(self, "_h", None):
            lib().mmot_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().mmot_plan_footprint(self._h, ctypes.byref(n)))
        return n.value

    def marginal_product(self, j: int, log_phi, out=None):
        import torch
        pa = _dev_f64(log_phi, (self.l, self.N), "log_phi")
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device=log_phi.device)
        po = _dev_f64(out, (self.N,), "out")
        _check(lib().mmot_marginal_product(self._h, int(j), _c_p(pa), _c_p(po)))
        return out

    def dense_marginal_product(self, j: int, log_phi, out=None):
        """mmot_dense_marginal_product: the O(N^l) definition on the device (comparison only)."""
        import torch
        pa = _dev_f64(log_phi, (self.l, self.N), "log_phi")
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device=log_phi.device)
        po = _dev_f64(out, (self.N,), "out")
        _check(lib().mmot_dense_marginal_product(self._h, int(j), _c_p(pa), _c_p(po)))
        return out

    def dense_sinkhorn_iter(self, log_u, log_phi, n_sweeps: int):
        """mmot_dense_sinkhorn_iter: Gauss-Seidel sweeps with the dense products (in place)."""
        pu = _dev_f64(log_u, (self.l, self.N), "log_u")
        pa = _dev_f64(log_phi, (self.l, self.N), "log_phi")
        _check(lib().mmot_dense_sinkhorn_iter(self._h, _c_p(pu), _c_p(pa), int(n_sweeps)))

    def sinkhorn_iter(self, log_u, log_phi, n_sweeps: int, want_err: bool = True):
        pu = _dev_f64(log_u, (self.l, self.N), "log_u")
        pa = _dev_f64(log_phi, (self.l, self.N), "log_phi")
        err = _c_d()
        _check(lib().mmot_sinkhorn_iter(self._h, _c_p(pu), _c_p(pa), int(n_sweeps),
                                        ctypes.byref(err) if want_err else None))
        return err.value if want_err else None

    def solve(self, log_u, log_phi=None):
        import torch
        pu = _dev_f64(log_u, (self.l, self.N), "log_u")
        if log_phi is None:
            log_phi = torch.empty((self.l, self.N), dtype=torch.float64, device=log_u.device)
        pa = _dev_f64(log_phi, (self.l, self.N), "log_phi")
        r = Result()
        _check(lib().mmot_solve(self._h, _c_p(pu), _c_p(pa), ctypes.byref(r)), allow=(OK, NOT_CONVERGED))
        return log_phi, r.as_dict()

    def objective(self, log_phi) -> float:
        pa = _dev_f64(log_phi, (self.l, self.N), "log_phi")
        W = _c_d()
        _check(lib().mmot_objective(self._h, _c_p(pa), ctypes.byref(W)))
        return W.value

    def marginal_errors(self, log_u, log_phi) -> np.ndarray:
        pu = _dev_f64(log_u, (self.l, self.N), "log_u")
        pa = _dev_f64(log_phi, (self.l, self.N), "log_phi")
        err = (_c_d * self.l)()
        _check(lib().mmot_marginal_errors(self._h, _c_p(pu), _c_p(pa), err))
        return np.array(list(err))


class Plan2D:
    """Three marginals on an N x M grid with separable L1 cost (mmot_plan_2d), FP64.
    Arrays are device float64 tensors [3][M][N] (potentials, marginals) or [M][N]."""

    def __init__(self, N: int, M: int, h1: float, h2: float, eps: float, tol: float = 1e-8, itr_max: int = 1000,
                 check_every: int = 10, warm_start: bool = False, stream=None):
        self.N, self.M = int(N), int(M)
        p = Problem2D(self.N, self.M, float(h1), float(h2), float(eps))
        o = Opts(float(tol), int(itr_max), int(check_every), FLAG_WARM_START if warm_start else 0)
        h = _c_p()
        _check(lib().mmot_plan_2d(ctypes.byref(p), ctypes.byref(o), _c_p(_stream_handle(stream)), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mmot_plan_2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def marginal_product(self, j: int, log_phi, out=None):
        import torch
        pa = _dev_f64(log_phi, (3, self.M, self.N), "log_phi")
        if out is None:
            out = torch.empty((self.M, self.N), dtype=torch.float64, device=log_phi.device)
        po = _dev_f64(out, (self.M, self.N), "out")
        _check(lib().mmot_marginal_product_2d(self._h, int(j), _c_p(pa), _c_p(po)))
        return out

    def solve(self, log_u, log_phi=None):
        import torch
        pu = _dev_f64(log_u, (3, self.M, self.N), "log_u")
        if log_phi is None:
            log_phi = torch.empty((3, self.M, self.N), dtype=torch.float64, device=log_u.device)
        pa = _dev_f64(log_phi, (3, self.M, self.N), "log_phi")
        r = Result()
        _check(lib().mmot_solve_2d(self._h, _c_p(pu), _c_p(pa), ctypes.byref(r)), allow=(OK, NOT_CONVERGED))
        return log_phi, r.as_dict()

    def objective(self, log_phi) -> float:
        pa = _dev_f64(log_phi, (3, self.M, self.N), "log_phi")
        W = _c_d()
        _check(lib().mmot_objective_2d(self._h, _c_p(pa), ctypes.byref(W)))
        return W.value

    def marginal_errors(self, log_u, log_phi) -> np.ndarray:
        pu = _dev_f64(log_u, (3, self.M, self.N), "log_u")
        pa = _dev_f64(log_phi, (3, self.M, self.N), "log_phi")
        err = (_c_d * 3)()
        _check(lib().mmot_marginal_errors_2d(self._h, _c_p(pu), _c_p(pa), err))
        return np.array(list(err))


NOALLOC_BYTES = 16 << 20


def marginal_product_noalloc(l: int, N: int, h: float, eps: float, j: int, log_phi, out, precision: int = FP64,
                             stream=None):
    """mmot_marginal_product_noalloc: the product into the caller's out tensor [N], using the library's
    fixed per-GPU workspace (no allocation, no plan)."""
    pa = _dev_f64(log_phi, (int(l), int(N)), "log_phi")
    po = _dev_f64(out, (int(N),), "out")
    p = Problem(int(l), int(N), float(h), float(eps), int(precision))
    _check(lib().mmot_marginal_product_noalloc(ctypes.byref(p), int(j), _c_p(pa), _c_p(po),
                                               _c_p(_stream_handle(stream))))
    return out


def last_batch_kernel_ms() -> float:
    """Device time of the last solve_batch, first kernel to last (HIP events on its stream)."""
    ms = _c_d()
    _check(lib().mmot_last_batch_kernel_ms(ctypes.byref(ms)))
    return ms.value


def last_batch_timing() -> dict:
    """Per-launch breakdown of the last solve_batch (mmot_last_batch_timing)."""
    t = BatchTiming()
    _check(lib().mmot_last_batch_timing(ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in BatchTiming._fields_}


def solve_batch(instances: Sequence[dict], precision: int = FP32, tol: float = 1e-6, itr_max: int = 100000,
                check_every: int = 10, warm_start: bool = False, stream=None, fast: bool = True,
                tiles: bool = False, graph: bool = True) -> list:
    """mmot_solve_batch: instances are dicts with l, N, h, eps, log_u, log_phi (device tensors) and
    optionally x (device tensor of N non-decreasing grid coordinates: a non-uniform grid).

    fast=False sets MMOT_FLAG_NO_FAST (every solve on the extended-range solver); tiles=True sets
    MMOT_FLAG_TILES (every instance cut into tiles that run on many teams of lanes)."""
    n = len(instances)
    arr = (Instance * max(n, 1))()
    for i, d in enumerate(instances):
        pu = _dev_f64(d["log_u"], (d["l"], d["N"]), "log_u")
        pa = _dev_f64(d["log_phi"], (d["l"], d["N"]), "log_phi")
        px = _dev_f64(d["x"], (d["N"],), "x") if d.get("x") is not None else None
        arr[i] = Instance(int(d["l"]), int(d["N"]), float(d["h"]), float(d["eps"]), pu, pa, px)
    o = Opts(float(tol), int(itr_max), int(check_every), _flags(warm_start, fast, tiles, graph))
    res = (Result * max(n, 1))()
    _check(lib().mmot_solve_batch(arr, n, int(precision), ctypes.byref(o), _c_p(_stream_handle(stream)), res),
           allow=(OK, NOT_CONVERGED))
    return [res[i].as_dict() for i in range(n)]


class Server:
    """Non-blocking continuous-batching server (mmot_serve_start/submit/poll/stop)."""

    def __init__(self, precision: int = FP32, tol: float = 1e-6, itr_max: int = 100000, check_every: int = 10,
                 max_slots: int = 1024, block_sweeps: int = 50, hbm_budget_bytes: int = 8 << 30, fast: bool = True):
        self.cfg = ServeCfg(int(precision), Opts(float(tol), int(itr_max), int(check_every), _flags(False, fast)),
                            int(max_slots), int(block_sweeps), int(hbm_budget_bytes))
        h = _c_p()
        _check(lib().mmot_serve_start(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h
        self._sizes = {}

    def submit(self, u: np.ndarray, h: float, eps: float) -> int:
        u = np.ascontiguousarray(u, dtype=np.float64)
        l, N = u.shape
        req = Request(l, N, float(h), float(eps), u.ctypes.data_as(ctypes.POINTER(_c_d)))
        t = ctypes.c_uint64()
        _check(lib().mmot_serve_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._sizes[t.value] = (l, N)
        return t.value

    def poll(self, ticket: int, want_potentials: bool = False):
        rec = RequestRecord()
        buf = None
        if want_potentials:
            l, N = self._sizes[ticket]
            buf = np.empty((l, N))
        rc = lib().mmot_serve_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(rec),
                                   _c_p(buf.ctypes.data) if buf is not None else None)
        if rc < 0:
            raise MmotError(rc, last_error())
        if rc == 0:
            return None
        out = dict(rec.result.as_dict(), t_submit=rec.t_submit, t_admit=rec.t_admit, t_done=rec.t_done)
        if buf is not None:
            out["log_phi"] = buf
        return out

    def cancel(self):
        """mmot_serve_cancel: drop queued requests, end running ones after the current round."""
        if getattr(self, "_h", None):
            _check(lib().mmot_serve_cancel(self._h))

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(lib().mmot_serve_stop(h))

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def serve(requests: Callable[[int], tuple | None], precision: int = FP32, tol: float = 1e-6, itr_max: int = 100000,
          check_every: int = 10, max_slots: int = 1024, block_sweeps: int = 50, hbm_budget_bytes: int = 8 << 30,
          max_records: int = 0, fast: bool = True):
    """Blocking mmot_serve.  requests(i) returns (u [l, N] array, h, eps, t_arrive) or None when done."""
    keep = {}

    def _cb(_user, idx, req_p, t_p):
        item = requests(int(idx))
        if item is None:
            return 1
        u, h, eps, t_arr = item
        u = np.ascontiguousarray(u, dtype=np.float64)
        keep["u"] = u
        l, N = u.shape
        req_p[0] = Request(l, N, float(h), float(eps), u.ctypes.data_as(ctypes.POINTER(_c_d)))
        t_p[0] = float(t_arr)
        return 0

    cb = REQUEST_FN(_cb)
    cfg = ServeCfg(int(precision), Opts(float(tol), int(itr_max), int(check_every), _flags(False, fast)),
                   int(max_slots), int(block_sweeps), int(hbm_budget_bytes))
    stats = ServeStats()
    recs = (RequestRecord * max(max_records, 1))()
    _check(lib().mmot_serve(ctypes.byref(cfg), cb, None, ctypes.byref(stats), recs if max_records else None,
                            int(max_records)))
    out = dict(completed=stats.completed, rejected=stats.rejected, wall_seconds=stats.wall_seconds,
               p50_latency=stats.p50_latency, p99_latency=stats.p99_latency,
               units_per_second=stats.units_per_second)
    if max_records:
        out["records"] = [dict(recs[i].result.as_dict(), t_submit=recs[i].t_submit, t_admit=recs[i].t_admit,
                               t_done=recs[i].t_done) for i in range(min(max_records, stats.completed))]
    return out
