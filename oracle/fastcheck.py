"""ctypes loader for oracle/fastcheck.c.  TEST INFRASTRUCTURE ONLY.

build() compiles the C file with gcc into oracle/_fastcheck.so; load() returns a
small wrapper.  Arrays are float64, C-contiguous, shape [l, N].  x (optional):
non-decreasing grid coordinates [N] shared by the marginals; h is then unused.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fastcheck.c")
_SO = os.path.join(_HERE, "_fastcheck.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        d, l_, i, p = ctypes.c_double, ctypes.c_long, ctypes.c_int, ctypes.c_void_p
        lib.fc_marginal_product.argtypes = [i, l_, d, d, p, p, i, p]
        lib.fc_objective.argtypes = [i, l_, d, d, p, p, p]
        lib.fc_marginal_errors.argtypes = [i, l_, d, d, p, p, p, p]
        lib.fc_sinkhorn.argtypes = [i, l_, d, d, p, p, p, l_, d, l_, p, p]
        for f in (lib.fc_marginal_product, lib.fc_objective, lib.fc_marginal_errors, lib.fc_sinkhorn):
            f.restype = i
        _lib = lib
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(x, N):
    """(array kept alive, pointer) for optional coordinates."""
    if x is None:
        return None, None
    g = _c(x)
    if g.shape != (N,):
        raise ValueError("grid must have N entries")
    return g, g.ctypes.data


def marginal_product_log(log_phi: np.ndarray, j: int, h: float, eps: float, x=None) -> np.ndarray:
    lib = _load()
    a = _c(log_phi)
    l, N = a.shape
    g, gp = _grid(x, N)
    out = np.empty(N)
    rc = lib.fc_marginal_product(l, N, h, eps, gp, a.ctypes.data, j, out.ctypes.data)
    if rc:
        raise RuntimeError("fc_marginal_product failed: %d" % rc)
    return out


def objective(log_phi: np.ndarray, h: float, eps: float, x=None) -> float:
    lib = _load()
    a = _c(log_phi)
    l, N = a.shape
    g, gp = _grid(x, N)
    W = ctypes.c_double()
    rc = lib.fc_objective(l, N, h, eps, gp, a.ctypes.data, ctypes.byref(W))
    if rc:
        raise RuntimeError("fc_objective failed: %d" % rc)
    return W.value


def marginal_errors(u: np.ndarray, log_phi: np.ndarray, h: float, eps: float, x=None) -> np.ndarray:
    lib = _load()
    a, uu = _c(log_phi), _c(u)
    l, N = a.shape
    g, gp = _grid(x, N)
    err = np.empty(l)
    rc = lib.fc_marginal_errors(l, N, h, eps, gp, uu.ctypes.data, a.ctypes.data, err.ctypes.data)
    if rc:
        raise RuntimeError("fc_marginal_errors failed: %d" % rc)
    return err


def sinkhorn(u: np.ndarray, h: float, eps: float, itmax: int, tol: float = 0.0,
             check_every: int = 1, log_phi0: np.ndarray | None = None, x=None) -> dict:
    lib = _load()
    uu = _c(u)
    l, N = uu.shape
    g, gp = _grid(x, N)
    a = np.full((l, N), -np.log(N)) if log_phi0 is None else _c(log_phi0).copy()
    iters = ctypes.c_long()
    res = ctypes.c_double()
    rc = lib.fc_sinkhorn(l, N, h, eps, gp, uu.ctypes.data, a.ctypes.data, itmax, tol, check_every,
                         ctypes.byref(iters), ctypes.byref(res))
    if rc:
        raise RuntimeError("fc_sinkhorn failed: %d" % rc)
    return dict(log_phi=a, iters=iters.value, res=res.value, W=objective(a, h, eps, x))


def sinkhorn_jacobi(u: np.ndarray, h: float, eps: float, itmax: int, tol: float = 0.0,
                    check_every: int = 1, log_phi0: np.ndarray | None = None, x=None) -> dict:
    """The damped all-marginals (Jacobi) iteration of oracle/dense.py (sinkhorn_jacobi)
    with this checker's products: every sweep forms all l products from the
    potentials at its start, then a_j <- a_j + (log u_j - a_j - log J_j) / l.
    Res sums the L1 errors of all l marginals."""
    uu = _c(u)
    l, N = uu.shape
    with np.errstate(divide="ignore"):
        log_u = np.log(uu)
    a = np.full((l, N), -np.log(N)) if log_phi0 is None else _c(log_phi0).copy()
    res = np.inf
    it = 0
    while it < itmax and res > tol:
        it += 1
        J = np.stack([marginal_product_log(a, j, h, eps, x) for j in range(l)])
        with np.errstate(invalid="ignore"):
            step = np.where(np.isneginf(log_u), -np.inf, log_u - a - J)
        a = np.where(np.isneginf(step), -np.inf, a + step / l)
        if it % check_every == 0 or it == itmax:
            res = float(marginal_errors(uu, a, h, eps, x).sum())
    return dict(log_phi=a, iters=it, res=res, W=objective(a, h, eps, x))
