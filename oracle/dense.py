"""Dense FP64 oracle: the plain definition of entropic l-marginal OT with L1 cost.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Everything here forms the full N^l tensors and follows the paper's definitions:
  * cost on a uniform mesh of step h:  c(i_1..i_l) = h * sum_{p<q} |i_p - i_q|
    (Sec. 3 for l = 3, Sec. 4.2 for general l); on a non-uniform mesh of
    coordinates x (Sec. 3 notes that the method carries over to one):
    c(i_1..i_l) = sum_{p<q} |x[i_p] - x[i_q]|, every marginal on the same x
    (marginals with smaller supports carry zeros on the other points);
  * Gibbs kernel K = exp(-c / eps) = lambda^{sum |i_p - i_q|}, lambda = exp(-h/eps)
    (Sec. 2, Eq. for K; Sec. 4.2);
  * Gibbs form of the plan t = K * prod_q phi_q(i_q) (Sec. 2 Eq. T value; Sec. 4.2);
  * Gauss-Seidel Sinkhorn: phi_j <- u_j / (K x_{q != j} phi_q) in the order
    j = 1..l, each product using the newest phi's (Sec. 2 update formulas,
    Sec. 4.2 update formulas for l marginals), started from phi = 1/N (Alg. 1);
  * residual Res = sum_{j < l} || phi_j * (K x_{q != j} phi_q) - u_j ||_1 taken
    after the sweep with the updated phi's (Alg. 1, Res line; the last marginal
    is exact after its own update, so the paper sums the first l - 1);
  * objective W_eps = <C, T> = sum c * t, the transport cost of the entropic
    plan without the entropy term (Sec. 2 Eq. mmot distance; Sec. 4.2).

The scaling vectors are carried as log-potentials a_q = log phi_q and every
contraction is a log-sum-exp with an exact max shift, so no value over- or
underflows (the log-domain stabilisation of the Remark in Sec. 2, taken to its
limit: all of phi is absorbed into the potentials).  A linear-domain variant of
the same iteration is kept for the paper's unstabilised behaviour.
"""
from __future__ import annotations

import numpy as np


def cost_exponent(l: int, N: int) -> np.ndarray:
    """Integer tensor E[i_1..i_l] = sum_{p<q} |i_p - i_q| (shape (N,)*l)."""
    idx = [np.arange(N).reshape((1,) * p + (N,) + (1,) * (l - 1 - p)) for p in range(l)]
    E = np.zeros((N,) * l, dtype=np.int64)
    for p in range(l):
        for q in range(p + 1, l):
            E = E + np.abs(idx[p] - idx[q])
    return E


def cost_tensor(l: int, N: int, h: float) -> np.ndarray:
    """C = h * E (Sec. 4.2, L1 pairwise cost on a uniform mesh)."""
    return h * cost_exponent(l, N).astype(np.float64)


def cost_tensor_grid(l: int, x: np.ndarray) -> np.ndarray:
    """C[i_1..i_l] = sum_{p<q} |x[i_p] - x[i_q]| on coordinates x (shape (N,)*l)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    pts = [x.reshape((1,) * p + (N,) + (1,) * (l - 1 - p)) for p in range(l)]
    C = np.zeros((N,) * l)
    for p in range(l):
        for q in range(p + 1, l):
            C = C + np.abs(pts[p] - pts[q])
    return C


def log_kernel(l: int, N: int, h: float, eps: float, x=None) -> np.ndarray:
    """log K = -C / eps.  h = 0 gives lambda = 1; eps = 0 is not allowed.
    x: grid coordinates (then h is unused)."""
    if x is not None:
        return -cost_tensor_grid(l, x) / eps
    return -(h / eps) * cost_exponent(l, N).astype(np.float64)


def _expand(v: np.ndarray, axis: int, l: int) -> np.ndarray:
    shape = [1] * l
    shape[axis] = v.shape[0]
    return v.reshape(shape)


def _lse(T: np.ndarray, axes) -> np.ndarray:
    """log(sum(exp(T))) over axes with an exact max shift; all -inf gives -inf."""
    m = np.max(T, axis=axes, keepdims=True)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        s = np.log(np.sum(np.exp(T - m_safe), axis=axes, keepdims=True)) + m_safe
    return np.squeeze(s, axis=axes)


def marginal_product_log(logK: np.ndarray, log_phi: np.ndarray, j: int) -> np.ndarray:
    """log of J_j = K x_{q != j} phi_q, indexed by i_j (Sec. 4.2 tensor-vector product).

    log_phi has shape [l, N]; row j is ignored.
    """
    l = logK.ndim
    T = logK.copy()
    for q in range(l):
        if q != j:
            T = T + _expand(log_phi[q], q, l)
    axes = tuple(q for q in range(l) if q != j)
    return _lse(T, axes)


def marginal_product_lin(K: np.ndarray, phi: np.ndarray, j: int) -> np.ndarray:
    """Linear-domain J_j = K x_{q != j} phi_q (the mode products of Sec. 2)."""
    l = K.ndim
    T = K
    # contract from the last axis down so axis numbers stay valid
    for q in reversed(range(l)):
        if q != j:
            T = np.tensordot(T, phi[q], axes=([q], [0]))
    return T


def log_plan(logK: np.ndarray, log_phi: np.ndarray) -> np.ndarray:
    """log t = log K + sum_q a_q(i_q) (Gibbs form, Sec. 2 / Sec. 4.2)."""
    l = logK.ndim
    T = logK.copy()
    for q in range(l):
        T = T + _expand(log_phi[q], q, l)
    return T


def plan_marginals(logK: np.ndarray, log_phi: np.ndarray) -> np.ndarray:
    """All l marginals of the plan, [l, N]."""
    T = np.exp(log_plan(logK, log_phi))
    l = T.ndim
    return np.stack([T.sum(axis=tuple(q for q in range(l) if q != j)) for j in range(l)])


def residual(logK: np.ndarray, log_phi: np.ndarray, u: np.ndarray) -> float:
    """Res = sum_{j < l} || phi_j * J_j - u_j ||_1 (Alg. 1)."""
    l = logK.ndim
    r = 0.0
    for j in range(l - 1):
        lj = marginal_product_log(logK, log_phi, j)
        r += float(np.sum(np.abs(np.exp(log_phi[j] + lj) - u[j])))
    return r


def objective(l: int, N: int, h: float, eps: float, log_phi: np.ndarray, x=None) -> float:
    """W_eps = <C, T> (Sec. 2 Eq. mmot distance, no entropy term)."""
    logK = log_kernel(l, N, h, eps, x)
    T = np.exp(log_plan(logK, log_phi))
    C = cost_tensor_grid(l, x) if x is not None else cost_tensor(l, N, h)
    return float(np.sum(C * T))


def sinkhorn(u: np.ndarray, h: float, eps: float, itmax: int, tol: float = 0.0,
             check_every: int = 1, log_phi0: np.ndarray | None = None, x=None) -> dict:
    """Generalised Gauss-Seidel Sinkhorn in the log domain (Alg. 1 for l marginals).

    u: [l, N] marginals.  Runs at most itmax sweeps; after every check_every-th
    sweep computes Res and stops once Res <= tol (tol = 0 runs all itmax).
    x: grid coordinates (non-uniform mesh).  Returns dict(log_phi, W, iters,
    res, res_hist).
    """
    l, N = u.shape
    logK = log_kernel(l, N, h, eps, x)
    with np.errstate(divide="ignore"):
        log_u = np.log(u)
    a = np.full((l, N), -np.log(N)) if log_phi0 is None else np.array(log_phi0, dtype=np.float64)
    res = np.inf
    hist = []
    it = 0
    while it < itmax and res > tol:
        it += 1
        for j in range(l):
            a[j] = log_u[j] - marginal_product_log(logK, a, j)
        if it % check_every == 0 or it == itmax:
            res = residual(logK, a, u)
            hist.append((it, res))
    W = objective(l, N, h, eps, a, x)
    return dict(log_phi=a, W=W, iters=it, res=res, res_hist=hist)


def sinkhorn_jacobi(u: np.ndarray, h: float, eps: float, itmax: int, tol: float = 0.0,
                    check_every: int = 1, x=None) -> dict:
    """All-marginals (Jacobi) variant of the iteration, damped by 1/l.

    Not the paper's order (Sec. 4.2 updates one marginal at a time with the
    newest potentials); an alternative that converges to the same plan.  Every
    sweep forms all l products J_j from the potentials at the start of the sweep
    and moves each a_j by 1/l of its own block update:
        a_j <- a_j + (log u_j - a_j - log J_j) / l.
    The new potentials are the mean of the l single-block updates, so by the
    concavity of the dual the dual value never decreases.  Res sums the L1
    errors of all l marginals (no marginal is exact after a Jacobi sweep).
    """
    l, N = u.shape
    logK = log_kernel(l, N, h, eps, x)
    with np.errstate(divide="ignore"):
        log_u = np.log(u)
    a = np.full((l, N), -np.log(N))
    res = np.inf
    it = 0
    while it < itmax and res > tol:
        it += 1
        J = np.stack([marginal_product_log(logK, a, j) for j in range(l)])
        with np.errstate(invalid="ignore"):
            step = np.where(np.isneginf(log_u), -np.inf, log_u - a - J)
        a = np.where(np.isneginf(step), -np.inf, a + step / l)
        if it % check_every == 0 or it == itmax:
            res = sum(float(np.sum(np.abs(np.exp(a[j] + marginal_product_log(logK, a, j)) - u[j]))) for j in range(l))
    return dict(log_phi=a, W=objective(l, N, h, eps, a, x), iters=it, res=res)


def dual_value(u: np.ndarray, logK: np.ndarray, log_phi: np.ndarray) -> float:
    """sum_j <u_j, a_j> - sum K prod_q phi_q: the (eps-scaled) dual objective whose block
    maximisers are the Sinkhorn updates (zero-mass entries contribute nothing)."""
    l = logK.ndim
    lin = 0.0
    for j in range(l):
        m = u[j] > 0
        lin += float(np.sum(u[j][m] * log_phi[j][m]))
    return lin - float(np.sum(np.exp(log_plan(logK, log_phi))))


def sinkhorn_linear(u: np.ndarray, h: float, eps: float, itmax: int) -> dict:
    """Alg. 1 exactly as stated, in the linear domain (no stabilisation).

    Stops at the first sweep that produces a non-finite or zero scaling value
    (over- or underflow), and reports that sweep in 'failed_at'.
    """
    l, N = u.shape
    K = np.exp(log_kernel(l, N, h, eps))
    phi = np.full((l, N), 1.0 / N)
    failed_at = None
    for it in range(1, itmax + 1):
        with np.errstate(all="ignore"):
            for j in range(l):
                phi[j] = u[j] / marginal_product_lin(K, phi, j)
        if not np.all(np.isfinite(phi)) or np.any(phi == 0.0):
            failed_at = it
            break
    return dict(phi=phi, failed_at=failed_at)
