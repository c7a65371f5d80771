"""Seeded synthetic marginals for entropic multi-marginal OT on a uniform 1-D grid.

This module is shared by the tests, the benchmark and the oracle checks.  It only
draws and normalises probability vectors; it holds none of the transport
arithmetic (no kernel, no cost, no Sinkhorn step).

Recipe (stands in for the paper's synthetic 1-D workloads of Sec. 5.1/5.2):
  * grid x_i = i / (N - 1), i = 0..N-1, on [0, 1], step h = 1 / (N - 1)
    (the paper puts N points uniformly on [0, 1], Sec. 5.1, and works on a
    uniform mesh of step h, Sec. 3);
  * each marginal is an equal-weight mixture of K Gaussians with means
    U[0.2, 0.8] and standard deviations U[0.05, 0.15], evaluated at the nodes;
  * then either a floor is added to the density before normalising
    (``floor``), or the normalised mixture is blended with the uniform
    distribution (``uniform_frac``);
  * marginal q of instance s draws from numpy PCG64 seeded with the
    sequence (master_seed, s, q), so every marginal is reproducible alone.

The Ricker workload of Sec. 5.2 is deterministic (``ricker_marginals``): N
uniform points on [-2, 2], three wavelets shifted by tau, squared and
normalised with the floor delta of that section.
"""
from __future__ import annotations

import numpy as np


def grid_step(N: int) -> float:
    """Grid step h of N uniform points on [0, 1]; a single point gets h = 1."""
    return 1.0 / (N - 1) if N > 1 else 1.0


def _rng(master_seed: int, instance: int, marginal: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([master_seed, instance, marginal])))


def mixture_marginal(N: int, K: int, rng: np.random.Generator, floor: float = 1e-3,
                     uniform_frac: float = 0.0) -> np.ndarray:
    """One probability vector of length N (float64, sums to 1 up to rounding)."""
    x = np.linspace(0.0, 1.0, N) if N > 1 else np.zeros(1)
    mu = rng.uniform(0.2, 0.8, size=K)
    sd = rng.uniform(0.05, 0.15, size=K)
    dens = np.zeros(N)
    for k in range(K):
        dens += np.exp(-0.5 * ((x - mu[k]) / sd[k]) ** 2) / (sd[k] * np.sqrt(2.0 * np.pi))
    dens /= K
    if uniform_frac > 0.0:
        p = dens / dens.sum()
        p = (1.0 - uniform_frac) * p + uniform_frac / N
    else:
        p = dens + floor
    return p / p.sum()


def marginals(l: int, N: int, K: int = 2, master_seed: int = 0, instance: int = 0,
              floor: float = 1e-3, uniform_frac: float = 0.0) -> np.ndarray:
    """Array [l, N] of marginals for one instance."""
    return np.stack([mixture_marginal(N, K, _rng(master_seed, instance, q), floor, uniform_frac)
                     for q in range(l)])


def uniform_random_marginals(l: int, N: int, seed: int = 0) -> np.ndarray:
    """The paper's Sec. 5.1 recipe: i.i.d. U[0, 1] entries, each row normalised."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(0.0, 1.0, size=(l, N))
    return u / u.sum(axis=1, keepdims=True)


def ricker_grid(N: int):
    """(t, h): N uniform points on [-2, 2] and their step (Sec. 5.2)."""
    t = np.linspace(-2.0, 2.0, N)
    return t, (4.0 / (N - 1) if N > 1 else 1.0)


def ricker(t: np.ndarray, A: float = 1.0, F0: float = 1.0) -> np.ndarray:
    """Ricker wavelet A (1 - 2 pi^2 F0^2 t^2) exp(-pi^2 F0^2 t^2) (Sec. 5.2)."""
    z = (np.pi * F0 * t) ** 2
    return A * (1.0 - 2.0 * z) * np.exp(-z)


def ricker_marginals(N: int, taus=(0.0, 0.75, 1.5), delta: float = 1e-3) -> np.ndarray:
    """Array [len(taus), N]: marginal q is (f_q^2 / |f_q^2|_1 + delta) / (1 + N delta).

    f_q(t) = R(t - tau_q) on the grid of ``ricker_grid`` with A = F0 = 1.  The
    1-norm is the plain sum over the nodes and the normalising constant in
    the denominator is N, so each row sums to 1 (Sec. 5.2's squared-signal
    normalisation with a floor, read on the discrete grid).
    """
    t, _ = ricker_grid(N)
    out = []
    for tau in taus:
        f2 = ricker(t - tau) ** 2
        out.append((f2 / f2.sum() + delta) / (1.0 + N * delta))
    return np.stack(out)


def graded_grid(N: int, seed: int = 0, spread: float = 0.8) -> np.ndarray:
    """N increasing coordinates on [0, 1]: gaps drawn uniformly from
    [1 - spread, 1 + spread] times the mean gap (seeded), scaled to end at 1."""
    if N == 1:
        return np.zeros(1)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2**31 - 2])))
    g = rng.uniform(1.0 - spread, 1.0 + spread, N - 1)
    x = np.concatenate([[0.0], np.cumsum(g)])
    return x / x[-1]


def grid_marginals(x: np.ndarray, l: int, K: int = 2, master_seed: int = 0, instance: int = 0,
                   floor: float = 1e-3) -> np.ndarray:
    """Array [l, N] of Gaussian-mixture masses at the coordinates x (the uniform
    recipe above with x in place of the uniform nodes)."""
    N = x.shape[0]
    out = []
    for q in range(l):
        rng = _rng(master_seed, instance, q)
        mu = rng.uniform(0.2, 0.8, size=K)
        sd = rng.uniform(0.05, 0.15, size=K)
        dens = np.zeros(N)
        for k in range(K):
            dens += np.exp(-0.5 * ((x - mu[k]) / sd[k]) ** 2) / (sd[k] * np.sqrt(2.0 * np.pi))
        p = dens / K + floor
        out.append(p / p.sum())
    return np.stack(out)


def merge_supports(supports, weights):
    """Marginals on their own supports -> (x, u) on one grid.

    supports[q]: coordinates of marginal q (any order, distinct within q);
    weights[q]: its non-negative masses.  x is the sorted union of all the
    coordinates; u[q] holds marginal q's normalised masses at its own points and
    zero elsewhere.
    """
    x = np.unique(np.concatenate([np.asarray(s, dtype=np.float64) for s in supports]))
    u = np.zeros((len(supports), x.shape[0]))
    for q, (s, w) in enumerate(zip(supports, weights)):
        s = np.asarray(s, dtype=np.float64)
        w = np.asarray(w, dtype=np.float64)
        np.add.at(u[q], np.searchsorted(x, s), w)
        u[q] /= u[q].sum()
    return x, u


def random_2d_marginals(N: int, M: int, seed: int = 0) -> np.ndarray:
    """Sec. 5.3's recipe on an N x M grid: three arrays of i.i.d. U[0, 1] entries,
    each normalised; shape [3][M][N] (entry (i1, i2) at [q, i2, i1])."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2**31 - 3])))
    u = rng.uniform(0.0, 1.0, size=(3, M, N))
    return u / u.reshape(3, -1).sum(axis=1)[:, None, None]


# Named workloads.  Each entry: l, N, K, eps, floor, uniform_frac.
WORKLOADS = {
    # plain method: l=3, N=64, 2 components, eps=0.1, fixed 500 sweeps
    "l3_n64_eps0.1": dict(l=3, N=64, K=2, eps=0.1, floor=1e-3, uniform_frac=0.0),
    # l=4, N=1000, 3 components, eps=1e-2
    "l4_n1000_eps0.01": dict(l=4, N=1000, K=3, eps=1e-2, floor=1e-3, uniform_frac=0.0),
    # dense comparator size of the same shape
    "l4_n100_eps0.01": dict(l=4, N=100, K=3, eps=1e-2, floor=1e-3, uniform_frac=0.0),
    # l=10, N=1e5, 5 components + 10% uniform, eps=1e-3
    "l10_n100000_eps0.001": dict(l=10, N=100000, K=5, eps=1e-3, floor=0.0, uniform_frac=0.1),
}


def workload(name: str, instance: int = 0, master_seed: int = 0):
    """(u [l, N], h, eps) for a named workload and instance index."""
    w = WORKLOADS[name]
    u = marginals(w["l"], w["N"], w["K"], master_seed, instance, w["floor"], w["uniform_frac"])
    return u, grid_step(w["N"]), w["eps"]


def batch_instances(count: int, master_seed: int = 0, l_range=(3, 8), n_range=(256, 65536),
                    eps_choices=(1e-1, 1e-2, 1e-3), K: int = 3):
    """Uneven batch: l uniform in l_range, N log-uniform in n_range, eps from eps_choices.

    Returns a list of dicts {l, N, h, eps, u}.  The shape draw uses its own
    stream (master_seed, -1) so that instance s's marginals do not depend on
    how many instances are drawn.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([master_seed, 2**31 - 1])))
    out = []
    for s in range(count):
        l = int(rng.integers(l_range[0], l_range[1] + 1))
        N = int(round(float(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))))
        eps = float(eps_choices[int(rng.integers(0, len(eps_choices)))])
        u = marginals(l, N, K, master_seed, s)
        out.append(dict(l=l, N=N, h=grid_step(N), eps=eps, u=u))
    return out
