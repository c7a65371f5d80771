"""The paper's O(N) recurrences for three marginals, from its equations.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Computes, for l = 3, linear domain, FP64, 1-based indices as in the paper:
  ftvp1(phi, psi, lam)     = K x_i phi x_j psi              (Sec. 3.1)
  ftvp2(phi, psi, lam, h)  = (C o K) x_i phi x_j psi        (Sec. 3.2)
Both split the double sum over (i, j) into the six ordering sets D_1..D_6 of
Sec. 3 (Eq. D_p), on which the exponent of lambda is the linear form
a_p i + b_p j + c_p k with the coefficient table of Eq. (a_p b_p c_p).  The
partial sums J_{k,p} (Eq. Jk) are built from the discounted prefix sums P and
suffix sums Q (Eq. PkQk) by the first- and second-level recurrences of
Eq. (recurrence formula Jk / PkQk); FTVP-2 adds the moment sums R, S of
Eq. (RkSk) and the recurrences of Eq. (recurrence formula hat Jk / RkSk).

Readings of the printed text taken here (each is checked against brute-force
enumeration in tests/test_oracle_paper.py):
  * the initial values R_{N,5} and R_{N,6} follow from the definitions of R in
    Eq. (RkSk), which carry the factor j = N (resp. i = N); the printed initial
    values drop that factor N;
  * the objective takes one factor h: FTVP-2 already returns h * sum_p hat J,
    so W = <varphi, FTVP-2(phi, psi)> (Alg. FS-3 prints an extra h);
  * the definition of R_{k,4} in Eq. (RkSk) has lambda^{b_4 j} (the printed
    lambda^{b_4 i} names a summation index that is not there).
"""
from __future__ import annotations

import numpy as np

# Eq. (a_p b_p c_p): exponent coefficients on the ordering sets D_1..D_6.
A = {1: -2, 2: 0, 3: -2, 4: 2, 5: 0, 6: 2}
B = {1: 0, 2: -2, 3: 2, 4: -2, 5: 2, 6: 0}
C = {1: 2, 2: 2, 3: 0, 4: 0, 5: -2, 6: -2}


def _one_based(v: np.ndarray) -> np.ndarray:
    """Copy v into an array of length N + 3 with v[1..N] = v, zeros elsewhere."""
    out = np.zeros(v.shape[0] + 3)
    out[1:v.shape[0] + 1] = v
    return out


def _first_level(phi, psi, lam, N):
    """P_{k,p}, Q_{k,p} by the recurrences of Eq. (recurrence formula PkQk)."""
    L = lambda e: lam ** e  # noqa: E731
    P = {p: np.zeros(N + 3) for p in range(1, 7)}
    Q = {p: np.zeros(N + 3) for p in (3, 4)}
    a, b, c = A, B, C
    # forward (prefix) sums
    P[1][1] = phi[1] * L(a[1] + b[1] + c[1])
    P[2][1] = psi[1] * L(2 * a[2] + b[2] + 2 * c[2])
    P[3][1] = phi[1] * L(a[3] + b[3] + c[3])
    P[4][1] = psi[1] * L(a[4] + b[4] + c[4])
    for k in range(2, N + 1):
        P[1][k] = L(b[1] + c[1]) * P[1][k - 1] + phi[k] * L((a[1] + b[1] + c[1]) * k)
        P[2][k] = L(a[2] + c[2]) * P[2][k - 1] + psi[k] * L(a[2] * (k + 1) + b[2] * k + c[2] * (k + 1))
        P[3][k] = L(b[3] + c[3]) * P[3][k - 1] + phi[k] * L((a[3] + b[3] + c[3]) * k)
        P[4][k] = L(a[4] + c[4]) * P[4][k - 1] + psi[k] * L((a[4] + b[4] + c[4]) * k)
    # backward (suffix) sums
    Q[3][N] = psi[N] * L(b[3])
    Q[4][N] = phi[N] * L(a[4])
    P[5][N] = psi[N] * L(a[5] * N + b[5] * N + c[5] * (N - 1))
    P[6][N] = phi[N] * L(a[6] * N + b[6] * (N - 1) + c[6] * (N - 2))
    for k in range(N - 1, 0, -1):
        Q[3][k] = L(b[3]) * Q[3][k + 1] + psi[k] * L(b[3])
        Q[4][k] = L(a[4]) * Q[4][k + 1] + phi[k] * L(a[4])
        P[5][k] = L(-a[5] - c[5]) * P[5][k + 1] + psi[k] * L(a[5] * k + b[5] * k + c[5] * (k - 1))
        P[6][k] = L(-b[6] - c[6]) * P[6][k + 1] + phi[k] * L(a[6] * k + b[6] * (k - 1) + c[6] * (k - 2))
    return P, Q


def _second_level(phi, psi, lam, N, P, Q):
    """J_{k,p} by Eq. (recurrence formula Jk)."""
    L = lambda e: lam ** e  # noqa: E731
    a, b, c = A, B, C
    J = {p: np.zeros(N + 3) for p in range(1, 7)}
    J[1][1] = phi[1] * psi[1] * L(a[1] + b[1] + c[1])
    J[2][1] = 0.0
    for k in range(2, N + 1):
        J[1][k] = L(c[1]) * J[1][k - 1] + psi[k] * P[1][k]
        J[2][k] = L(c[2]) * J[2][k - 1] + phi[k] * P[2][k - 1]
    for k in range(1, N + 1):
        # Q_{N+1,.} is an empty suffix sum (= 0)
        J[3][k] = P[3][k] * Q[3][k + 1]
        J[4][k] = P[4][k] * Q[4][k + 1]
    J[5][N] = 0.0
    for k in range(N - 1, 0, -1):
        J[5][k] = L(-c[5]) * J[5][k + 1] + phi[k + 1] * P[5][k + 1]
    J[6][N] = 0.0
    if N >= 2:
        J[6][N - 1] = 0.0
    for k in range(N - 2, 0, -1):
        J[6][k] = L(-c[6]) * J[6][k + 1] + psi[k + 1] * P[6][k + 2]
    return J


def ftvp1(phi: np.ndarray, psi: np.ndarray, lam: float) -> np.ndarray:
    """(K x_i phi x_j psi)_k for k = 1..N (returned 0-based, length N); Sec. 3.1."""
    N = phi.shape[0]
    ph, ps = _one_based(phi), _one_based(psi)
    P, Q = _first_level(ph, ps, lam, N)
    J = _second_level(ph, ps, lam, N, P, Q)
    return sum(J[p][1:N + 1] for p in range(1, 7))


def ftvp2(phi: np.ndarray, psi: np.ndarray, lam: float, h: float) -> np.ndarray:
    """((C o K) x_i phi x_j psi)_k, k = 1..N, returned 0-based; Sec. 3.2."""
    return _ftvp2(phi, psi, lam, h, 1.0)


def ftvp2_printed_init(phi: np.ndarray, psi: np.ndarray, lam: float, h: float) -> np.ndarray:
    """FTVP-2 with R_{N,5}, R_{N,6} started without the factor N, as printed.

    Kept only so a test can show that this reading disagrees with brute force
    for N >= 2 while the corrected one agrees.
    """
    return _ftvp2(phi, psi, lam, h, 1.0 / phi.shape[0])


def _ftvp2(phi, psi, lam, h, r56_scale):
    N = phi.shape[0]
    ph, ps = _one_based(phi), _one_based(psi)
    P, Q = _first_level(ph, ps, lam, N)
    J = _second_level(ph, ps, lam, N, P, Q)
    L = lambda e: lam ** e  # noqa: E731
    a, b, c = A, B, C
    R = {p: np.zeros(N + 3) for p in range(1, 7)}
    S = {p: np.zeros(N + 3) for p in (3, 4)}
    # Eq. (recurrence formula RkSk): moment sums, forward
    R[1][1] = a[1] * ph[1] * L(a[1] + b[1] + c[1])
    R[2][1] = b[2] * ps[1] * L(2 * a[2] + b[2] + 2 * c[2])
    R[3][1] = a[3] * ph[1] * L(a[3] + b[3] + c[3])
    R[4][1] = b[4] * ps[1] * L(a[4] + b[4] + c[4])
    for k in range(2, N + 1):
        R[1][k] = L(b[1] + c[1]) * R[1][k - 1] + a[1] * k * ph[k] * L((a[1] + b[1] + c[1]) * k)
        R[2][k] = L(a[2] + c[2]) * R[2][k - 1] + b[2] * k * ps[k] * L(a[2] * (k + 1) + b[2] * k + c[2] * (k + 1))
        R[3][k] = L(b[3] + c[3]) * R[3][k - 1] + a[3] * k * ph[k] * L((a[3] + b[3] + c[3]) * k)
        R[4][k] = L(a[4] + c[4]) * R[4][k - 1] + b[4] * k * ps[k] * L((a[4] + b[4] + c[4]) * k)
    # backward; R_{N,5}, R_{N,6} from their definitions (factor N kept)
    S[3][N] = b[3] * N * ps[N] * L(b[3])
    S[4][N] = a[4] * N * ph[N] * L(a[4])
    R[5][N] = r56_scale * b[5] * N * ps[N] * L(a[5] * N + b[5] * N + c[5] * (N - 1))
    R[6][N] = r56_scale * a[6] * N * ph[N] * L(a[6] * N + b[6] * (N - 1) + c[6] * (N - 2))
    for k in range(N - 1, 0, -1):
        S[3][k] = L(b[3]) * S[3][k + 1] + b[3] * k * ps[k] * L(b[3])
        S[4][k] = L(a[4]) * S[4][k + 1] + a[4] * k * ph[k] * L(a[4])
        R[5][k] = L(-a[5] - c[5]) * R[5][k + 1] + b[5] * k * ps[k] * L(a[5] * k + b[5] * k + c[5] * (k - 1))
        R[6][k] = L(-b[6] - c[6]) * R[6][k + 1] + a[6] * k * ph[k] * L(a[6] * k + b[6] * (k - 1) + c[6] * (k - 2))
    # Eq. (recurrence formula hat Jk)
    Jh = {p: np.zeros(N + 3) for p in range(1, 7)}
    Jh[1][1] = (a[1] + b[1] + c[1]) * ph[1] * ps[1] * L(a[1] + b[1] + c[1])
    Jh[2][1] = 0.0
    for k in range(2, N + 1):
        Jh[1][k] = L(c[1]) * (Jh[1][k - 1] + c[1] * J[1][k - 1]) + ps[k] * (R[1][k] + (b[1] + c[1]) * k * P[1][k])
        Jh[2][k] = L(c[2]) * (Jh[2][k - 1] + c[2] * J[2][k - 1]) + ph[k] * (R[2][k - 1] + (a[2] + c[2]) * k * P[2][k - 1])
    for k in range(1, N + 1):
        Jh[3][k] = R[3][k] * Q[3][k + 1] + P[3][k] * S[3][k + 1] + c[3] * k * J[3][k]
        Jh[4][k] = R[4][k] * Q[4][k + 1] + P[4][k] * S[4][k + 1] + c[4] * k * J[4][k]
    Jh[5][N] = 0.0
    for k in range(N - 1, 0, -1):
        Jh[5][k] = (L(-c[5]) * (Jh[5][k + 1] - c[5] * J[5][k + 1])
                    + ph[k + 1] * (R[5][k + 1] + (a[5] * (k + 1) + c[5] * k) * P[5][k + 1]))
    Jh[6][N] = 0.0
    if N >= 2:
        Jh[6][N - 1] = 0.0
    for k in range(N - 2, 0, -1):
        Jh[6][k] = (L(-c[6]) * (Jh[6][k + 1] - c[6] * J[6][k + 1])
                    + ps[k + 1] * (R[6][k + 2] + (b[6] * (k + 1) + c[6] * k) * P[6][k + 2]))
    return h * sum(Jh[p][1:N + 1] for p in range(1, 7))


def fs3_sinkhorn(u: np.ndarray, v: np.ndarray, w: np.ndarray, lam: float, h: float, itmax: int):
    """Three-marginal Sinkhorn with FTVP-1 products (Alg. FS-3), linear domain.

    K is symmetric under any permutation of (i, j, k), so every update uses the
    same FTVP-1 routine on the other two scaling vectors (Sec. 3.3).  Returns
    (phi, psi, varphi, W) with W = <varphi, FTVP-2(phi, psi)> (one factor h).
    """
    N = u.shape[0]
    phi = np.full(N, 1.0 / N)
    psi = np.full(N, 1.0 / N)
    vphi = np.full(N, 1.0 / N)
    for _ in range(itmax):
        phi = u / ftvp1(psi, vphi, lam)
        psi = v / ftvp1(phi, vphi, lam)
        vphi = w / ftvp1(phi, psi, lam)
    W = float(np.dot(vphi, ftvp2(phi, psi, lam, h)))
    return phi, psi, vphi, W
