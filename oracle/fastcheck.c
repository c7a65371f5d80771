/*
 * FP64 log-domain checker for entropic l-marginal OT with L1 cost on a 1-D
 * grid: uniform of step h, or any non-decreasing coordinates x[0..N-1] shared
 * by the l marginals (x = NULL selects the uniform grid).  TEST INFRASTRUCTURE
 * ONLY: the product path never links or calls it.
 *
 * It computes the same quantities as the dense oracle (oracle/dense.py) in
 * O(N * l * 2^(l-1)) per marginal product instead of O(N^l), so that sizes
 * whose N^l tensor does not fit can still be checked.  Tests pin it to the
 * dense oracle on small l and N.
 *
 * Derivation (gap form of the cost; the paper splits the sum into l! ordering
 * classes instead, Sec. 4.2).  For indices i_1..i_l in 0..N-1 let
 * m_x = #{q : i_q <= x}.  Each pair p<q is separated by exactly |i_p - i_q|
 * gaps (x, x+1), and gap x separates m_x (l - m_x) pairs, so
 *     sum_{p<q} |i_p - i_q| = sum_{x=0}^{N-2} m_x (l - m_x),
 * and K = lambda^(that) = prod_x g(m_x) with g(m) = lambda^(m (l - m)).
 * On coordinates x the same count gives sum_{p<q} |x_{i_p} - x_{i_q}| =
 * sum_x (x_{x+1} - x_x) m_x (l - m_x), so gap x carries its own factor
 * g_x(m) = exp(-(x_{x+1} - x_x) m (l - m) / eps) (Sec. 3 remarks that the method
 * carries over to a non-uniform mesh).
 * For the product J_j(y) = sum over i_q (q != j), i_j = y, of K prod phi_q(i_q),
 * let R be the l-1 marginals other than j and S a subset of R.
 *   forward:  F_x(S) = sum of prod_{q in S} phi_q(i_q) * prod_{gaps < x} g(.)
 *             over placements of S in [0, x] (j is to the right of x);
 *             F_x(S) = sum_{T subset S} G_{x-1}(S \ T) prod_{q in T} phi_q(x),
 *             G_x(S) = g(|S|) F_x(S), G_{-1}(S) = [S empty];
 *   backward: H_x(U) = g(|U|) B_x(U), B_x(U) = sum_{T subset U} H_{x+1}(U\T)
 *             prod_{q in T} phi_q(x), H_N(U) = [U empty];
 *   combine:  J_j(y) = sum_{S subset R} F_y(S) H_{y+1}(R \ S).
 * The inner sum over T is done item by item (each marginal placed at most
 * once per position).  Every value is a natural logarithm and every sum a
 * log-sum-exp, so nothing over- or underflows.
 *
 * Objective W = <C, T> (Sec. 2 Eq. mmot distance): carry with every state the
 * cost-weighted sum as well; crossing gap x multiplies a state by g(m) and adds
 * m (l - m) times its value to its weighted part (times the gap's length on
 * coordinates).  Then, on the uniform grid,
 * (C o K) x_{q != j} phi_q (y) = h sum_S [F^w_y(S) H_{y+1}(R\S) + F_y(S) H^w_{y+1}(R\S)]
 * and W = sum_y phi_j(y) times that (no factor h on coordinates).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define FC_MAXL 16

static double lse2(double x, double y)
{
    if (x == -INFINITY) return y;
    if (y == -INFINITY) return x;
    if (x >= y) return x + log1p(exp(y - x));
    return y + log1p(exp(x - y));
}

static int popc(unsigned v)
{
    int c = 0;
    while (v) { c += (int)(v & 1u); v >>= 1; }
    return c;
}

/* Length of the gap between positions p - 1 and p (p >= 1). */
static double gap_len(const double *x, double h, long p)
{
    return x ? x[p] - x[p - 1] : h;
}

static int grid_ok(const double *x, long N)
{
    if (!x) return 1;
    for (long p = 0; p < N; ++p)
        if (!isfinite(x[p]) || (p > 0 && x[p] < x[p - 1])) return 0;
    return 1;
}

/* Factors of a gap of length d on coordinates: log g(m) and log of the cost
   weight m (l - m) d of the objective's weighted part. */
static void set_gap(int l, double d, double eps, double *lg, double *lc)
{
    for (int m = 0; m <= l; ++m) {
        lg[m] = -(double)(m * (l - m)) * (d / eps);
        lc[m] = (m * (l - m) > 0) ? log((double)(m * (l - m)) * d) : -INFINITY;
    }
}

/* log J_j for all y.  a: [l][N] log-potentials (row j ignored).  0 on success. */
int fc_marginal_product(int l, long N, double h, double eps, const double *x, const double *a, int j,
                        double *logJ)
{
    if (l < 2 || l > FC_MAXL || N < 1 || j < 0 || j >= l || !(eps > 0.0) || h < 0.0 || !grid_ok(x, N)) return -1;
    const int n = l - 1;
    const long D = 1L << n;
    int items[FC_MAXL];
    double lg[FC_MAXL + 1];
    for (int q = 0, r = 0; q < l; ++q) if (q != j) items[r++] = q;
    for (int m = 0; m <= l; ++m) lg[m] = -(double)(m * (l - m)) * (h / eps);

    double *F = (double *)malloc(sizeof(double) * (size_t)N * (size_t)D);
    double *A = (double *)malloc(sizeof(double) * (size_t)D);
    if (!F || !A) { free(F); free(A); return -2; }

    /* forward */
    for (long S = 0; S < D; ++S) A[S] = (S == 0) ? 0.0 : -INFINITY;   /* G_{-1} */
    for (long p = 0; p < N; ++p) {
        if (p > 0) {
            if (x)
                for (int m = 0; m <= l; ++m) lg[m] = -(double)(m * (l - m)) * (gap_len(x, h, p) / eps);
            for (long S = 0; S < D; ++S) A[S] = lg[popc((unsigned)S)] + F[(p - 1) * D + S];
        }
        for (int r = 0; r < n; ++r) {
            const double ax = a[(long)items[r] * N + p];
            const long bit = 1L << r;
            for (long S = 0; S < D; ++S)
                if (S & bit) A[S] = lse2(A[S], A[S ^ bit] + ax);
        }
        memcpy(F + p * D, A, sizeof(double) * (size_t)D);
    }
    /* backward + combine; A holds H_{p+1} */
    for (long U = 0; U < D; ++U) A[U] = (U == 0) ? 0.0 : -INFINITY;   /* H_N */
    for (long p = N - 1; p >= 0; --p) {
        double acc = -INFINITY;
        for (long S = 0; S < D; ++S) acc = lse2(acc, F[p * D + S] + A[(D - 1) ^ S]);
        logJ[p] = acc;
        for (int r = 0; r < n; ++r) {
            const double ax = a[(long)items[r] * N + p];
            const long bit = 1L << r;
            for (long U = 0; U < D; ++U)
                if (U & bit) A[U] = lse2(A[U], A[U ^ bit] + ax);
        }
        /* H_p = g B_p with the gap (p - 1, p); H_0 is never used */
        if (x && p > 0)
            for (int m = 0; m <= l; ++m) lg[m] = -(double)(m * (l - m)) * (gap_len(x, h, p) / eps);
        for (long U = 0; U < D; ++U) A[U] += lg[popc((unsigned)U)];
    }
    free(F);
    free(A);
    return 0;
}

/* W = <C, T> for the plan of potentials a (Sec. 2 Eq. mmot distance). */
int fc_objective(int l, long N, double h, double eps, const double *x, const double *a, double *W)
{
    if (l < 2 || l > FC_MAXL || N < 1 || !(eps > 0.0) || h < 0.0 || !grid_ok(x, N)) return -1;
    const int j = l - 1, n = l - 1;
    const long D = 1L << n;
    int items[FC_MAXL];
    double lg[FC_MAXL + 1], lc[FC_MAXL + 1];
    for (int q = 0, r = 0; q < l; ++q) if (q != j) items[r++] = q;
    for (int m = 0; m <= l; ++m) {
        lg[m] = -(double)(m * (l - m)) * (h / eps);
        lc[m] = (m * (l - m) > 0) ? log((double)(m * (l - m))) : -INFINITY;
    }
    double *Fv = (double *)malloc(sizeof(double) * (size_t)N * (size_t)D);
    double *Fw = (double *)malloc(sizeof(double) * (size_t)N * (size_t)D);
    double *Av = (double *)malloc(sizeof(double) * (size_t)D);
    double *Aw = (double *)malloc(sizeof(double) * (size_t)D);
    double *Jh = (double *)malloc(sizeof(double) * (size_t)N);
    if (!Fv || !Fw || !Av || !Aw || !Jh) { free(Fv); free(Fw); free(Av); free(Aw); free(Jh); return -2; }

    for (long S = 0; S < D; ++S) { Av[S] = (S == 0) ? 0.0 : -INFINITY; Aw[S] = -INFINITY; }
    for (long p = 0; p < N; ++p) {
        if (p > 0) {
            if (x) set_gap(l, gap_len(x, h, p), eps, lg, lc);
            for (long S = 0; S < D; ++S) {
                const int m = popc((unsigned)S);
                const double v = Fv[(p - 1) * D + S], w = Fw[(p - 1) * D + S];
                Av[S] = lg[m] + v;
                Aw[S] = lg[m] + lse2(w, lc[m] + v);
            }
        }
        for (int r = 0; r < n; ++r) {
            const double ax = a[(long)items[r] * N + p];
            const long bit = 1L << r;
            for (long S = 0; S < D; ++S)
                if (S & bit) {
                    Av[S] = lse2(Av[S], Av[S ^ bit] + ax);
                    Aw[S] = lse2(Aw[S], Aw[S ^ bit] + ax);
                }
        }
        memcpy(Fv + p * D, Av, sizeof(double) * (size_t)D);
        memcpy(Fw + p * D, Aw, sizeof(double) * (size_t)D);
    }
    for (long U = 0; U < D; ++U) { Av[U] = (U == 0) ? 0.0 : -INFINITY; Aw[U] = -INFINITY; }
    for (long p = N - 1; p >= 0; --p) {
        double acc = -INFINITY;
        for (long S = 0; S < D; ++S) {
            const long Sc = (D - 1) ^ S;
            acc = lse2(acc, Fw[p * D + S] + Av[Sc]);
            acc = lse2(acc, Fv[p * D + S] + Aw[Sc]);
        }
        Jh[p] = acc;
        for (int r = 0; r < n; ++r) {
            const double ax = a[(long)items[r] * N + p];
            const long bit = 1L << r;
            for (long U = 0; U < D; ++U)
                if (U & bit) {
                    Av[U] = lse2(Av[U], Av[U ^ bit] + ax);
                    Aw[U] = lse2(Aw[U], Aw[U ^ bit] + ax);
                }
        }
        if (x && p > 0) set_gap(l, gap_len(x, h, p), eps, lg, lc);
        for (long U = 0; U < D; ++U) {
            const int m = popc((unsigned)U);
            const double v = Av[U], w = Aw[U];
            Av[U] = lg[m] + v;
            Aw[U] = lg[m] + lse2(w, lc[m] + v);
        }
    }
    /* W = h * sum_y exp(a_j(y) + log Jhat(y)) (no h on coordinates), summed
       with a max shift */
    double mx = -INFINITY;
    for (long y = 0; y < N; ++y) {
        const double t = a[(long)j * N + y] + Jh[y];
        if (t > mx) mx = t;
    }
    double s = 0.0;
    if (mx > -INFINITY)
        for (long y = 0; y < N; ++y) s += exp(a[(long)j * N + y] + Jh[y] - mx);
    *W = (x ? 1.0 : h) * s * exp(mx);
    free(Fv); free(Fw); free(Av); free(Aw); free(Jh);
    return 0;
}

/* L1 errors of all l marginals of the plan: err[j] = sum_y |phi_j J_j - u_j|. */
int fc_marginal_errors(int l, long N, double h, double eps, const double *x, const double *u, const double *a,
                       double *err)
{
    double *lj = (double *)malloc(sizeof(double) * (size_t)N);
    if (!lj) return -2;
    for (int j = 0; j < l; ++j) {
        int rc = fc_marginal_product(l, N, h, eps, x, a, j, lj);
        if (rc) { free(lj); return rc; }
        double e = 0.0;
        for (long y = 0; y < N; ++y) e += fabs(exp(a[(long)j * N + y] + lj[y]) - u[(long)j * N + y]);
        err[j] = e;
    }
    free(lj);
    return 0;
}

/*
 * Gauss-Seidel Sinkhorn (Alg. 1 for l marginals, Sec. 4.2 update formulas):
 * a_j <- log u_j - log J_j for j = 0..l-1 per sweep, newest potentials first.
 * a (in/out) holds the starting potentials.  After every check_every-th sweep
 * (and the last) Res = sum_{j<l-1} ||phi_j J_j - u_j||_1 is computed and the
 * loop stops once Res <= tol.  *iters = sweeps done, *res = last Res.
 */
int fc_sinkhorn(int l, long N, double h, double eps, const double *x, const double *u, double *a,
                long itmax, double tol, long check_every, long *iters, double *res)
{
    if (check_every < 1) check_every = 1;
    double *lj = (double *)malloc(sizeof(double) * (size_t)N);
    double *err = (double *)malloc(sizeof(double) * (size_t)l);
    if (!lj || !err) { free(lj); free(err); return -2; }
    double r = INFINITY;
    long it = 0;
    while (it < itmax && r > tol) {
        ++it;
        for (int j = 0; j < l; ++j) {
            int rc = fc_marginal_product(l, N, h, eps, x, a, j, lj);
            if (rc) { free(lj); free(err); return rc; }
            for (long y = 0; y < N; ++y) a[(long)j * N + y] = log(u[(long)j * N + y]) - lj[y];
        }
        if (it % check_every == 0 || it == itmax) {
            r = 0.0;
            for (int j = 0; j < l - 1; ++j) {
                fc_marginal_product(l, N, h, eps, x, a, j, lj);
                for (long y = 0; y < N; ++y) r += fabs(exp(a[(long)j * N + y] + lj[y]) - u[(long)j * N + y]);
            }
        }
    }
    *iters = it;
    *res = r;
    free(lj);
    free(err);
    return 0;
}
