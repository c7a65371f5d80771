// Register-resident solver: one workgroup per instance, block floating point.
//
// Same dynamic program as scan.hpp (gap form of the L1 cost, subset states,
// level-synchronous discounted scans), laid out for instances whose N fits one
// workgroup chunk (64 * waves * V positions, thread t owns positions
// t V .. t V + V - 1):
//   * the l rows of scaling factors phi_q = exp(a_q) stay in registers from
//     sweep to sweep; the potentials a_q themselves (FP64) live in memory and
//     are touched once per update;
//   * inside a thread every state and every row keeps ONE exponent for its V
//     values (block floating point), so the inner multiply-adds are plain FMAs
//     in the mantissa type; values crossing lanes and wavefronts are
//     extended-range numbers (XF);
//   * lanes combine by Kogge-Stone shuffles, wavefronts through LDS (one
//     barrier per level and direction).
// Block floating point is exact up to rounding while the values one thread
// holds span less exponent range than the mantissa type can represent next to
// each other.  Before each product the workgroup checks that bound; a product
// that would exceed it is computed by the extended-range pass of scan.hpp
// instead (wavefront 0), so every iterate is the extended-range solver's up to
// rounding.
#pragma once
#include <type_traits>

#include "scan.hpp"

namespace mmot {

constexpr int FAST_MAXW = 16;  // wavefronts per workgroup at most

template <typename M, int L, int V>
struct FastConst {
    XG<M> g[L];                 // g(k) as an extended-range factor
    GV<M> gv[L];                // g(k) as a value
    GV<M> gp[L][V];             // g(k)^(t + 1), t < V
    XG<M> gstep[L][6];          // g(k)^(V 2^s): lanes
    XG<M> gwave[L][FAST_MAXW];  // g(k)^(64 V d): wavefronts
    XG<M> glane[L][WAVE];       // g(k)^(V s): carry to the s-th lane in scan order
};

// Fill the constants (block-cooperative; caller syncs).
template <typename M, int L, int V>
__device__ void fast_consts(FastConst<M, L, V> &C, double hoe, int tid, int nthreads)
{
    constexpr int W = 2 + V + 6 + FAST_MAXW + WAVE;
    for (int idx = tid; idx < L * W; idx += nthreads) {
        const int k = idx % L, w = idx / L;
        const double lg = -(double)(k * (L - k)) * hoe;
        if (w == 0) C.g[k] = xg_from_log<M>(lg);
        else if (w == 1) C.gv[k] = gv_from_log<M>(lg);
        else if (w < 2 + V) C.gp[k][w - 2] = gv_from_log<M>(lg * (double)(w - 1));
        else if (w < 2 + V + 6) C.gstep[k][w - 2 - V] = xg_from_log<M>(lg * (double)(V << (w - 2 - V)));
        else if (w < 2 + V + 6 + FAST_MAXW) {
            const int d = w - 8 - V;
            C.gwave[k][d] = xg_from_log<M>(lg * (double)(WAVE * V * d));
        } else {
            const int sl = w - 8 - V - FAST_MAXW;
            C.glane[k][sl] = xg_from_log<M>(lg * (double)(V * sl));
        }
    }
}

// Block-wide FP64 sum (same value in every thread); uses red[0..FAST_MAXW).
__device__ __forceinline__ double block_sum(double x, double *red, int lane, int wave, int nw)
{
    x = wave_sum(x);
    lds_barrier();
    if (lane == 0) red[wave] = x;
    lds_barrier();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

// Block-wide OR with one barrier; consecutive calls alternate between the two
// halves of fl[2][FAST_MAXW] (phase), so no reset is needed.
__device__ __forceinline__ bool block_any(bool p, int *fl, int &phase, int lane, int wave, int nw)
{
    const bool w = __ballot(p) != 0;
    if (lane == 0) fl[phase * FAST_MAXW + wave] = w ? 1 : 0;
    lds_barrier();
    int r = 0;
    for (int i = 0; i < nw; ++i) r |= fl[phase * FAST_MAXW + i];
    phase ^= 1;
    return r != 0;
}

// One direction of the level-synchronous scan over the whole instance chunk.
//   pm/pe: block-floating-point rows; rows 0 .. l-2 are the summed marginals
//   Fm/Fe: out, states (mantissas relative to 2^Fe[S]) at the thread's positions;
//          the largest |Fm[S][.]| is in [1/4, 2], or all are 0 and Fe[S] is the
//          zero exponent
//   cin:   out, state at the position before the thread's first (scan order), XF
//   xw:    LDS, [2][FAST_MAXW][D] wavefront aggregates; level k of this scan uses
//          half (k + par) & 1
template <int L, int V, typename M, bool FWD>
__device__ __forceinline__ void bscan(const M (&pm)[L][V], const int (&pe)[L], M (&Fm)[1 << (L - 1)][V],
                                      int (&Fe)[1 << (L - 1)], XF<M> (&cin)[1 << (L - 1)],
                                      const FastConst<M, L, V> &C, XF<M> *xw, int par, int lane, int wave, int nw)
{
    constexpr int n = L - 1;
    constexpr int D = 1 << n;
    constexpr int NWMAX = fast_threads(L, sizeof(M) == 4 ? 1 : 0) / WAVE;
    const int sl = FWD ? lane : WAVE - 1 - lane;
    const int sw = FWD ? wave : nw - 1 - wave;

#pragma unroll
    for (int k = 1; k <= n; ++k) {
        const int half = (k + par) & 1;
        M loc[D][V];
        int Ein[D];
#pragma unroll
        for (int S = 1; S < D; ++S) {
            if (popc(S) != k) continue;
            // exponent bound of each inflow term and their maximum
            int Et[D];
            int E = XF_ZERO_E;
#pragma unroll
            for (int T = 1; T < D; ++T) {
                if ((T & S) != T) continue;
                int et = 0;
#pragma unroll
                for (int r = 0; r < n; ++r)
                    if (T & (1 << r)) et += pe[r];
                const int Sp = S ^ T;
                if (Sp) et += Fe[Sp] + C.g[popc(Sp)].e;
                Et[T] = et;
                E = max(E, et);
            }
            // previous-position states before the thread's first position
            M cm[D];
#pragma unroll
            for (int Sp = 1; Sp < D; ++Sp)
                if ((Sp & S) == Sp && Sp != S) cm[Sp] = xldexp(cin[Sp].m, cin[Sp].e - Fe[Sp]);
            M mx = M(0);
#pragma unroll
            for (int t = 0; t < V; ++t) {
                const int v = FWD ? t : V - 1 - t;
                const int vp = FWD ? v - 1 : v + 1;
                M in = M(0);
#pragma unroll
                for (int T = 1; T < D; ++T) {
                    if ((T & S) != T) continue;
                    M pp = M(1);
#pragma unroll
                    for (int r = 0; r < n; ++r)
                        if (T & (1 << r)) pp *= pm[r][v];
                    const int Sp = S ^ T;
                    if (Sp == 0) {
                        in = fma(xldexp(M(1), Et[T] - E), pp, in);
                    } else {
                        const M prev = (t == 0) ? cm[Sp] : Fm[Sp][vp];
                        const M cf = xldexp(C.g[popc(Sp)].hi, Et[T] - E);
                        in = fma(cf * prev, pp, in);
                    }
                }
                loc[S][v] = (t == 0) ? in : gmul(C.gv[k], loc[S][vp], in);
                mx = max(mx, loc[S][v]);
            }
            // tighten the exponent to the values actually there (zero: zero exponent)
            Ein[S] = (mx == M(0)) ? XF_ZERO_E : E;
            if (mx != M(0)) {
                const int d = xexpo(mx);
                Ein[S] += d;
#pragma unroll
                for (int v = 0; v < V; ++v) loc[S][v] = xldexp(loc[S][v], -d);
            }
        }
        // lanes: Kogge-Stone on the thread aggregates (extended range), DPP moves
        XB<M> excl[D];
#pragma unroll
        for (int S = 1; S < D; ++S) {
            if (popc(S) != k) continue;
            const XB<M> a = xb_of(xnorm(XF<M>{loc[S][FWD ? V - 1 : 0], Ein[S]}));
            XB<M> incl;
            if (FWD) {
                incl = ks_up_dpp(a, C.gstep[k], C.glane[k], lane);
                excl[S] = dpp_xb<0x138>(incl);  // wave_shr:1, zero in lane 0
            } else {
                incl = ks_down_dpp(a, C.gstep[k], C.glane[k], lane);
                excl[S] = dpp_xb<0x130>(incl);  // wave_shl:1, zero in lane 63
            }
            const XF<M> wagg = xf_of(rlane_xb(incl, FWD ? WAVE - 1 : 0));
            if (lane == 0) xw[(half * FAST_MAXW + sw) * D + S] = wagg;
        }
        lds_barrier();
        // wavefronts: carry into this wavefront from the earlier ones, then per lane
#pragma unroll
        for (int S = 1; S < D; ++S) {
            if (popc(S) != k) continue;
            // (unrolled to the block's wavefront count, so the LDS reads go out together)
            XB<M> wc = {M(0), 0};
#pragma unroll
            for (int w = 0; w < NWMAX - 1; ++w) {  // slots are indexed in scan order
                XB<M> o = xb_of(xw[(half * FAST_MAXW + w) * D + S]);
                if (w >= sw) o = XB<M>{M(0), 0};
                wc = xb_addg(wc, o, C.gwave[k][max(sw - 1 - w, 0)]);
            }
            const XF<M> c = xf_of(xb_addg(excl[S], wc, C.glane[k][sl]));
            cin[S] = c;
            // block exponent of the state: the larger of the local part and the carry part
            const int ec = c.m == M(0) ? XF_ZERO_E : c.e + C.g[k].e;
            const int F = max(Ein[S], ec);
            Fe[S] = F;
            const M sc = xldexp(M(1), Ein[S] - F);
            const M cmk = xldexp(c.m, c.e - F);
#pragma unroll
            for (int t = 0; t < V; ++t) {
                const int v = FWD ? t : V - 1 - t;
                Fm[S][v] = gmul(C.gp[k][t], cmk, loc[S][v] * sc);
            }
        }
    }
}

// Natural log of a combine result j 2^E (FP64; -inf for j = 0).
template <typename M>
__device__ __forceinline__ double jlog(M j, int E)
{
    if (j == M(0)) return -INFINITY;
    if constexpr (sizeof(M) == 4)
        return xlog_hw(j, E);
    else
        return xto_log(XF<M>{j, E});
}

// log J_j at the thread's positions from the two scans (natural log, FP64),
// handed to at(v, log J_j) position by position.  The forward states come from
// LDS: fm[((S - 1) V + v) T + tid], fe[(S - 1) T + tid] with T threads per
// workgroup.
template <int L, int V, typename M, typename At>
__device__ __forceinline__ void bcombine(const M *fm, const int *fe, int tid, int T,
                                         const M (&Bm)[1 << (L - 1)][V], const int (&Be)[1 << (L - 1)],
                                         const XF<M> (&cinB)[1 << (L - 1)], const FastConst<M, L, V> &C, At &&at)
{
    constexpr int D = 1 << (L - 1);
    int Fe[D];
#pragma unroll
    for (int S = 1; S < D; ++S) Fe[S] = fe[(S - 1) * T + tid];
    // positions v < V-1: the next position's backward state is in this thread
    if (V > 1) {
        int TE[D];
        int E = XF_ZERO_E;
#pragma unroll
        for (int S = 0; S < D; ++S) {
            const int U = (D - 1) ^ S;
            TE[S] = (S ? Fe[S] : 0) + (U ? Be[U] + C.g[popc(U)].e : 0);
            E = max(E, TE[S]);
        }
        M cf[D];
#pragma unroll
        for (int S = 0; S < D; ++S) {
            const int U = (D - 1) ^ S;
            cf[S] = xldexp(U ? C.g[popc(U)].hi : M(1), TE[S] - E);
        }
#pragma unroll
        for (int v = 0; v < V - 1; ++v) {
            M j = M(0);
#pragma unroll
            for (int S = 0; S < D; ++S) {
                const int U = (D - 1) ^ S;
                const M f = S ? fm[((S - 1) * V + v) * T + tid] : M(1);
                const M b = U ? Bm[U][v + 1] : M(1);
                j = fma(cf[S] * f, b, j);
            }
            at(v, jlog(j, E));
        }
    }
    // last position: the next position's backward state is the carry into this thread
    {
        int TE[D];
        int E = XF_ZERO_E;
#pragma unroll
        for (int S = 0; S < D; ++S) {
            const int U = (D - 1) ^ S;
            TE[S] = (S ? Fe[S] : 0) + (U ? cinB[U].e + C.g[popc(U)].e : 0);
            E = max(E, TE[S]);
        }
        M j = M(0);
#pragma unroll
        for (int S = 0; S < D; ++S) {
            const int U = (D - 1) ^ S;
            const M f = S ? fm[((S - 1) * V + V - 1) * T + tid] : M(1);
            const M b = U ? cinB[U].m * C.g[popc(U)].hi : M(1);
            j = fma(xldexp(f, TE[S] - E), b, j);
        }
        at(V - 1, jlog(j, E));
    }
}

// log J_j at the thread's positions (both scans + combine, handed to at(v, .));
// rows 0 .. l-2 of
// pm/pe are the l - 1 marginals other than j, in any order (the subset
// dynamic program is symmetric in them).  The forward states wait in LDS
// (fm, fe) while the backward scan runs.
template <int L, int V, typename M, typename At>
__device__ __forceinline__ void bproduct(const M (&pm)[L][V], const int (&pe)[L], const FastConst<M, L, V> &C,
                                         XF<M> *xw, M *fm, int *fe, int tid, int T, int lane, int wave, int nw,
                                         At &&at)
{
    constexpr int n = L - 1;
    constexpr int D = 1 << n;
    {
        M Fm[D][V];
        int Fe[D];
        XF<M> cinF[D];
        bscan<L, V, M, true>(pm, pe, Fm, Fe, cinF, C, xw, 0, lane, wave, nw);
#pragma unroll
        for (int S = 1; S < D; ++S) {
            fe[(S - 1) * T + tid] = Fe[S];
#pragma unroll
            for (int v = 0; v < V; ++v) fm[((S - 1) * V + v) * T + tid] = Fm[S][v];
        }
    }
    M Bm[D][V];
    int Be[D];
    XF<M> cinB[D];
    bscan<L, V, M, false>(pm, pe, Bm, Be, cinB, C, xw, n, lane, wave, nw);
    bcombine<L, V, M>(fm, fe, tid, T, Bm, Be, cinB, C, at);
}

// One term u |exp(d) - 1| of the stopping estimate (d = a_old - a_new at a
// position, u = exp(log_u) there), in FP32: it only decides when the FP64
// residual is computed.  |d| <= 1/16: the cubic Taylor polynomial (relative
// error below 1e-5); beyond, the polynomial is a lower bound for d > 0 and is
// capped at 1 for d < 0 (where |exp(d) - 1| < 1).
__device__ __forceinline__ double est_term(double lu, double d)
{
    const float u = __builtin_amdgcn_exp2f((float)(lu * LOG2E));
    const float x = (float)d;
    float t = fabsf(x * fmaf(x, fmaf(x, 1.0f / 6.0f, 0.5f), 1.0f));
    if (x < 0.0f) t = fminf(t, 1.0f);
    return (double)(u * t);
}

// Shared memory of one workgroup.
template <int L, int V, typename M>
struct FastShared {
    static constexpr int T = fast_threads(L, sizeof(M) == 4 ? 1 : 0);
    static constexpr int D1 = (1 << (L - 1)) - 1;
    FastConst<M, L, V> c;
    XF<M> xw[2 * FAST_MAXW * (1 << (L - 1))];
    double red[FAST_MAXW];
    int fl[2 * FAST_MAXW];
    M fm[D1 * V * T];  // forward states during the backward scan
    int fe[D1 * T];
};

template <typename M, int L, int V>
__device__ __forceinline__ bool bf_fits(int row_spread, int decay_bits)
{
    return bf_fits_range(sizeof(M) == 4 ? 1 : 0, L, V, row_spread, decay_bits);
}

// Block-floating-point row at the thread's positions from the potentials in memory.
template <typename M, int V>
__device__ __forceinline__ int load_row(const double *__restrict__ a, long N, long p0, M (&m)[V], int &e)
{
    double x[V];
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = (p0 + v < N) ? gld(&a[p0 + v]) : -INFINITY;
    return bf_row<M, V>(x, m, e);
}

// Decay of the discount factors per position, in bits.
template <typename M, int L, int V>
__device__ __forceinline__ int decay_bits(const FastConst<M, L, V> &C)
{
    int dec = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) dec = max(dec, 1 - C.g[k].e);
    return dec;
}

// Sweeps of one instance by one workgroup (N <= blockDim.x * V), resumed from
// the progress record Tr; the potentials live in memory (FP64).  Runs the
// Gauss-Seidel updates (Alg. 1 update lines, products in precision M) until a
// residual check is due -- every check_every sweeps if > 0, after the last
// sweep, or once the estimate est (the marginal errors seen by the updates of
// one sweep, before each update) falls below tol * f -- and hands the instance
// to the check kernel, or until the launch's sweep budget (o.budget, if > 0) is
// spent.  A product whose values would span too wide an exponent range inside a
// thread hands it to the extended-range solver instead, which resumes at that
// marginal.
template <int L, int V, typename M>
__device__ __forceinline__ void fast_sweeps(const Inst *__restrict__ I, const Ptrs P, const RunOpts o,
                                            Track *__restrict__ Tr, FastShared<L, V, M> &sh)
{
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront-uniform
    const long N = I->N;
    const int flags = o.flags | P.flags;
    const long itr_max = P.itr_cap > 0 ? P.itr_cap : o.itr_max;
    const long p0 = (long)tid * V;
    double *__restrict__ pa = P.a;
    const double *__restrict__ plu = P.log_u;
    const double f = Tr->f;
    long it = Tr->it;

    fast_consts<M, L, V>(sh.c, I->hoe, tid, blockDim.x);
    if (it == 0 && !(flags & F_WARM)) {
        // phi = 1/N (Alg. 1 initialisation)
        const double a0 = -log((double)N);
        for (long p = tid; p < (long)L * N; p += blockDim.x) pa[p] = a0;
    }
    __syncthreads();
    const int dec = decay_bits(sh.c);

    // rows as a ring: while marginal j is updated, slot s holds marginal (j + 1 + s) mod l
    M pm[L][V];
    int pe[L], sp[L];
#pragma unroll
    for (int s = 0; s < L; ++s) sp[s] = load_row<M, V>(pa + (long)((1 + s) % L) * N, N, p0, pm[s], pe[s]);

    int state = TS_DONE, phase = 0, j_stop = 0, status = ST_OK;
    double est = 0.0, est_mid = Tr->est_mid;
    int done = 0;  // sweeps of this launch
    while (it < itr_max) {
        ++it;
        est = 0.0;
        j_stop = L;
#pragma unroll 1
        for (int j = 0; j < L; ++j) {
            int s = 0;
#pragma unroll
            for (int q = 0; q < L - 1; ++q) s = max(s, sp[q]);
            if (block_any(!bf_fits<M, L, V>(s, dec), sh.fl, phase, lane, wave, nw)) {
                j_stop = j;
                break;
            }
            double an[V];
            double *__restrict__ aj = pa + (long)j * N + p0;
            const double *__restrict__ luj = plu + (long)j * N + p0;
            // the update's operands are loaded before the scans (global loads: they land
            // while the scans run, and LDS reads never wait for them)
            double luv[V], aov[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const bool in = p0 + v < N;
                luv[v] = in ? gld(&luj[v]) : -INFINITY;
                aov[v] = in ? gld(&aj[v]) : 0.0;
            }
            bproduct<L, V, M>(pm, pe, sh.c, sh.xw, sh.fm, sh.fe, tid, FastShared<L, V, M>::T, lane, wave, nw,
                              [&](int v, double lj) {
                                  const bool in = p0 + v < N;
                                  const double lu = luv[v];
                                  double x = lu - lj;
                                  if (lu > -INFINITY) {
                                      if (j < L - 1) est += est_term(lu, aov[v] - x);
                                  } else {
                                      x = -INFINITY;
                                  }
                                  if (in) gst(&aj[v], x);
                                  an[v] = x;
                              });
            // new row j into the last slot, then rotate the ring by one
            sp[L - 1] = bf_row<M, V>(an, pm[L - 1], pe[L - 1]);
            M tm[V];
#pragma unroll
            for (int v = 0; v < V; ++v) tm[v] = pm[0][v];
            const int te = pe[0], ts = sp[0];
#pragma unroll
            for (int q = 0; q < L - 1; ++q) {
#pragma unroll
                for (int v = 0; v < V; ++v) pm[q][v] = pm[q + 1][v];
                pe[q] = pe[q + 1];
                sp[q] = sp[q + 1];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) pm[L - 1][v] = tm[v];
            pe[L - 1] = te;
            sp[L - 1] = ts;
        }
        if (j_stop < L) {
            state = TS_ROBUST;
            if (j_stop == 0) --it;  // the sweep has not started: the solver begins it afresh
            break;
        }
        est = block_sum(est, sh.red, lane, wave, nw);
        if (!(est == est)) {
            status = ST_NUMERIC;
            state = TS_DONE;
            break;
        }
        const bool chk = !(flags & F_NO_CHECK) && ((o.check_every > 0 && it % o.check_every == 0) ||
                                                    it == itr_max || (o.tol >= 0.0 && est <= o.tol * f));
        if (chk) {
            state = TS_CHECK;
            break;
        }
        // a sweep budget pauses the instance without a check (the next launch
        // goes on from the same iterate)
        ++done;
        if (o.budget > 0) {
            if (2 * done == o.budget) est_mid = est;
            if (done >= o.budget) {
                state = TS_SWEEP;
                break;
            }
        }
    }
    if (tid == 0) {
        Tr->it = it;
        Tr->est = est;
        Tr->est_mid = est_mid;
        Tr->state = state;
        Tr->j0 = state == TS_ROBUST ? j_stop : 0;
        if (state == TS_DONE) Tr->status = status;
    }
}

// FP64 residual of one instance by one workgroup (Alg. 1 Res line):
// sum over j < l-1 of sum_y |phi_j(y) J_j(y) - u_j(y)|, then the stopping
// decision for the check the sweep kernel asked for.
template <int L, int V>
__device__ __forceinline__ void fast_check(const Inst *__restrict__ I, const Ptrs P, const RunOpts o,
                                           Track *__restrict__ Tr, FastShared<L, V, double> &sh)
{
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront-uniform
    const long N = I->N;
    const long itr_max = P.itr_cap > 0 ? P.itr_cap : o.itr_max;
    const long p0 = (long)tid * V;
    const double *__restrict__ pa = P.a;
    const double *__restrict__ plu = P.log_u;

    fast_consts<double, L, V>(sh.c, I->hoe, tid, blockDim.x);
    __syncthreads();
    const int dec = decay_bits(sh.c);
    // slot s holds marginal (j + 1 + s) mod l while J_j is formed
    double pm[L][V];
    int pe[L], sp[L];
#pragma unroll
    for (int s = 0; s < L; ++s) sp[s] = load_row<double, V>(pa + (long)((1 + s) % L) * N, N, p0, pm[s], pe[s]);
    int phase = 0;
    bool wide = false;
    double r = 0.0;
#pragma unroll 1
    for (int j = 0; j < L - 1; ++j) {
        int s = 0;
#pragma unroll
        for (int q = 0; q < L - 1; ++q) s = max(s, sp[q]);
        if (block_any(!bf_fits<double, L, V>(s, dec), sh.fl, phase, lane, wave, nw)) {
            wide = true;
            break;
        }
        double luv[V], aov[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool in = p0 + v < N;
            luv[v] = in ? gld(&plu[(long)j * N + p0 + v]) : -INFINITY;
            aov[v] = in ? gld(&pa[(long)j * N + p0 + v]) : 0.0;
        }
        bproduct<L, V, double>(pm, pe, sh.c, sh.xw, sh.fm, sh.fe, tid, FastShared<L, V, double>::T, lane, wave, nw,
                               [&](int v, double lj) {
                                   if (p0 + v < N) {
                                       const double lu = luv[v];
                                       if (lu > -INFINITY) r += fabs(exp(aov[v] + lj) - exp(lu));
                                   }
                               });
        // rotate the ring by one (the rows do not change)
        double tm[V];
#pragma unroll
        for (int v = 0; v < V; ++v) tm[v] = pm[0][v];
        const int te = pe[0], ts = sp[0];
#pragma unroll
        for (int q = 0; q < L - 1; ++q) {
#pragma unroll
            for (int v = 0; v < V; ++v) pm[q][v] = pm[q + 1][v];
            pe[q] = pe[q + 1];
            sp[q] = sp[q + 1];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) pm[L - 1][v] = tm[v];
        pe[L - 1] = te;
        sp[L - 1] = ts;
    }
    const double res = block_sum(r, sh.red, lane, wave, nw);
    if (tid == 0) {
        if (wide) {
            // the extended-range solver takes over at the start of the next sweep,
            // checking right away
            Tr->state = TS_ROBUST;
            Tr->j0 = L;
        } else {
            const long it = Tr->it;
            Tr->res = res;
            Tr->checked = 1;
            if (!(res == res)) {
                Tr->state = TS_DONE;
                Tr->status = ST_NUMERIC;
            } else if (res <= o.tol || it >= itr_max) {
                Tr->state = TS_DONE;
                Tr->status = ST_OK;
            } else {
                if (o.tol >= 0.0 && Tr->est <= o.tol * Tr->f) Tr->f *= 0.5;
                Tr->state = TS_SWEEP;
            }
        }
    }
}

}  // namespace mmot
