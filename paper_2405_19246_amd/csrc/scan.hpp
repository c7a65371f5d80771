// The O(N) tensor-vector product of the L1 Gibbs kernel on one wavefront.
//
// Gap form.  For indices i_1..i_l let m_x = #{q : i_q <= x}.  Every pair p<q
// is separated by |i_p - i_q| grid gaps and gap x separates m_x (l - m_x)
// pairs, so K = lambda^{sum_{p<q}|i_p-i_q|} = prod_x g(m_x), g(m) = lambda^{m(l-m)}.
// (For l = 3 this is why every coefficient of FTVP-1, Sec. 3.1, is lambda^2.)
// The paper removes the absolute values by splitting into l! ordering classes
// (Sec. 3 Eq. D_p; Sec. 4.2); merging the classes that share a prefix leaves a
// dynamic program over which of the summed marginals lie left of x.
//
// For the product J_j(y) = sum_{i_q, q != j; i_j = y} K prod_{q != j} phi_q(i_q)
// let R be the l - 1 marginals other than j (bit r of a mask is R's r-th
// member) and S a subset of R:
//   forward   F_x(S) = g(|S|) F_{x-1}(S) + sum_{0 != T subset S} g(|S\T|) F_{x-1}(S\T) prod_{q in T} phi_q(x)
//   backward  B_x(U) = g(|U|) B_{x+1}(U) + (the same inflow from B_{x+1})
//   combine   J_j(y) = sum_S F_y(S) g(|R\S|) B_{y+1}(R\S)
// with F(empty) = B(empty) = 1 and zero states beyond both ends.  For l = 3 the
// three forward states are the prefix sums of Sec. 3.1 (P_{k,1}, P_{k,4}, and
// J_{k,1} + J_{k,2} as one scan), the backward ones its suffix sums.
//
// Parallel form.  A wavefront owns a chunk of 64 V consecutive positions, lane
// L the V positions L V .. L V + V - 1.  The states are solved one level
// |S| = 1, 2, .., l - 1 at a time: at level k each state is a scalar
// discounted recurrence v_x = g(k) v_{x-1} + in_x whose inflow only involves
// final lower-level states, so it is scanned with the associative operator
// (v1 over w1 positions) . (v2) = g^{w2} v1 + v2: sequentially over the lane's
// V positions, Kogge-Stone across the 64 lanes (shuffles), and the chunk's
// carry-in from the previous chunk added in closed form g^{t+1} c.  Chunks are
// walked in order; the backward direction mirrors lanes and positions.
#pragma once
#include <type_traits>
#include "xf.hpp"

namespace mmot {

__device__ __forceinline__ constexpr int popc(int x) { return __builtin_popcount(x); }

// Level-synchronous scan of one chunk in one direction.
//   phi[r][v]  scaling factor of R's r-th member at the lane's v-th position
//   st[S][v]   out: state S at each position (S = 0 unused)
//   cin[S]     out: state S at the position before the lane's first one (scan order)
//   carry[S]   in: state at the position before the chunk; out: at the chunk's last one
//   lanep[k]   g(k)^(V * scan lane)
template <int L, int V, typename E, bool FWD>
__device__ __forceinline__ void level_scan(const XF<typename ET<E>::MT> (&phi)[L - 1][V], E (&st)[1 << (L - 1)][V],
                                           E (&cin)[1 << (L - 1)], E (&carry)[1 << (L - 1)],
                                           const Disc<typename ET<E>::MT> *__restrict__ K,
                                           const XG<typename ET<E>::MT> (&lanep)[L], double slf, int sl)
{
    using T_ = ET<E>;
    using M = typename T_::MT;
    constexpr int n = L - 1;
    constexpr int D = 1 << n;

#pragma unroll
    for (int k = 1; k <= n; ++k) {
        E loc[D][V];
#pragma unroll
        for (int t = 0; t < V; ++t) {
            const int v = FWD ? t : V - 1 - t;
            const int vp = FWD ? v - 1 : v + 1;
            // lower-level states at the previous position, times their gap factor
            E G[D];
#pragma unroll
            for (int S = 1; S < D; ++S) {
                if (popc(S) < k) {
                    const E prev = (t == 0) ? cin[S] : st[S][vp];
                    G[S] = T_::disc(prev, K->g1[popc(S)], K->ck[popc(S)]);
                }
            }
            // products of scaling factors of the members placed at this position
            XF<M> pp[D];
#pragma unroll
            for (int T = 1; T < D; ++T) {
                if (popc(T) <= k) {
                    const int low = __builtin_ctz(T);
                    pp[T] = (T == (1 << low)) ? phi[low][v] : xmul(pp[T & (T - 1)], phi[low][v]);
                }
            }
#pragma unroll
            for (int S = 1; S < D; ++S) {
                if (popc(S) != k) continue;
                E in = T_::zero();
                bool first = true;
#pragma unroll
                for (int T = 1; T < D; ++T) {
                    if ((T & S) != T) continue;
                    const E term = (T == S) ? E(T_::scale(T_::one(), pp[T])) : T_::scale(G[S ^ T], pp[T]);
                    in = first ? term : T_::add(in, term);
                    first = false;
                }
                loc[S][v] = (t == 0) ? in : T_::add(T_::disc(loc[S][vp], K->g1[k], K->ck[k]), in);
            }
        }
        // carries of level k across lanes and from the previous chunk
#pragma unroll
        for (int S = 1; S < D; ++S) {
            if (popc(S) != k) continue;
            E incl = loc[S][FWD ? V - 1 : 0];
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const int d = 1 << s;
                const E o = FWD ? T_::shup(incl, d) : T_::shdn(incl, d);
                if (sl >= d) incl = T_::add(incl, T_::disc(o, K->gstep[k][s], double(V * d) * K->ck[k]));
            }
            const E ex = FWD ? T_::shup(incl, 1) : T_::shdn(incl, 1);
            E c = T_::disc(carry[S], lanep[k], double(V) * slf * K->ck[k]);
            if (sl > 0) c = T_::add(ex, c);
            cin[S] = c;
#pragma unroll
            for (int t = 0; t < V; ++t) {
                const int v = FWD ? t : V - 1 - t;
                st[S][v] = T_::add(loc[S][v], T_::disc(c, K->gfix[k][t], double(t + 1) * K->ck[k]));
            }
            carry[S] = T_::rl(st[S][FWD ? V - 1 : 0], FWD ? WAVE - 1 : 0);
        }
    }
}

// ---- FP32 scans in block floating point -------------------------------------
//
// Same recurrences as level_scan, but inside one lane the V values of a row or
// of a state share one exponent: the inflow sums and the in-lane discounted
// scan are plain FP32 FMAs on mantissas, and extended-range values are only
// formed where a lane hands its aggregate on (Kogge-Stone across lanes, the
// chunk carry).  Exact up to FP32 rounding while the values of one lane span
// less exponent range than FP32 holds next to each other (bf_fits_range).
// Discount factors keep their hi + lo mantissa everywhere, as in level_scan.

// Plain hi + lo value of a discount factor held as an extended-range one.
__device__ __forceinline__ GV<float> gv_of(const XG<float> &g) { return {xldexp(g.hi, g.e), xldexp(g.lo, g.e)}; }

// Decay of the discount factors per grid position, in bits.
template <int L>
__device__ __forceinline__ int disc_decay_bits(const Disc<float> *__restrict__ K)
{
    int dec = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) dec = max(dec, 1 - K->g1[k].e);
    return dec;
}

//   pm/pe  rows of R's members at the lane's positions: mantissas relative to 2^pe[r]
//   Fm/Fe  out: states, mantissas relative to 2^Fe[S]; the largest |Fm[S][.]| is
//          in [1/4, 2], or all are 0 and Fe[S] is the zero exponent
//   cin    out: state at the position before the lane's first one (scan order)
//   carry  in: state at the position before the chunk; out: at the chunk's last one
//   lanep  g(k)^(V * scan lane)
template <int L, int V, bool FWD>
__device__ __forceinline__ void level_scan_bf(const float (&pm)[L - 1][V], const int (&pe)[L - 1],
                                              float (&Fm)[1 << (L - 1)][V], int (&Fe)[1 << (L - 1)],
                                              XF<float> (&cin)[1 << (L - 1)], XF<float> (&carry)[1 << (L - 1)],
                                              const Disc<float> *__restrict__ K, const XG<float> (&lanep)[L], int sl)
{
    constexpr int n = L - 1;
    constexpr int D = 1 << n;

#pragma unroll
    for (int k = 1; k <= n; ++k) {
        const GV<float> gk = gv_of(K->g1[k]);
        float loc[D][V];
        int Ein[D];
#pragma unroll
        for (int S = 1; S < D; ++S) {
            if (popc(S) != k) continue;
            // exponent bound of each inflow term T (members placed at this position)
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
                if (Sp) et += Fe[Sp] + K->g1[popc(Sp)].e;
                Et[T] = et;
                E = max(E, et);
            }
            // its coefficient g(|S\T|) 2^(Et - E), hi + lo
            float ch[D], cl[D];
#pragma unroll
            for (int T = 1; T < D; ++T) {
                if ((T & S) != T) continue;
                const int Sp = S ^ T;
                ch[T] = xldexp(Sp ? K->g1[popc(Sp)].hi : 1.0f, Et[T] - E);
                cl[T] = Sp ? xldexp(K->g1[popc(Sp)].lo, Et[T] - E) : 0.0f;
            }
            // lower-level states before the lane's first position, as mantissas
            float cm[D];
#pragma unroll
            for (int Sp = 1; Sp < D; ++Sp)
                if ((Sp & S) == Sp && Sp != S) cm[Sp] = xldexp(cin[Sp].m, cin[Sp].e - Fe[Sp]);
            float mx = 0.0f;
#pragma unroll
            for (int t = 0; t < V; ++t) {
                const int v = FWD ? t : V - 1 - t;
                const int vp = FWD ? v - 1 : v + 1;
                float in = 0.0f;
#pragma unroll
                for (int T = 1; T < D; ++T) {
                    if ((T & S) != T) continue;
                    float pp = 1.0f;
#pragma unroll
                    for (int r = 0; r < n; ++r)
                        if (T & (1 << r)) pp *= pm[r][v];
                    const int Sp = S ^ T;
                    if (Sp == 0) {
                        in = fmaf(ch[T], pp, in);
                    } else {
                        const float prev = (t == 0) ? cm[Sp] : Fm[Sp][vp];
                        in = fmaf(fmaf(cl[T], prev, ch[T] * prev), pp, in);
                    }
                }
                loc[S][v] = (t == 0) ? in : gmul(gk, loc[S][vp], in);
                mx = fmaxf(mx, loc[S][v]);
            }
            // tighten the exponent to the values actually there (all zero: zero exponent)
            Ein[S] = (mx == 0.0f) ? XF_ZERO_E : E;
            if (mx != 0.0f) {
                const int d = xexpo(mx);
                Ein[S] += d;
#pragma unroll
                for (int v = 0; v < V; ++v) loc[S][v] = xldexp(loc[S][v], -d);
            }
        }
        // carries of level k across lanes and from the previous chunk
#pragma unroll
        for (int S = 1; S < D; ++S) {
            if (popc(S) != k) continue;
            XF<float> incl = xnorm(XF<float>{loc[S][FWD ? V - 1 : 0], Ein[S]});
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const int d = 1 << s;
                XF<float> o;
                if (FWD) o = {__shfl_up(incl.m, d), __shfl_up(incl.e, d)};
                else o = {__shfl_down(incl.m, d), __shfl_down(incl.e, d)};
                if (sl >= d) incl = xadd(incl, xmulg(o, K->gstep[k][s]));
            }
            XF<float> ex;
            if (FWD) ex = {__shfl_up(incl.m, 1), __shfl_up(incl.e, 1)};
            else ex = {__shfl_down(incl.m, 1), __shfl_down(incl.e, 1)};
            XF<float> c = xmulg(carry[S], lanep[k]);
            if (sl > 0) c = xadd(ex, c);
            c = xnorm(c);
            cin[S] = c;
            // block exponent of the state: the larger of the local part and the carry part
            const int ec = (c.m == 0.0f) ? XF_ZERO_E : c.e + K->g1[k].e;
            const int F = max(Ein[S], ec);
            Fe[S] = F;
            const float sc = xldexp(1.0f, Ein[S] - F);
            const float cmk = xldexp(c.m, c.e - F);
#pragma unroll
            for (int t = 0; t < V; ++t) {
                const int v = FWD ? t : V - 1 - t;
                Fm[S][v] = gmul(gv_of(K->gfix[k][t]), cmk, loc[S][v] * sc);
            }
            const XF<float> last = xnorm(XF<float>{Fm[S][FWD ? V - 1 : 0], F});
            carry[S] = {rlane(last.m, FWD ? WAVE - 1 : 0), rlane(last.e, FWD ? WAVE - 1 : 0)};
        }
    }
}

// log J_j at the lane's positions from both scans of a chunk (natural log, FP64):
// J(y) = sum_S F_y(S) g(|R\S|) B_{y+1}(R\S).
template <int L, int V>
__device__ __forceinline__ void combine_bf(const float (&Fm)[1 << (L - 1)][V], const int (&Fe)[1 << (L - 1)],
                                           const float (&Bm)[1 << (L - 1)][V], const int (&Be)[1 << (L - 1)],
                                           const XF<float> (&cinB)[1 << (L - 1)], const Disc<float> *__restrict__ K,
                                           double (&lj)[V])
{
    constexpr int D = 1 << (L - 1);
    if (V > 1) {
        // positions v < V-1: the next position's backward state is in this lane
        int TE[D];
        int E = XF_ZERO_E;
#pragma unroll
        for (int S = 0; S < D; ++S) {
            const int U = (D - 1) ^ S;
            TE[S] = (S ? Fe[S] : 0) + (U ? Be[U] + K->g1[popc(U)].e : 0);
            E = max(E, TE[S]);
        }
        float ch[D], cl[D];
#pragma unroll
        for (int S = 0; S < D; ++S) {
            const int U = (D - 1) ^ S;
            ch[S] = xldexp(U ? K->g1[popc(U)].hi : 1.0f, TE[S] - E);
            cl[S] = U ? xldexp(K->g1[popc(U)].lo, TE[S] - E) : 0.0f;
        }
#pragma unroll
        for (int v = 0; v < V - 1; ++v) {
            float jv = 0.0f;
#pragma unroll
            for (int S = 0; S < D; ++S) {
                const int U = (D - 1) ^ S;
                const float t = (S ? Fm[S][v] : 1.0f) * (U ? Bm[U][v + 1] : 1.0f);
                jv = fmaf(ch[S], t, fmaf(cl[S], t, jv));
            }
            lj[v] = (jv == 0.0f) ? -INFINITY : xto_log(XF<float>{jv, E});
        }
    }
    // the lane's last position: the next position's backward state is its carry-in
    int TE[D];
    int E = XF_ZERO_E;
#pragma unroll
    for (int S = 0; S < D; ++S) {
        const int U = (D - 1) ^ S;
        TE[S] = (S ? Fe[S] : 0) + (U ? cinB[U].e + K->g1[popc(U)].e : 0);
        E = max(E, TE[S]);
    }
    float jv = 0.0f;
#pragma unroll
    for (int S = 0; S < D; ++S) {
        const int U = (D - 1) ^ S;
        const float f = xldexp(S ? Fm[S][V - 1] : 1.0f, TE[S] - E);
        const float b = U ? fmaf(cinB[U].m, K->g1[popc(U)].lo, cinB[U].m * K->g1[popc(U)].hi) : 1.0f;
        jv = fmaf(f, b, jv);
    }
    lj[V - 1] = (jv == 0.0f) ? -INFINITY : xto_log(XF<float>{jv, E});
}

// Result.status values set on the device.
static constexpr int ST_OK = 0;
static constexpr int ST_NUMERIC = -3;
static constexpr int ST_NOT_CONVERGED = -4;

// Discount table of the update pass in mantissa type M.
template <int L, typename M>
__device__ __forceinline__ const Disc<M> *upd_disc(const Inst *I)
{
    if constexpr (std::is_same<M, float>::value)
        return &I->d32;
    else
        return &I->d64;
}


template <typename E>
__device__ __forceinline__ void store_elem(void *base, long idx, int lane_ok, E x)
{
    if (lane_ok) gst_e(reinterpret_cast<E *>(base) + idx, x);
}

// Wave-wide FP64 sum, the same value in every lane.  (A butterfly leaves each
// lane with its own summation order, and a stopping test on per-lane sums
// could split the wavefront; lane 0's sum is broadcast.)
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    return rlane(x, 0);
}

__device__ __forceinline__ XF<double> wave_sum_xf(XF<double> x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const XF<double> o = {__shfl_xor(x.m, d), __shfl_xor(x.e, d)};
        x = xadd(x, o);
    }
    return {rlane(x.m, 0), rlane(x.e, 0)};
}

// What a product, update or check pass does with log J_j at position p; returns
// the position's contribution to the pass's sum.
//   P_PRODUCT: out[p] = log J_j(p)
//   P_UPDATE:  a_j(p) = log u_j(p) - log J_j(p); returns u_j(p) |exp(a_old - a_new) - 1|
//   P_CHECK:   returns |exp(a_j(p) + log J_j(p)) - u_j(p)|
template <int MODE>
__device__ __forceinline__ double finish_lj(double lj, int j, long N, long p, double *__restrict__ a,
                                            const double *__restrict__ log_u, double *__restrict__ out)
{
    if constexpr (MODE == P_PRODUCT) {
        out[p] = lj;
        return 0.0;
    } else if constexpr (MODE == P_UPDATE) {
        const double lu = log_u[(long)j * N + p];
        const double ao = a[(long)j * N + p];
        const double an = lu > -INFINITY ? lu - lj : -INFINITY;
        a[(long)j * N + p] = an;
        return lu > -INFINITY ? exp(lu) * fabs(expm1(ao - an)) : 0.0;
    } else {
        const double lu = log_u[(long)j * N + p];
        return fabs(exp(a[(long)j * N + p] + lj) - exp(lu));
    }
}

// finish_lj with a_j(p) (ao) and log u_j(p) (lu) already loaded; stores through
// global-address-space pointers.
template <int MODE>
__device__ __forceinline__ double finish_pre(double lj, double lu, double ao, int j, long N, long p,
                                             double *__restrict__ a, double *__restrict__ out)
{
    if constexpr (MODE == P_PRODUCT) {
        gst(&out[p], lj);
        return 0.0;
    } else if constexpr (MODE == P_UPDATE) {
        const double an = lu > -INFINITY ? lu - lj : -INFINITY;
        gst(&a[(long)j * N + p], an);
        return lu > -INFINITY ? exp(lu) * fabs(expm1(ao - an)) : 0.0;
    } else {
        return fabs(exp(ao + lj) - exp(lu));
    }
}

// One marginal pass over an instance on one wavefront.
//   P_PRODUCT:   out[y] = log J_j(y)
//   P_UPDATE:    a_j(y) = log u_j(y) - log J_j(y)           (Gauss-Seidel step);
//                returns sum_y u_j(y) |exp(a_j,old(y) - a_j(y)) - 1|, the
//                marginal error before the step (FP64)
//   P_CHECK:     returns sum_y |exp(a_j(y) + log J_j(y)) - u_j(y)|  (FP64)
//   P_OBJECTIVE: returns h sum_y phi_j(y) ((C o K) x_{q != j} phi_q)(y) / h ... = W_eps
// a: [l][N] potentials; scratch: checkpoint space for ceil(N / 64V) (D - 1) elements.
template <int L, int V, typename E, int MODE>
__device__ double marginal_pass(const Inst *__restrict__ I, const Disc<typename ET<E>::MT> *__restrict__ K, int j,
                                double *__restrict__ a, const double *__restrict__ log_u, double *__restrict__ out,
                                void *__restrict__ scratch, int lane)
{
    using T_ = ET<E>;
    using M = typename T_::MT;
    constexpr int n = L - 1;
    constexpr int D = 1 << n;
    constexpr int CH = WAVE * V;
    const long N = I->N;
    const long C = (N + CH - 1) / CH;

    XG<M> lanepF[L], lanepB[L];
    const int slF = lane, slB = WAVE - 1 - lane;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        lanepF[k] = xg_from_log<M>(K->lgV[k] * (double)slF);
        lanepB[k] = xg_from_log<M>(K->lgV[k] * (double)slB);
    }

    int items[n];
#pragma unroll
    for (int r = 0; r < n; ++r) items[r] = (r < j) ? r : r + 1;

    // FP32 products and updates take the block-floating-point scans for every
    // chunk whose rows fit them (wavefront-uniform choice), the extended-range
    // scans otherwise; both keep the chunk carries in extended range.
    constexpr bool BF = std::is_same<E, XF<float>>::value && (MODE == P_PRODUCT || MODE == P_UPDATE);
    constexpr bool PRE = std::is_same<M, double>::value;
    auto load_a = [&](long c, double(&av)[n][V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const long p = c * CH + (long)lane * V + v;
#pragma unroll
            for (int r = 0; r < n; ++r) av[r][v] = (p < N) ? gld(&a[(long)items[r] * N + p]) : -INFINITY;
        }
    };
    auto to_phi = [&](const double(&av)[n][V], XF<M>(&phi)[n][V]) {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int r = 0; r < n; ++r) phi[r][v] = xfrom_log<M>(av[r][v]);
    };
    // rows in block floating point; true if every lane's values fit
    int dec = 0;
    if constexpr (BF) dec = disc_decay_bits<L>(K);
    auto to_bf = [&](const double(&av)[n][V], float(&pm)[n][V], int(&pe)[n]) {
        int sp = 0;
#pragma unroll
        for (int r = 0; r < n; ++r) sp = max(sp, bf_row<float, V>(av[r], pm[r], pe[r]));
        return __ballot(!bf_fits_range(1, L, V, sp, dec)) == 0;
    };

    E carryF[D], carryB[D];
#pragma unroll
    for (int S = 0; S < D; ++S) {
        carryF[S] = T_::zero();
        carryB[S] = T_::zero();
    }
    // forward sweep over chunks, saving each chunk's carry-in (only if >1 chunk)
    if (C > 1) {
        for (long c = 0; c < C; ++c) {
            double av[n][V];
            load_a(c, av);
#pragma unroll
            for (int S = 1; S < D; ++S) store_elem(scratch, c * (D - 1) + (S - 1), lane == 0, carryF[S]);
            if constexpr (BF) {
                float pm[n][V];
                int pe[n];
                if (to_bf(av, pm, pe)) {
                    float Fm[D][V];
                    int Fe[D];
                    XF<float> cin[D];
                    level_scan_bf<L, V, true>(pm, pe, Fm, Fe, cin, carryF, K, lanepF, slF);
                    continue;
                }
            }
            XF<M> phi[n][V];
            to_phi(av, phi);
            E st[D][V], cin[D];
            level_scan<L, V, E, true>(phi, st, cin, carryF, K, lanepF, (double)slF, slF);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }

    double acc = 0.0;
    XF<double> accx = xzero<double>();
    for (long c = C - 1; c >= 0; --c) {
        double av[n][V];
        load_a(c, av);
        // the epilogue's operands (a_j, log u_j at the chunk's positions): with FP64
        // mantissas loaded before the scans, so that they have landed when the
        // combine needs them; with FP32 ones, whose scans hold more state per
        // register budget, at the combine (held across the scans they spill)
        double ajc[V], luc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const long p = c * CH + (long)lane * V + v;
            const bool in = p < N;
            if constexpr (PRE) {
                ajc[v] = (MODE != P_PRODUCT && in) ? gld(&a[(long)j * N + p]) : 0.0;
                luc[v] = ((MODE == P_UPDATE || MODE == P_CHECK) && in) ? gld(&log_u[(long)j * N + p]) : 0.0;
            }
        }
        if (C > 1) {
#pragma unroll
            for (int S = 1; S < D; ++S) carryF[S] = gld_e(reinterpret_cast<const E *>(scratch) + c * (D - 1) + (S - 1));
        }
        if constexpr (BF) {
            float pm[n][V];
            int pe[n];
            if (to_bf(av, pm, pe)) {
                float Fm[D][V], Bm[D][V];
                int Fe[D], Be[D];
                XF<float> cinF[D], cinB[D];
                level_scan_bf<L, V, true>(pm, pe, Fm, Fe, cinF, carryF, K, lanepF, slF);
                level_scan_bf<L, V, false>(pm, pe, Bm, Be, cinB, carryB, K, lanepB, slB);
                double ljv[V];
                combine_bf<L, V>(Fm, Fe, Bm, Be, cinB, K, ljv);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const long p = c * CH + (long)lane * V + v;
                    if (p < N) acc += PRE ? finish_pre<MODE>(ljv[v], luc[v], ajc[v], j, N, p, a, out)
                                          : finish_lj<MODE>(ljv[v], j, N, p, a, log_u, out);
                }
                continue;
            }
        }
        XF<M> phi[n][V];
        to_phi(av, phi);
        E F[D][V], cinF[D];
        level_scan<L, V, E, true>(phi, F, cinF, carryF, K, lanepF, (double)slF, slF);
        E B[D][V], cinB[D];
        level_scan<L, V, E, false>(phi, B, cinB, carryB, K, lanepB, (double)slB, slB);

#pragma unroll
        for (int v = 0; v < V; ++v) {
            const long p = c * CH + (long)lane * V + v;
            E J = T_::zero();
#pragma unroll
            for (int S = 0; S < D; ++S) {
                const int U = (D - 1) ^ S;
                const E f = (S == 0) ? T_::one() : F[S][v];
                E hb;
                if (U == 0) {
                    hb = T_::one();
                } else {
                    const E bn = (v < V - 1) ? B[U][v + 1] : cinB[U];
                    hb = T_::disc(bn, K->g1[popc(U)], K->ck[popc(U)]);
                }
                J = (S == 0) ? T_::prod(f, hb) : T_::add(J, T_::prod(f, hb));
            }
            if (p < N) {
                if constexpr (MODE == P_OBJECTIVE) {
                    const XF<double> ph = xfrom_log<double>(ajc[v]);
                    accx = xadd(accx, xmul(ph, J.w));
                } else {
                    acc += PRE ? finish_pre<MODE>(xto_log(J), luc[v], ajc[v], j, N, p, a, out)
                               : finish_lj<MODE>(xto_log(J), j, N, p, a, log_u, out);
                }
            }
        }
    }
    if constexpr (MODE == P_UPDATE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        return wave_sum(acc);
    }
    if constexpr (MODE == P_CHECK) return wave_sum(acc);
    if constexpr (MODE == P_OBJECTIVE) return I->h * xto_double(wave_sum_xf(accx));
    return 0.0;
}

}  // namespace mmot
