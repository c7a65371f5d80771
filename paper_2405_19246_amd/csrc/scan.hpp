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

enum PassMode { P_PRODUCT = 0, P_UPDATE = 1, P_CHECK = 2, P_OBJECTIVE = 3 };

template <typename E>
__device__ __forceinline__ void store_elem(void *base, long idx, int lane_ok, E x)
{
    if (lane_ok) reinterpret_cast<E *>(base)[idx] = x;
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

    auto load_phi = [&](long c, XF<M>(&phi)[n][V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const long p = c * CH + (long)lane * V + v;
#pragma unroll
            for (int r = 0; r < n; ++r)
                phi[r][v] = (p < N) ? xfrom_log<M>(a[(long)items[r] * N + p]) : xzero<M>();
        }
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
            XF<M> phi[n][V];
            load_phi(c, phi);
#pragma unroll
            for (int S = 1; S < D; ++S) store_elem(scratch, c * (D - 1) + (S - 1), lane == 0, carryF[S]);
            E st[D][V], cin[D];
            level_scan<L, V, E, true>(phi, st, cin, carryF, K, lanepF, (double)slF, slF);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }

    double acc = 0.0;
    XF<double> accx = xzero<double>();
    for (long c = C - 1; c >= 0; --c) {
        XF<M> phi[n][V];
        load_phi(c, phi);
        if (C > 1) {
#pragma unroll
            for (int S = 1; S < D; ++S) carryF[S] = reinterpret_cast<const E *>(scratch)[c * (D - 1) + (S - 1)];
        }
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
                    const XF<double> ph = xfrom_log<double>(a[(long)j * N + p]);
                    accx = xadd(accx, xmul(ph, J.w));
                } else {
                    const double lj = xto_log(J);
                    if constexpr (MODE == P_PRODUCT) {
                        out[p] = lj;
                    } else if constexpr (MODE == P_UPDATE) {
                        // marginal error this update removes: u |exp(a_old - a_new) - 1|
                        const double lu = log_u[(long)j * N + p];
                        const double ao = a[(long)j * N + p];
                        const double an = lu > -INFINITY ? lu - lj : -INFINITY;
                        if (lu > -INFINITY) acc += exp(lu) * fabs(expm1(ao - an));
                        a[(long)j * N + p] = an;
                    } else {
                        const double lu = log_u[(long)j * N + p];
                        acc += fabs(exp(a[(long)j * N + p] + lj) - exp(lu));
                    }
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
