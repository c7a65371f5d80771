// The O(N) tensor-vector product with the subset states spread over the lanes.
//
// Same dynamic program as scan.hpp (gap form of the L1 cost, Sec. 4.2 with the
// ordering classes merged into subsets), laid out for many marginals: the 2^(l-1)
// states of one position live across the lanes of a team and a few registers per
// lane, and positions are walked one after the other.  Per position a state S of
// the l - 1 summed marginals R takes
//     A(S) <- g(|S|) A(S)                       (the gap before the position)
//     A(S) <- A(S) + A(S \ r) phi_r(x)         for each item r in S, one item at a time
// (the item-by-item form of placing any subset of R at x: l 2^(l-2) multiply-adds
// per position instead of the 3^(l-1) of a sum over all placed subsets), so no
// lane keeps more than a handful of states and nothing spills.
//
// Layout.  State index S = i * TL + t: the low LB = log2(TL) bits of S (items
// 0..LB-1) are the lane t inside the team, the high bits (items LB..l-2) the
// register i.  An item step over a lane bit reads the partner state from the lane
// 2^b below (DPP row shift inside rows of 16 lanes, a swizzle for 16, a permute
// for 32); over a register bit it stays in the lane.  Backward states are held
// complemented: the lane and register of forward state S hold the backward state
// of R \ S, so the backward item step reads the lane 2^b above and the combine
//     J_j(y) = sum_S F_y(S) g(|R \ S|) B_{y+1}(R \ S)
// is a per-lane product followed by one team-wide sum.
//
// The combine needs F_y and B_{y+1} together.  The forward walk stores its state
// every CK positions (checkpoints in scratch memory); the backward walk takes the
// blocks last to first, recomputes each block's CK forward states from its
// checkpoint into registers and combines while it steps backwards.  Every value
// is an extended-range number (XF: mantissa and exact integer power-of-two
// exponent), as in the one-wavefront solver, so no potential size over- or
// underflows.
#pragma once
#include <type_traits>

#include "scan.hpp"

namespace mmot {

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

// Registers an element of a scan occupies (mantissa + exponent).
template <typename E>
struct EWords;
template <>
struct EWords<XF<float>> {
    static constexpr int n = 2;
};
template <>
struct EWords<XF<double>> {
    static constexpr int n = 3;
};
template <>
struct EWords<DXF> {
    static constexpr int n = 6;
};

// Team layout of the states of an l-marginal product in element type E.
template <int L, typename E>
struct WL {
    static constexpr int n = L - 1;               // summed marginals
    static constexpr int D = wide_states(L);      // states (subsets of R)
    static constexpr int TL = wide_tl(L);         // lanes per team
    static constexpr int TPW = WAVE / TL;         // teams per wavefront
    static constexpr int RG = wide_rg(L);         // states per lane
    static constexpr int LB = ilog2c(TL);         // items held across lanes
    static constexpr int RB = ilog2c(RG);         // items held across registers
    static constexpr int CK = wide_ck(L, EWords<E>::n);  // positions per recompute block
    static constexpr bool SA = wide_store_all(L, EWords<E>::n);  // forward states of every position kept
};

// ---- lane moves inside a team ---------------------------------------------------
// UP = false: the value of lane t - 2^B; UP = true: of lane t + 2^B.  Only lanes
// whose source lies in the same team use the result.
template <int B, bool UP>
__device__ __forceinline__ int lmove(int x)
{
    if constexpr (B < 4) {
        return __builtin_amdgcn_update_dpp(0, x, UP ? (0x100 + (1 << B)) : (0x110 + (1 << B)), 0xF, 0xF, true);
    } else if constexpr (B == 4) {
        return __builtin_amdgcn_ds_swizzle(x, 0x401F);  // lane ^ 16 inside 32 lanes
    } else {
        return __builtin_amdgcn_ds_bpermute((int)(((threadIdx.x & 63) ^ 32) << 2), x);
    }
}
template <int B, bool UP>
__device__ __forceinline__ float lmove(float x)
{
    return __int_as_float(lmove<B, UP>(__float_as_int(x)));
}
template <int B, bool UP>
__device__ __forceinline__ double lmove(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = lmove<B, UP>((int)(b & 0xffffffffLL));
    const int hi = lmove<B, UP>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int B, bool UP, typename M>
__device__ __forceinline__ XF<M> lmove(XF<M> x)
{
    return {lmove<B, UP>(x.m), lmove<B, UP>(x.e)};
}
template <int B, bool UP>
__device__ __forceinline__ DXF lmove(DXF x)
{
    return {lmove<B, UP>(x.v), lmove<B, UP>(x.w)};
}

// c ? a : b field by field (a select of whole structs can become a per-lane
// choice between two private-memory addresses).
template <typename M>
__device__ __forceinline__ XF<M> esel(bool c, XF<M> a, XF<M> b)
{
    return {c ? a.m : b.m, c ? a.e : b.e};
}
__device__ __forceinline__ DXF esel(bool c, DXF a, DXF b) { return {esel(c, a.v, b.v), esel(c, a.w, b.w)}; }

// Wavefront-local ordering of the LDS accesses between the lanes of a team (one
// team never spans more than a wavefront).  The fences cover LDS only: the
// walks' global loads and stores are each used by the lane that issued them, so
// a team_sync need not wait for them to land.
__device__ __forceinline__ void team_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// As team_sync, also ordering global memory: for global data one lane writes and
// other lanes of the team read later in the same launch (potentials).
__device__ __forceinline__ void team_sync_global()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}


// Per-lane constants of one walk: g(level) for the levels this lane's registers
// can hold.  Forward state S_i = i TL + t has level m + |t| + |i|; the
// complemented backward state has level m + n - |t| - |i|.
template <int L, typename E>
struct WConst {
    using M = typename ET<E>::MT;
    static constexpr int RB = WL<L, E>::RB;
    XG<M> g[RB + 1];
    double pc[RB + 1];  // level (l - level) (times the gap's length on a non-uniform grid):
                        // weight of a gap for the objective
};

// a + b p for extended values, the result left unnormalized: the exponents are
// aligned to the larger one and the mantissas meet in one FMA.  Within one
// position a state takes at most l - 1 such steps, so its mantissa stays far
// inside the mantissa type's range until wstep renormalizes it.
template <typename M>
__device__ __forceinline__ XF<M> xmac_lazy(XF<M> a, XF<M> b, XF<M> p)
{
    const int te = b.e + p.e;
    const int e = max(a.e, te);
    return {fma(b.m, xldexp(p.m, te - e), xldexp(a.m, a.e - e)), e};
}
__device__ __forceinline__ DXF xmac_lazy(DXF a, DXF b, XF<double> p)
{
    return {xmac_lazy(a.v, b.v, p), xmac_lazy(a.w, b.w, p)};
}
__device__ __forceinline__ DXF xnorm(DXF x) { return {xnorm(x.v), xnorm(x.w)}; }

// One position of a walk: the gap factor, then the items placed at the position.
// ph[r] is phi of item r at the position.  BWD: complemented backward states.
template <int L, typename E, bool BWD, int RG_ = WL<L, E>::RG>
__device__ __forceinline__ void wstep(E (&A)[RG_], const XF<typename ET<E>::MT> *ph, const WConst<L, E> &c, int t)
{
    using W = WL<L, E>;
    using T_ = ET<E>;
#pragma unroll
    for (int i = 0; i < W::RG; ++i) A[i] = T_::disc(A[i], c.g[popc(i)], c.pc[popc(i)]);
    // items across lanes.  With teams of 16 lanes or more every moved value comes
    // from a live lane of the team (or is the DPP's zero at a row edge), so every
    // lane takes the MAC and a lane whose states do not hold the item multiplies
    // by an exact zero (exponent XF_ZERO_E): its mantissa and exponent stay as
    // they were.  Narrower teams share DPP rows with neighbours that may have
    // left, and select instead.
#pragma unroll
    for (int r = 0; r < W::LB; ++r) {
        const bool upd = BWD ? !((t >> r) & 1) : ((t >> r) & 1);
        const XF<typename T_::MT> p = (W::TL >= 16) ? esel(upd, ph[r], xzero<typename T_::MT>()) : ph[r];
#pragma unroll
        for (int i = 0; i < W::RG; ++i) {
            const E o = (r == 0)   ? lmove<0, BWD>(A[i])
                        : (r == 1) ? lmove<1, BWD>(A[i])
                        : (r == 2) ? lmove<2, BWD>(A[i])
                        : (r == 3) ? lmove<3, BWD>(A[i])
                        : (r == 4) ? lmove<4, BWD>(A[i])
                                   : lmove<5, BWD>(A[i]);
            const E nv = xmac_lazy(A[i], o, p);
            A[i] = (W::TL >= 16) ? nv : esel(upd, nv, A[i]);
        }
    }
    // items across registers
#pragma unroll
    for (int rb = 0; rb < W::RB; ++rb) {
        const XF<typename T_::MT> p = ph[W::LB + rb];
#pragma unroll
        for (int i = 0; i < W::RG; ++i) {
            const bool set = (i >> rb) & 1;
            if (BWD ? !set : set) A[i] = xmac_lazy(A[i], A[i ^ (1 << rb)], p);
        }
    }
#pragma unroll
    for (int i = 0; i < W::RG; ++i) A[i] = xnorm(A[i]);
}

// Sum over the lanes of a team; the total lands in the team's last lane.
template <int L, typename E>
__device__ __forceinline__ E team_total(E x, int t)
{
    using W = WL<L, E>;
    using T_ = ET<E>;
#pragma unroll
    for (int b = 0; b < W::LB; ++b) {
        const E o = (b == 0)   ? lmove<0, false>(x)
                    : (b == 1) ? lmove<1, false>(x)
                    : (b == 2) ? lmove<2, false>(x)
                    : (b == 3) ? lmove<3, false>(x)
                    : (b == 4) ? lmove<4, false>(x)
                               : lmove<5, false>(x);
        const E nx = T_::add(x, o);
        x = esel((t >> b) & 1, nx, x);
    }
    return x;
}

// Team context: its lanes, LDS staging of scaling factors, checkpoint scratch.
template <int L, typename E>
struct WTeam {
    using M = typename ET<E>::MT;
    int t;                 // lane inside the team
    bool last;             // the team's last lane (holds team totals)
    XF<M> *ph;             // LDS [CK][n] scaling factors of the staged block
    XG<M> *gt;             // LDS [CK + 1][l + 1] gap factors g(level) of the staged block (row s:
                           // the gap before its position s); one row on the uniform grid
    double *gd;            // LDS [CK + 1] those gaps' lengths (non-uniform grid)
    double *vj, *vu;       // LDS [CK] a_j and log u_j at the staged block's positions
    E *ck;                 // scratch: checkpoints [blocks][D]
};

// Stage phi of the summed marginals at the positions of one block into LDS:
// slot s is position x0 + s (s < cnt), item r is marginal r < j ? r : r + 1.
// With them the gap factors g_s(level) = exp(-d_s level (l - level) / eps) of the
// gaps d_s between positions x0 + s - 1 and x0 + s, s = 0..cnt (a gap outside
// [0, N) has length 0): on the uniform grid every gap is h and one row, from
// h / eps, serves the whole block.  With stage_j, also a_j (and log u_j if
// log_u is given) at the block's positions, for the combine's epilogue.
template <int L, typename E>
__device__ __forceinline__ void stage_phi(const WTeam<L, E> &tm, const Inst *__restrict__ I,
                                          const double *__restrict__ a, int j, long x0, int cnt,
                                          bool stage_j = false, const double *__restrict__ log_u = nullptr)
{
    using W = WL<L, E>;
    using M = typename ET<E>::MT;
    const long N = I->N;
    team_sync();
    for (int k = tm.t; k < W::CK * W::n; k += W::TL) {
        const int s = k / W::n, r = k - s * W::n;
        const int q = r < j ? r : r + 1;
        XF<M> v = xzero<M>();
        if (s < cnt) v = xfrom_log<M>(gld(&a[(long)q * N + x0 + s]));
        tm.ph[s * W::n + r] = v;
    }
    if (stage_j)
        for (int s = tm.t; s < cnt; s += W::TL) {
            tm.vj[s] = gld(&a[(long)j * N + x0 + s]);
            if (log_u) tm.vu[s] = gld(&log_u[(long)j * N + x0 + s]);
        }
    const double *xs = I->x;
    const int rows = xs ? cnt + 1 : 1;
    for (int k = tm.t; k < rows * (L + 1); k += W::TL) {
        const int s = k / (L + 1), lev = k - s * (L + 1);
        double lg;
        if (xs) {
            const long p = x0 + s;
            const double d = (p >= 1 && p < N) ? gld(&xs[p]) - gld(&xs[p - 1]) : 0.0;
            if (lev == 0) tm.gd[s] = d;
            lg = -(double)(lev * (L - lev)) * (d * I->ieps);
        } else {
            lg = -(double)(lev * (L - lev)) * I->hoe;
        }
        tm.gt[k] = xg_from_log<M>(lg);
    }
    team_sync();
}

// Walk constants of one position from the staged gap factors: row of the gap
// crossed, this lane's level base and direction (as wconst).  The objective's
// cost weight of a gap is level (l - level) times its length on a non-uniform
// grid, times 1 on the uniform grid (where h multiplies the total).
template <int L, typename E>
__device__ __forceinline__ WConst<L, E> wconst_row(const WTeam<L, E> &tm, bool grid, int row, int base, int sign)
{
    using M = typename ET<E>::MT;
    WConst<L, E> c;
    const XG<M> *g = tm.gt + (grid ? row : 0) * (L + 1);
    const double d = grid ? tm.gd[row] : 1.0;
#pragma unroll
    for (int k = 0; k <= WL<L, E>::RB; ++k) {
        const int lev = base + sign * k;
        const bool ok = lev >= 0 && lev <= L;
        const XG<M> v = g[ok ? lev : 0];
        c.g[k] = {ok ? v.hi : M(0), ok ? v.lo : M(0), ok ? v.e : XF_ZERO_E, 0};
        c.pc[k] = ok ? (double)(lev * (L - lev)) * d : 0.0;
    }
    return c;
}

// Accumulator of a pass's per-position results (the FP64 estimate, residual or
// objective terms), held by the team's last lane.
struct WAcc {
    double s;
    XF<double> x;
};

// One product pass of marginal j over positions [p0, p1) of one instance on one
// team, with the forward state at p0 - 1 (cf, or the empty placement if NULL)
// and the complemented backward state at p1 (cb, or empty if NULL).  What is
// done with log J_j(y) follows finish_lj (P_PRODUCT / P_UPDATE / P_CHECK); for
// P_OBJECTIVE (E = DXF) the team's last lane accumulates phi_j(y) times the
// cost-weighted product.  Returns the accumulated sum in the team's last lane.
template <int L, typename E, int MODE>
__device__ WAcc wide_pass(const WTeam<L, E> &tm, const Inst *__restrict__ I, int j, double *__restrict__ a,
                          const double *__restrict__ log_u, double *__restrict__ out, long p0, long p1, const E *cf,
                          const E *cb)
{
    using W = WL<L, E>;
    using T_ = ET<E>;
    constexpr int RG = W::RG, CK = W::CK, n = W::n, D = W::D;
    const long N = I->N;
    const int t = tm.t;
    const int pt = popc(t);
    const bool grid = I->x != nullptr;

    WAcc acc = {0.0, xzero<double>()};
    const long len = p1 - p0;
    if (len <= 0) return acc;
    const long nblk = (len + CK - 1) / CK;

    // forward walk: the state before every block (W::SA: after every position)
    E A[RG];
#pragma unroll
    for (int i = 0; i < RG; ++i) {
        const int S = i * W::TL + t;
        A[i] = cf ? gld_e(&cf[S]) : esel(S == 0, T_::one(), T_::zero());
    }
    for (long b = 0; b < nblk; ++b) {
        const long x0 = p0 + b * CK;
        const int cnt = (int)min((long)CK, p1 - x0);
        if constexpr (!W::SA) {
#pragma unroll
            for (int i = 0; i < RG; ++i) gst_e(&tm.ck[b * D + i * W::TL + t], A[i]);
            if (b == nblk - 1) break;  // the last block's forward states are recomputed below
        }
        stage_phi<L, E>(tm, I, a, j, x0, cnt);
        for (int s = 0; s < cnt; ++s) {
            wstep<L, E, false>(A, tm.ph + s * n, wconst_row<L, E>(tm, grid, s, pt, 1), t);
            if constexpr (W::SA) {
#pragma unroll
                for (int i = 0; i < RG; ++i) gst_e(&tm.ck[(x0 - p0 + s) * D + i * W::TL + t], A[i]);
            }
        }
    }
    team_sync();

    // backward walk, block by block from the last
    E Bs[RG];
#pragma unroll
    for (int i = 0; i < RG; ++i) {
        const int S = i * W::TL + t;
        Bs[i] = cb ? gld_e(&cb[S]) : esel(S == D - 1, T_::one(), T_::zero());
    }
    for (long b = nblk - 1; b >= 0; --b) {
        const long x0 = p0 + b * CK;
        const int cnt = (int)min((long)CK, p1 - x0);
        stage_phi<L, E>(tm, I, a, j, x0, cnt, MODE != P_PRODUCT,
                        (MODE == P_UPDATE || MODE == P_CHECK) ? log_u : nullptr);
        // forward states of the block: read back (W::SA) or recomputed from the checkpoint
        E F[CK][RG];
        if constexpr (W::SA) {
#pragma unroll
            for (int s = 0; s < CK; ++s)
#pragma unroll
                for (int i = 0; i < RG; ++i)
                    F[s][i] = gld_e(&tm.ck[(x0 - p0 + min(s, cnt - 1)) * D + i * W::TL + t]);
        } else {
#pragma unroll
            for (int i = 0; i < RG; ++i) A[i] = gld_e(&tm.ck[b * D + i * W::TL + t]);
#pragma unroll
            for (int s = 0; s < CK; ++s) {
                if (s < cnt) wstep<L, E, false>(A, tm.ph + s * n, wconst_row<L, E>(tm, grid, s, pt, 1), t);
#pragma unroll
                for (int i = 0; i < RG; ++i) F[s][i] = A[i];
            }
        }
#pragma unroll
        for (int s = CK - 1; s >= 0; --s) {
            if (s >= cnt) continue;
            const long y = x0 + s;
            // the gap (y, y + 1): row s + 1
            const WConst<L, E> cB = wconst_row<L, E>(tm, grid, s + 1, n - pt, -1);
            // J(y) = sum_S F_y(S) g(|R \ S|) B_{y+1}(R \ S)
            E part = T_::zero();
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                const E hb = T_::disc(Bs[i], cB.g[popc(i)], cB.pc[popc(i)]);
                part = (i == 0) ? T_::prod(F[s][i], hb) : T_::add(part, T_::prod(F[s][i], hb));
            }
            const E J = team_total<L, E>(part, t);
            if (tm.last) {
                // the epilogue of finish_lj, with a_j and log u_j from the staged block
                if constexpr (MODE == P_OBJECTIVE) {
                    const XF<double> ph = xfrom_log<double>(tm.vj[s]);
                    acc.x = xadd(acc.x, xmul(ph, J.w));
                } else if constexpr (MODE == P_PRODUCT) {
                    gst(&out[y], xto_log(J));
                } else if constexpr (MODE == P_UPDATE) {
                    const double lj = xto_log(J), lu = tm.vu[s], ao = tm.vj[s];
                    const double an = lu > -INFINITY ? lu - lj : -INFINITY;
                    gst(&a[(long)j * N + y], an);
                    acc.s += lu > -INFINITY ? exp(lu) * fabs(expm1(ao - an)) : 0.0;
                } else {
                    acc.s += fabs(exp(tm.vj[s] + xto_log(J)) - exp(tm.vu[s]));
                }
            }
            wstep<L, E, true>(Bs, tm.ph + s * n, cB, t);
        }
    }
    team_sync_global();  // a_j written by the last lane is read by every lane in the next pass
    return acc;
}

}  // namespace mmot

namespace mmot {

// A value of the team's last lane, in every lane of the team.
template <int L, typename E>
__device__ __forceinline__ double team_bcast_last(double x)
{
    using W = WL<L, E>;
    if constexpr (W::TPW == 1) {
        return rlane(x, WAVE - 1);
    } else {
        const int src = (int)(threadIdx.x & (WAVE - 1)) | (W::TL - 1);
        const long long b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffLL));
        const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}

// Next instance ticket of a team, the same value in every lane of the team:
// every lane takes part in the atomic (the team's first lane adds 1).
template <int L, typename E>
__device__ __forceinline__ int team_ticket(int *ticket, int t)
{
    using W = WL<L, E>;
    const int v = atomicAdd(ticket, t == 0 ? 1 : 0);
    if constexpr (W::TPW == 1) {
        return __builtin_amdgcn_readfirstlane(v);
    } else {
        const int src = (int)(threadIdx.x & (WAVE - 1)) & ~(W::TL - 1);
        return __builtin_amdgcn_ds_bpermute(src << 2, v);
    }
}

// LDS bytes one team needs to stage scaling factors for every element kind.
template <int L>
struct WShared {
    static constexpr int n = L - 1;
    static constexpr int B32 = WL<L, XF<float>>::CK * n * (int)sizeof(XF<float>);
    static constexpr int B64 = WL<L, XF<double>>::CK * n * (int)sizeof(XF<double>);
    static constexpr int BOB = WL<L, DXF>::CK * n * (int)sizeof(XF<double>);
    static constexpr int M1 = B32 > B64 ? B32 : B64;
    static constexpr int PH = ((M1 > BOB ? M1 : BOB) + 15) / 16 * 16;
    // gap-factor rows: as many as the longest block has positions, plus one
    static constexpr int C1 = WL<L, XF<float>>::CK > WL<L, XF<double>>::CK ? WL<L, XF<float>>::CK
                                                                           : WL<L, XF<double>>::CK;
    static constexpr int ROWS = (C1 > WL<L, DXF>::CK ? C1 : WL<L, DXF>::CK) + 1;
    static constexpr int GT = ROWS * (L + 1) * (int)sizeof(XG<double>);
    // gap lengths [ROWS], a_j and log u_j [ROWS] each
    static constexpr int BYTES = (PH + GT + 3 * ROWS * (int)sizeof(double) + 15) / 16 * 16;
    static constexpr int TPWMAX = WL<L, XF<float>>::TPW;  // TL does not depend on the element kind
};

static_assert(sizeof(XF<float>) == 8 && sizeof(XF<double>) == 16 && sizeof(DXF) == 32,
              "element sizes assumed by wide_scratch_bytes");

template <int L, typename E>
__device__ __forceinline__ WTeam<L, E> make_team(char *lds, void *scratch)
{
    using W = WL<L, E>;
    const int lane = threadIdx.x & (WAVE - 1);
    WTeam<L, E> tm;
    tm.t = lane & (W::TL - 1);
    tm.last = tm.t == W::TL - 1;
    char *base = lds + (lane / W::TL) * WShared<L>::BYTES;
    tm.ph = reinterpret_cast<XF<typename ET<E>::MT> *>(base);
    tm.gt = reinterpret_cast<XG<typename ET<E>::MT> *>(base + WShared<L>::PH);
    tm.gd = reinterpret_cast<double *>(base + WShared<L>::PH + WShared<L>::GT);
    tm.vj = tm.gd + WShared<L>::ROWS;
    tm.vu = tm.vj + WShared<L>::ROWS;
    tm.ck = reinterpret_cast<E *>(scratch);
    return tm;
}

// Sweeps of one instance on one team (Alg. 1 loop: Gauss-Seidel updates in
// precision M, FP64 residual), same stopping rule as solve_one.  The objective
// follows in its own launch (k_wide_objective), so that its wider elements do
// not set this kernel's register count.
template <int L, typename M>
__device__ void wide_solve(char *lds, const Inst *__restrict__ I, const Ptrs P, const RunOpts o,
                           Result *__restrict__ R)
{
    using EU = XF<M>;
    const WTeam<L, EU> tu = make_team<L, EU>(lds, P.scratch);
    const WTeam<L, XF<double>> tc = make_team<L, XF<double>>(lds, P.scratch);
    constexpr int TL = WL<L, EU>::TL;
    const long N = I->N;
    double *a = P.a;
    const double *lu = P.log_u;
    const int flags = o.flags | P.flags;
    const long itr_max = P.itr_cap > 0 ? P.itr_cap : o.itr_max;

    if (!(flags & F_WARM) && P.it0 == 0) {
        // phi = 1/N (Alg. 1 initialisation)
        const double a0 = -log((double)N);
        for (long p = tu.t; p < (long)L * N; p += TL) a[p] = a0;
        team_sync_global();
    }
    long it = P.it0;
    int jr = P.j0;
    double res = INFINITY, f = 1.0;
    int status = ST_OK;
    bool checked = false;
    while (it < itr_max || jr > 0) {
        const bool resumed = jr > 0;
        if (!resumed) ++it;
        double est = 0.0;
        for (int j = jr; j < L; ++j) {
            const WAcc e = wide_pass<L, EU, P_UPDATE>(tu, I, j, a, lu, nullptr, 0, N, nullptr, nullptr);
            if (j < L - 1) est += e.s;
        }
        est = team_bcast_last<L, EU>(est);
        jr = 0;
        const bool trig = !resumed && o.tol >= 0.0 && est <= o.tol * f;
        const bool chk = !(flags & F_NO_CHECK) &&
                         ((resumed && P.j0 == L) || (o.check_every > 0 && it % o.check_every == 0) ||
                          it >= itr_max || trig);
        if (chk) {
            checked = true;
            double r = 0.0;
            for (int j = 0; j < L - 1; ++j)
                r += wide_pass<L, XF<double>, P_CHECK>(tc, I, j, a, lu, nullptr, 0, N, nullptr, nullptr).s;
            res = team_bcast_last<L, EU>(r);
            if (!(res == res)) {
                status = ST_NUMERIC;
                break;
            }
            if (res <= o.tol) break;
            if (trig) f *= 0.5;
        }
    }
    if (status == ST_OK && checked && o.tol >= 0.0 && !(res <= o.tol)) status = ST_NOT_CONVERGED;
    if (tu.last) {
        R->W = 0.0;
        R->marg_err = res;
        R->iters = it;
        R->status = status;
        R->l = L;
        R->N = N;
    }
}

// Persistent batch of l = L instances: each team takes the next instance ticket
// until the list is exhausted.
template <int L, typename M>
__global__ __launch_bounds__(64) void k_wide_batch(const Inst *I, const Ptrs *P, const int *order, int count,
                                                   RunOpts o, Result *R, int *ticket)
{
    __shared__ __attribute__((aligned(16))) char lds[WShared<L>::TPWMAX * WShared<L>::BYTES];
    const int t = (int)threadIdx.x & (WL<L, XF<M>>::TL - 1);
    for (;;) {
        const int tk = team_ticket<L, XF<M>>(ticket, t);
        if (tk >= count) break;
        const int idx = order[tk];
        wide_solve<L, M>(lds, &I[idx], P[idx], o, &R[idx]);
    }
}

// FP64 objective (Sec. 2 Eq. mmot distance) of the listed instances whose solve
// ended with status ST_OK (unless F_NO_OBJ), one team each; a non-finite value
// turns the status into ST_NUMERIC.
template <int L>
__global__ __launch_bounds__(64) void k_wide_objective(const Inst *I, const Ptrs *P, const int *order, int count,
                                                       RunOpts o, Result *R, int *ticket)
{
    __shared__ __attribute__((aligned(16))) char lds[WShared<L>::TPWMAX * WShared<L>::BYTES];
    const int t = (int)threadIdx.x & (WL<L, DXF>::TL - 1);
    for (;;) {
        const int tk = team_ticket<L, DXF>(ticket, t);
        if (tk >= count) break;
        const int idx = order[tk];
        if (R[idx].status != ST_OK || ((o.flags | P[idx].flags) & F_NO_OBJ)) continue;
        const WTeam<L, DXF> to = make_team<L, DXF>(lds, P[idx].scratch);
        const WAcc w = wide_pass<L, DXF, P_OBJECTIVE>(to, &I[idx], L - 1, P[idx].a, P[idx].log_u, nullptr, 0,
                                                      I[idx].N, nullptr, nullptr);
        if (to.last) {
            const double W = I[idx].h * xto_double(w.x);
            R[idx].W = W;
            if (!(W == W) || W == INFINITY) R[idx].status = ST_NUMERIC;
        }
    }
}

// One product (MODE P_PRODUCT, element XF<M>) or the objective (P_OBJECTIVE, DXF)
// of one instance on the first team of one wavefront.
template <int L, typename E, int MODE>
__global__ __launch_bounds__(64) void k_wide_pass(const Inst *I, Ptrs P, int j, double *result)
{
    __shared__ __attribute__((aligned(16))) char lds[WShared<L>::TPWMAX * WShared<L>::BYTES];
    if (threadIdx.x >= WL<L, E>::TL) return;
    const WTeam<L, E> tm = make_team<L, E>(lds, P.scratch);
    const WAcc r = wide_pass<L, E, MODE>(tm, I, j, P.a, P.log_u, P.out, 0, I->N, nullptr, nullptr);
    if (tm.last && result) result[0] = (MODE == P_OBJECTIVE) ? I->h * xto_double(r.x) : r.s;
}

// FP64 errors of all l marginals of one instance.
template <int L>
__global__ __launch_bounds__(64) void k_wide_check_all(const Inst *I, Ptrs P, double *err)
{
    __shared__ __attribute__((aligned(16))) char lds[WShared<L>::TPWMAX * WShared<L>::BYTES];
    if (threadIdx.x >= WL<L, XF<double>>::TL) return;
    const WTeam<L, XF<double>> tm = make_team<L, XF<double>>(lds, P.scratch);
    for (int j = 0; j < L; ++j) {
        const WAcc r = wide_pass<L, XF<double>, P_CHECK>(tm, I, j, P.a, P.log_u, nullptr, 0, I->N, nullptr, nullptr);
        if (tm.last) err[j] = r.s;
    }
}

}  // namespace mmot

namespace mmot {

// ---- tiles: one instance spread over many teams ------------------------------
//
// Positions are cut into tiles of B.  A tile's effect on the forward state is
// affine in the state it starts from: with S' the summed marginals already
// placed before the tile and T those placed inside it,
//     F_end(S) = sum_{S' subset S} F_start(S') Q_{|S'|}(S \ S'),
// where Q_m(T) is the walk over the tile from the empty placement with every gap
// discount shifted by m members (g(m + |T|) instead of g(|T|)), because the gap
// weights only depend on how many members lie to the left.  The backward
// direction is the mirror image.  So a product runs in three launches:
//   1. every (tile, m, direction): the walk that gives Q_m   (k_tile_agg)
//   2. every direction: the carries from tile to tile, in order (k_tile_chain)
//   3. every tile: the product pass from its true carries      (k_tile_final)

// Walk of one job (tile t, offset m, direction dir) from the empty placement;
// stores the final state as Q_m of the tile.
template <int L, typename E>
__device__ void tile_agg_job(const WTeam<L, E> &tm, const Inst *__restrict__ I, const TileInst &T, const double *a,
                             int j, int t, int m, int dir)
{
    using W = WL<L, E>;
    using T_ = ET<E>;
    constexpr int RG = W::RG, CK = W::CK, n = W::n, D = W::D;
    const long N = I->N;
    const long p0 = (long)t * T.B, p1 = min(N, p0 + T.B);
    const int pt = popc(tm.t);
    const bool grid = I->x != nullptr;
    E A[RG];
    if (dir == 0) {
#pragma unroll
        for (int i = 0; i < RG; ++i) A[i] = esel(i * W::TL + tm.t == 0, T_::one(), T_::zero());
        for (long x0 = p0; x0 < p1; x0 += CK) {
            const int cnt = (int)min((long)CK, p1 - x0);
            stage_phi<L, E>(tm, I, a, j, x0, cnt);
            for (int s = 0; s < cnt; ++s)
                wstep<L, E, false>(A, tm.ph + s * n, wconst_row<L, E>(tm, grid, s, pt + m, 1), tm.t);
        }
    } else {
#pragma unroll
        for (int i = 0; i < RG; ++i) A[i] = esel(i * W::TL + tm.t == D - 1, T_::one(), T_::zero());
        const long nb = (p1 - p0 + CK - 1) / CK;
        for (long b = nb - 1; b >= 0; --b) {
            const long x0 = p0 + b * CK;
            const int cnt = (int)min((long)CK, p1 - x0);
            stage_phi<L, E>(tm, I, a, j, x0, cnt);
            for (int s = cnt - 1; s >= 0; --s)
                wstep<L, E, true>(A, tm.ph + s * n, wconst_row<L, E>(tm, grid, s + 1, m + n - pt, -1), tm.t);
        }
    }
    E *q = reinterpret_cast<E *>(T.agg) + (((long)t * 2 + dir) * L + m) * D;
#pragma unroll
    for (int i = 0; i < RG; ++i) gst_e(&q[i * W::TL + tm.t], A[i]);
    team_sync();
}

// Jobs of the tiled launches: x = instance, y = tile (or direction), z = offset m, w = direction.
// state_need: the job runs only for instances whose TileTrack.state is this.
template <int L, typename E>
__global__ __launch_bounds__(64) void k_tile_agg(const Inst *I, const Ptrs *P, const TileInst *TI, const TileTrack *Tr,
                                                 const int4 *jobs, int njobs, int j, int state_need)
{
    __shared__ __attribute__((aligned(16))) char lds[WShared<L>::TPWMAX * WShared<L>::BYTES];
    using W = WL<L, E>;
    const int team = (int)threadIdx.x / W::TL;
    const int jid = (int)blockIdx.x * W::TPW + team;
    if (jid >= njobs) return;
    const int4 jb = jobs[jid];
    if (Tr && Tr[jb.x].state != state_need) return;
    const WTeam<L, E> tm = make_team<L, E>(lds, nullptr);
    tile_agg_job<L, E>(tm, &I[jb.x], TI[jb.x], P[jb.x].a, j, jb.y, jb.z, jb.w);
}

// acc + a b with the deferred normalisation of xmac_lazy (dual numbers: the
// value part and the product rule for the cost-weighted part).
template <typename M>
__device__ __forceinline__ XF<M> chain_mac(XF<M> acc, XF<M> a, XF<M> b)
{
    return xmac_lazy(acc, a, b);
}
__device__ __forceinline__ DXF chain_mac(DXF acc, DXF a, DXF b)
{
    return {xmac_lazy(acc.v, a.v, b.v), xmac_lazy(xmac_lazy(acc.w, a.v, b.w), a.w, b.v)};
}

constexpr int CHAIN_THREADS = 512;
constexpr int CHAIN_CHUNK = 16;  // subset terms per work item

// Number of work items of a hop over the subsets of n items: S with 2^|S|
// subsets has ceil(2^|S| / CHAIN_CHUNK) of them.
__host__ __device__ constexpr int chain_items(int n)
{
    int tot = 0;
    for (int S = 0; S < (1 << n); ++S) tot += ((1 << __builtin_popcount(S)) + CHAIN_CHUNK - 1) / CHAIN_CHUNK;
    return tot;
}

// Element kinds in LDS as word planes: word w of element i at plane[w][i], so
// that lanes reading neighbouring elements hit neighbouring banks (a 16-byte
// struct stride puts a wavefront's reads on a quarter of the banks).  Only the
// words that carry data are stored (not the padding of XF<double>).
template <typename E>
struct Words;
template <>
struct Words<XF<float>> {
    static constexpr int NW = 2;
    static constexpr int at(int k) { return k; }
};
template <>
struct Words<XF<double>> {
    static constexpr int NW = 3;
    static constexpr int at(int k) { return k; }
};
template <>
struct Words<DXF> {
    static constexpr int NW = 6;
    static constexpr int at(int k) { return k < 3 ? k : k + 1; }
};

template <typename E, int COUNT>
__device__ __forceinline__ E pl_load(const int *pl, int i)
{
    E v;
    int *d = reinterpret_cast<int *>(&v);
#pragma unroll
    for (int k = 0; k < Words<E>::NW; ++k) d[Words<E>::at(k)] = pl[k * COUNT + i];
    return v;
}
template <typename E, int COUNT>
__device__ __forceinline__ void pl_store(int *pl, int i, E v)
{
    const int *d = reinterpret_cast<const int *>(&v);
#pragma unroll
    for (int k = 0; k < Words<E>::NW; ++k) pl[k * COUNT + i] = d[Words<E>::at(k)];
}

// The hop's aggregates are staged in LDS when they fit beside the rest.
template <int L, typename E>
constexpr bool chain_stages()
{
    return (size_t)4 * Words<E>::NW * ((size_t)L * WL<L, E>::D + WL<L, E>::D + chain_items(L - 1)) +
               sizeof(int) * (size_t)chain_items(L - 1) <=
           (size_t)136 * 1024;
}

// Carries from tile to tile in one direction, one workgroup of CHAIN_THREADS per
// (instance, direction).  In subset space (forward: S as held; backward: the
// complement of the index), c_next(S) = sum_{S' subset S} c(S') Q_{|S'|}(S \ S')
// with c(empty) = 1.  The 3^(l-1) terms of a hop are dealt to the threads as work
// items of at most CHAIN_CHUNK subsets S' of one S (S' walked downwards from a
// stored start); each item's partial sum goes to LDS and a second phase adds the
// items of each S.  The tile's l 2^(l-1) aggregates are read into registers
// during the previous hop and stored to LDS at the start of their own, so a hop
// waits on no global load.
template <int L, typename E>
__global__ __launch_bounds__(CHAIN_THREADS) void k_tile_chain(const TileInst *TI, const TileTrack *Tr,
                                                              const int2 *jobs, int njobs, int state_need)
{
    using T_ = ET<E>;
    constexpr int D = WL<L, E>::D;
    constexpr int n = L - 1;
    constexpr int MAXI = chain_items(n);
    constexpr bool STAGE = chain_stages<L, E>();
    constexpr int QN = L * D;
    constexpr int PF = STAGE ? (QN + CHAIN_THREADS - 1) / CHAIN_THREADS : 1;
    constexpr int NW = Words<E>::NW;
    __shared__ int c[NW * D];
    __shared__ int part[NW * MAXI];
    __shared__ int item[MAXI];  // S | start S' << 10 | count << 20
    __shared__ int ioff[D + 1];
    __shared__ int qs[STAGE ? NW * QN : 1];
    // The hop reads aggregate rank m D + subset; D is a multiple of the 32 LDS banks
    // and many of the subsets read together are multiples of 32 too, so the plain
    // index would pile a wavefront's reads onto bank 0.  The staged copy lives at
    // a swizzled index: the low five bits XOR-ed with the next ten (a permutation
    // inside every aligned group of 32, so inside [0, QN) when QN is a multiple of 32).
    auto qsw = [](int i) { return (QN % 32 == 0) ? i ^ (((i >> 5) ^ (i >> 10)) & 31) : i; };
    // the carries likewise (the subsets read together are often multiples of 32)
    auto csw = [](int i) { return (D % 32 == 0) ? i ^ ((i >> 5) & 31) : i; };
    const int2 jb = jobs[blockIdx.x];
    if (Tr && Tr[jb.x].state != state_need) return;
    const TileInst T = TI[jb.x];
    const int dir = jb.y;
    const int tid = threadIdx.x;
    auto idx = [&](int S) { return dir == 0 ? S : (D - 1) ^ S; };
    // item table: offsets by a prefix sum of the per-state counts, then every
    // thread lists its own states' items (subsets of S in decreasing order,
    // CHAIN_CHUNK at a time)
    for (int S = tid; S < D; S += blockDim.x) ioff[S + 1] = ((1 << popc(S)) + CHAIN_CHUNK - 1) / CHAIN_CHUNK;
    lds_barrier();
    if (tid == 0) {
        ioff[0] = 0;
        for (int S = 0; S < D; ++S) ioff[S + 1] += ioff[S];
    }
    lds_barrier();
    for (int S = tid; S < D; S += blockDim.x) {
        int o = ioff[S], Sp = S, left = 1 << popc(S);
        while (left > 0) {
            const int cnt = min(CHAIN_CHUNK, left);
            item[o++] = S | (Sp << 10) | (cnt << 20);
            for (int k = 0; k < cnt; ++k) Sp = (Sp - 1) & S;
            left -= cnt;
        }
    }
    for (int S = tid; S < D; S += blockDim.x) pl_store<E, D>(c, csw(S), esel(S == 0, T_::one(), T_::zero()));
    E *carry = reinterpret_cast<E *>(T.carry);
    const E *agg = reinterpret_cast<const E *>(T.agg);
    auto hop_q = [&](int s) { return agg + ((long)(dir == 0 ? s : T.ntile - 1 - s) * 2 + dir) * QN; };
    // prefetch registers: the data words of aggregate min(tid + k 512, QN - 1), read
    // through a global-address-space pointer (a flat load would also count
    // against the LDS wait counter and stall every LDS read of the hop until it
    // landed)
    using GInt = const __attribute__((address_space(1))) int;
    int pre[PF][NW];
    auto fetch = [&](const E *q) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            GInt *src = (GInt *)(q + min(tid + k * CHAIN_THREADS, QN - 1));
#pragma unroll
            for (int w = 0; w < NW; ++w) pre[k][w] = src[Words<E>::at(w)];
        }
    };
    if (STAGE && T.ntile > 1) fetch(hop_q(0));
    lds_barrier();
    for (int s = 0; s < T.ntile; ++s) {
        const int t = dir == 0 ? s : T.ntile - 1 - s;
        for (int S = tid; S < D; S += blockDim.x)
            gst_e(&carry[((long)t * 2 + dir) * D + idx(S)], pl_load<E, D>(c, csw(S)));
        if (s == T.ntile - 1) break;
        const E *qg = hop_q(s);  // the hop's aggregates in global memory (used when not staged)
        if (STAGE) {
#pragma unroll
            for (int k = 0; k < PF; ++k)
                if (tid + k * CHAIN_THREADS < QN) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) qs[w * QN + qsw(tid + k * CHAIN_THREADS)] = pre[k][w];
                }
            lds_barrier();
            fetch(hop_q(min(s + 1, T.ntile - 2)));
        }
        auto qat = [&](int i) -> E {
            if constexpr (STAGE) {
                return pl_load<E, QN>(qs, qsw(i));
            } else {
                E v;
                int *d = reinterpret_cast<int *>(&v);
                GInt *src = (GInt *)(qg + i);
#pragma unroll
                for (int w = 0; w < NW; ++w) d[Words<E>::at(w)] = src[Words<E>::at(w)];
                return v;
            }
        };
        for (int it = tid; it < ioff[D]; it += blockDim.x) {
            const int w = item[it];
            const int S = w & 1023, cnt = w >> 20;
            int Sp = (w >> 10) & 1023;
            // all of the item's LDS reads first (terms past cnt read entry 0 and are
            // skipped), then the multiply-adds on two independent accumulators
            E cv[CHAIN_CHUNK], qv[CHAIN_CHUNK];
#pragma unroll
            for (int k = 0; k < CHAIN_CHUNK; ++k) {
                const int s2 = k < cnt ? Sp : 0;
                cv[k] = pl_load<E, D>(c, csw(s2));
                qv[k] = qat(popc(s2) * D + idx(S ^ s2));
                Sp = (Sp - 1) & S;
            }
            E acc0 = T_::zero(), acc1 = T_::zero();
#pragma unroll
            for (int k = 0; k < CHAIN_CHUNK; k += 2) {
                if (k < cnt) acc0 = chain_mac(acc0, cv[k], qv[k]);
                if (k + 1 < cnt) acc1 = chain_mac(acc1, cv[k + 1], qv[k + 1]);
            }
            pl_store<E, MAXI>(part, it, xnorm(T_::add(xnorm(acc0), xnorm(acc1))));
        }
        lds_barrier();
        // the items of each state, four reads at a time
        for (int S = tid; S < D; S += blockDim.x) {
            const int b = ioff[S], e = ioff[S + 1];
            E acc = pl_load<E, MAXI>(part, b);
            for (int it = b + 1; it < e; it += 4) {
                E v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = (it + u < e) ? pl_load<E, MAXI>(part, it + u) : T_::zero();
                acc = T_::add(acc, T_::add(T_::add(v[0], v[1]), T_::add(v[2], v[3])));
            }
            pl_store<E, D>(c, csw(S), acc);
        }
        lds_barrier();
    }
}

// The product pass of one tile from its carries; the team's per-tile sum goes to
// part[j][t].
template <int L, typename E, int MODE>
__global__ __launch_bounds__(64) void k_tile_final(const Inst *I, const Ptrs *P, const TileInst *TI,
                                                   const TileTrack *Tr, const int2 *jobs, int njobs, int j,
                                                   int state_need)
{
    __shared__ __attribute__((aligned(16))) char lds[WShared<L>::TPWMAX * WShared<L>::BYTES];
    using W = WL<L, E>;
    constexpr int D = W::D;
    const int team = (int)threadIdx.x / W::TL;
    const int jid = (int)blockIdx.x * W::TPW + team;
    if (jid >= njobs) return;
    const int2 jb = jobs[jid];
    if (Tr && Tr[jb.x].state != state_need) return;
    const TileInst T = TI[jb.x];
    const Inst *In = &I[jb.x];
    const Ptrs Pp = P[jb.x];
    const int t = jb.y;
    const long p0 = (long)t * T.B, p1 = min(In->N, p0 + T.B);
    const WTeam<L, E> tm = make_team<L, E>(lds, T.ck + (long)t * T.ck_stride);
    const E *carry = reinterpret_cast<const E *>(T.carry);
    const WAcc r = wide_pass<L, E, MODE>(tm, In, j, Pp.a, Pp.log_u, Pp.out, p0, p1, carry + ((long)t * 2 + 0) * D,
                                         carry + ((long)t * 2 + 1) * D);
    if (tm.last) gst(&T.part[(long)j * T.ntile + t], (MODE == P_OBJECTIVE) ? In->h * xto_double(r.x) : r.s);
}

// After the update passes of a sweep: the estimate, then whether a residual
// check is due (same rule as the one-team solver).  One thread per instance.
template <int L>
__global__ void k_tile_ctrl_sweep(const Ptrs *P, const TileInst *TI, TileTrack *Tr, int count, RunOpts o)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    TileTrack &R = Tr[i];
    if (R.state != TS_SWEEP) return;
    const TileInst T = TI[i];
    double est = 0.0;
    for (int j = 0; j < L - 1; ++j)
        for (int t = 0; t < T.ntile; ++t) est += T.part[(long)j * T.ntile + t];
    const long itr_max = P[i].itr_cap > 0 ? P[i].itr_cap : o.itr_max;
    const int flags = o.flags | P[i].flags;
    R.it += 1;
    R.est = est;
    if (!(est == est)) {
        R.state = TS_DONE;
        R.status = ST_NUMERIC;
        return;
    }
    const bool chk = !(flags & F_NO_CHECK) && ((o.check_every > 0 && R.it % o.check_every == 0) ||
                                                R.it >= itr_max || (o.tol >= 0.0 && est <= o.tol * R.f));
    if (chk) R.state = TS_CHECK;
    else if (R.it >= itr_max) R.state = TS_DONE;
}

// After the check passes: the FP64 residual and the stopping decision.
template <int L>
__global__ void k_tile_ctrl_check(const Ptrs *P, const TileInst *TI, TileTrack *Tr, int count, RunOpts o)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    TileTrack &R = Tr[i];
    if (R.state != TS_CHECK) return;
    const TileInst T = TI[i];
    double res = 0.0;
    for (int j = 0; j < L - 1; ++j)
        for (int t = 0; t < T.ntile; ++t) res += T.part[(long)j * T.ntile + t];
    const long itr_max = P[i].itr_cap > 0 ? P[i].itr_cap : o.itr_max;
    R.res = res;
    R.checked = 1;
    if (!(res == res)) {
        R.state = TS_DONE;
        R.status = ST_NUMERIC;
    } else if (res <= o.tol || R.it >= itr_max) {
        R.state = TS_DONE;
        R.status = ST_OK;
    } else {
        if (o.tol >= 0.0 && R.est <= o.tol * R.f) R.f *= 0.5;
        R.state = TS_SWEEP;
    }
}

}  // namespace mmot
