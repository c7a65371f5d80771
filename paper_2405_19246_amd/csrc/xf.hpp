// Device arithmetic on extended-range values (see XF in common.hpp) and on the
// pair (value, cost-weighted value) used for the objective.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace mmot {

constexpr double LN2_HI = 6.93147180369123816490e-01;  // high part, exact times small ints
constexpr double LN2_LO = 1.90821492927058770002e-10;
constexpr double LOG2E = 1.44269504088896338700e+00;

__device__ __forceinline__ float xldexp(float m, int e) { return __builtin_amdgcn_ldexpf(m, e); }
__device__ __forceinline__ double xldexp(double m, int e) { return __builtin_amdgcn_ldexp(m, e); }
__device__ __forceinline__ float xmant(float m) { return __builtin_amdgcn_frexp_mantf(m); }
__device__ __forceinline__ double xmant(double m) { return __builtin_amdgcn_frexp_mant(m); }
__device__ __forceinline__ int xexpo(float m) { return __builtin_amdgcn_frexp_expf(m); }
__device__ __forceinline__ int xexpo(double m) { return __builtin_amdgcn_frexp_exp(m); }
__device__ __forceinline__ float xexp_r(double r, float) { return expf((float)r); }
__device__ __forceinline__ double xexp_r(double r, double) { return exp(r); }
__device__ __forceinline__ double xlog_m(float m) { return (double)logf(m); }
__device__ __forceinline__ double xlog_m(double m) { return log(m); }

template <typename M>
__device__ __forceinline__ XF<M> xzero() { return {M(0), XF_ZERO_E}; }
template <typename M>
__device__ __forceinline__ XF<M> xone() { return {M(0.5), 1}; }

template <typename M>
__device__ __forceinline__ XF<M> xadd(XF<M> a, XF<M> b)
{
    const int e = max(a.e, b.e);
    const M m = xldexp(a.m, a.e - e) + xldexp(b.m, b.e - e);
    return {xmant(m), e + xexpo(m)};
}

template <typename M>
__device__ __forceinline__ XF<M> xmul(XF<M> a, XF<M> b)
{
    return {a.m * b.m, max(a.e + b.e, XF_ZERO_E)};
}

// exp(a) for a natural log a (FP64): round a / ln 2 to an integer k, reduce with
// a two-part ln 2, exponentiate the remainder in the mantissa precision.
template <typename M>
__device__ __forceinline__ XF<M> xfrom_log(double a)
{
    if (!(a > -1.0e15)) {
        if (a != a) return {M(NAN), 0};
        return xzero<M>();
    }
    if (!(a < 1.0e15)) return {M(NAN), 0};
    const double k = rint(a * LOG2E);
    double r = fma(-k, LN2_HI, a);
    r = fma(-k, LN2_LO, r);
    const M m = xexp_r(r, M(0));
    return {xmant(m), (int)k + xexpo(m)};
}

// exp(a) as a discount factor with a hi + lo mantissa (see XG).
template <typename M>
__device__ __forceinline__ XG<M> xg_from_log(double a)
{
    if (!(a > -1.0e15)) return {M(0), M(0), XF_ZERO_E, 0};
    const double k = rint(a * LOG2E);
    double r = fma(-k, LN2_HI, a);
    r = fma(-k, LN2_LO, r);
    const double v = exp(r);
    const int ev = xexpo(v);
    const double vm = xldexp(v, -ev);  // in [0.5, 1)
    const M hi = (M)vm;
    const M lo = (M)(vm - (double)hi);
    return {hi, lo, (int)k + ev, 0};
}

// x times a discount factor.
template <typename M>
__device__ __forceinline__ XF<M> xmulg(XF<M> x, XG<M> g)
{
    if constexpr (sizeof(M) == 4)
        return {fmaf(x.m, g.hi, x.m * g.lo), max(x.e + g.e, XF_ZERO_E)};
    else
        return {x.m * g.hi, max(x.e + g.e, XF_ZERO_E)};
}

// Natural log of an extended value, FP64.
template <typename M>
__device__ __forceinline__ double xto_log(XF<M> x)
{
    if (x.m == M(0)) return -INFINITY;
    const double e = (double)x.e;
    return fma(e, LN2_HI, fma(e, LN2_LO, xlog_m(x.m)));
}

// Natural log of m 2^e for an FP32 mantissa m (normal, > 0): the hardware
// base-2 logarithm of m plus e, times ln 2 in FP64.  Error about an ulp of m,
// the precision the FP32 products carry anyway.
__device__ __forceinline__ double xlog_hw(float m, int e)
{
    const double t = (double)__builtin_amdgcn_logf(m) + (double)e;
    return fma(t, LN2_HI, t * LN2_LO);
}

// exp(a) as an FP32 extended value: a log2(e) split in FP64 into an integer k
// and a fraction f in [-1/2, 1/2]; 2^f from the hardware base-2 exponential.
__device__ __forceinline__ XF<float> xfrom_log_hw(double a)
{
    if (!(a > -1.0e15)) {
        if (a != a) return {NAN, 0};
        return xzero<float>();
    }
    if (!(a < 1.0e15)) return {NAN, 0};
    const double t = a * LOG2E;
    const double k = rint(t);
    const float m = __builtin_amdgcn_exp2f((float)(t - k));
    return {xmant(m), (int)k + xexpo(m)};
}

template <typename M>
__device__ __forceinline__ double xto_double(XF<M> x)
{
    return xldexp((double)x.m, x.e);
}

// ---- cross-lane moves ----
__device__ __forceinline__ float rlane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int rlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double rlane(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Discount factors as plain values with a hi + lo mantissa (0 when they fall
// below the mantissa type's normal range: their contribution is negligible).
template <typename M>
struct GV {
    M hi, lo;
};

template <typename M>
__device__ __forceinline__ GV<M> gv_from_log(double a)
{
    const double v = exp(a);
    const M hi = (M)v;
    const M lo = (M)(v - (double)hi);
    constexpr double tiny = sizeof(M) == 4 ? 1.0e-37 : 1.0e-300;
    if (!(v > tiny)) return {M(0), M(0)};
    return {hi, lo};
}

template <typename M>
__device__ __forceinline__ M gmul(GV<M> g, M x, M add)
{
    return fma(x, g.hi, fma(x, g.lo, add));
}

// Extended value with a normalised mantissa; zero gets the zero exponent.
template <typename M>
__device__ __forceinline__ XF<M> xnorm(XF<M> x)
{
    if (x.m == M(0)) return xzero<M>();
    return {xmant(x.m), x.e + xexpo(x.m)};
}

// Block-floating-point row of scaling factors phi = exp(a) at a thread's V
// positions: mantissas m[v] (relative to 2^e) and the exponent e; returns the
// exponent spread of the finite entries (0 if none).
template <typename M, int V>
__device__ __forceinline__ int bf_row(const double (&a)[V], M (&m)[V], int &e)
{
    XF<M> x[V];
    int hi = XF_ZERO_E, lo = -XF_ZERO_E;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        if constexpr (sizeof(M) == 4)
            x[v] = xfrom_log_hw(a[v]);
        else
            x[v] = xfrom_log<M>(a[v]);
        if (x[v].m != M(0)) {
            hi = max(hi, x[v].e);
            lo = min(lo, x[v].e);
        }
    }
    e = hi;
#pragma unroll
    for (int v = 0; v < V; ++v) m[v] = xldexp(x[v].m, x[v].e - hi);
    return hi >= lo ? hi - lo : 0;
}


// DPP lane moves (GFX9 controls, checked on the device): lanes without a
// source lane, or in rows outside ROWMASK, get `old`.
//   0x101..0x108 row_shl:1..8 and 0x111..0x118 row_shr:1..8 (within rows of 16
//   lanes), 0x130 wave_shl:1, 0x138 wave_shr:1, 0x142 row_bcast:15 (lane 15 of
//   each row to the next row), 0x143 row_bcast:31 (lane 31 to rows 2 and 3).
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ int dpp_i(int old, int x)
{
    return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ float dpp_m(float x)
{
    return __int_as_float(dpp_i<CTRL, ROWMASK>(0, __float_as_int(x)));
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_m(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i<CTRL, ROWMASK>(0, (int)(b & 0xffffffffLL));
    const int hi = dpp_i<CTRL, ROWMASK>(0, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Lane-scan element: an extended value with a biased exponent (XF exponent +
// XB_BIAS, so that the zero value is (0, 0)) and a mantissa left unnormalized
// between the steps of one scan (each step at most doubles it, so it stays far
// inside the mantissa type's range).  Lanes without a source lane then read an
// exact zero from DPP moves with bound_ctrl set.
constexpr int XB_BIAS = -XF_ZERO_E;
template <typename M>
struct XB {
    M m;
    int e;
};

template <typename M>
__device__ __forceinline__ XB<M> xb_of(XF<M> x)  // x normalized (zero: XF_ZERO_E)
{
    return {x.m, x.e + XB_BIAS};
}

template <typename M>
__device__ __forceinline__ XF<M> xf_of(XB<M> x)
{
    if (x.m == M(0)) return xzero<M>();
    return {xmant(x.m), x.e - XB_BIAS + xexpo(x.m)};
}

// DPP move with full row and bank masks; lanes without a source read 0.
template <int CTRL>
__device__ __forceinline__ int dpp_z(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_z(float x)
{
    return __int_as_float(dpp_z<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_z(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp_z<CTRL>((int)(b & 0xffffffffLL));
    const int hi = dpp_z<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, typename M>
__device__ __forceinline__ XB<M> dpp_xb(XB<M> x)
{
    return {dpp_z<CTRL>(x.m), dpp_z<CTRL>(x.e)};
}
// Row broadcasts (partial row masks: the rows left out read zero).
template <int CTRL, int ROWMASK, typename M>
__device__ __forceinline__ XB<M> dpp_xb_rows(XB<M> x)
{
    return {dpp_m<CTRL, ROWMASK>(x.m), dpp_i<CTRL, ROWMASK>(0, x.e)};
}

template <typename M>
__device__ __forceinline__ XB<M> rlane_xb(XB<M> x, int l)
{
    return {rlane(x.m, l), rlane(x.e, l)};
}

// x + g o: g a discount factor (at most 1, so a zero o keeps an exponent at
// most 1, below every live value's).
template <typename M>
__device__ __forceinline__ XB<M> xb_addg(XB<M> x, XB<M> o, XG<M> g)
{
    const M om = fma(o.m, g.hi, o.m * g.lo);
    const int oe = o.e + g.e;
    const int e = max(x.e, oe);
    return {xldexp(x.m, x.e - e) + xldexp(om, oe - e), e};
}

// Inclusive scan of per-lane aggregates towards higher lanes under the
// operator (a over w positions) . b = g^(V w) a + b, DPP moves only: shifts by
// 1, 2, 4, 8 inside rows of 16 lanes, then lane 15 of each row to the next row
// and lane 31 to the upper half.  gstep[s] = g^(V 2^s); glane[s] = g^(V s).
template <typename M>
__device__ __forceinline__ XB<M> ks_up_dpp(XB<M> x, const XG<M> *gstep, const XG<M> *glane, int lane)
{
    x = xb_addg(x, dpp_xb<0x111>(x), gstep[0]);
    x = xb_addg(x, dpp_xb<0x112>(x), gstep[1]);
    x = xb_addg(x, dpp_xb<0x114>(x), gstep[2]);
    x = xb_addg(x, dpp_xb<0x118>(x), gstep[3]);
    x = xb_addg(x, dpp_xb_rows<0x142, 0xA>(x), glane[(lane & 15) + 1]);
    x = xb_addg(x, dpp_xb_rows<0x143, 0xC>(x), glane[lane >= 32 ? lane - 31 : 0]);
    return x;
}

// The same scan towards lower lanes: shifts inside rows of 16 lanes, then the
// totals from the first lane of rows 1, 2, 3 to the last lane (read as
// wavefront-uniform values) carried into the rows below.
template <typename M>
__device__ __forceinline__ XB<M> ks_down_dpp(XB<M> x, const XG<M> *gstep, const XG<M> *glane, int lane)
{
    x = xb_addg(x, dpp_xb<0x101>(x), gstep[0]);
    x = xb_addg(x, dpp_xb<0x102>(x), gstep[1]);
    x = xb_addg(x, dpp_xb<0x104>(x), gstep[2]);
    x = xb_addg(x, dpp_xb<0x108>(x), gstep[3]);
    const XB<M> t3 = rlane_xb(x, 48);
    const XB<M> t2 = xb_addg(rlane_xb(x, 32), t3, glane[16]);
    const XB<M> t1 = xb_addg(rlane_xb(x, 16), t2, glane[16]);
    const int r = lane >> 4;
    const XB<M> t = r == 0 ? t1 : r == 1 ? t2 : r == 2 ? t3 : XB<M>{M(0), 0};
    return xb_addg(x, t, glane[16 - (lane & 15)]);
}


// ---- element kinds used by the scans ----
// XF<M>: plain value.  DXF: (value, cost-weighted value) for the objective.
struct DXF {
    XF<double> v;
    XF<double> w;
};

template <typename E>
struct ET;

template <typename M>
struct ET<XF<M>> {
    using MT = M;
    using El = XF<M>;
    static __device__ __forceinline__ El zero() { return xzero<M>(); }
    static __device__ __forceinline__ El one() { return xone<M>(); }
    static __device__ __forceinline__ El add(El a, El b) { return xadd(a, b); }
    // times a scalar value (a product of scaling factors)
    static __device__ __forceinline__ El scale(El a, XF<M> s) { return xmul(a, s); }
    // across p gaps at level k: times g(k)^p; the weighted count p * k (l - k) is unused
    static __device__ __forceinline__ El disc(El a, XG<M> gp, double) { return xmulg(a, gp); }
    static __device__ __forceinline__ El prod(El a, El b) { return xmul(a, b); }
    static __device__ __forceinline__ El shup(El a, int d) { return {__shfl_up(a.m, d), __shfl_up(a.e, d)}; }
    static __device__ __forceinline__ El shdn(El a, int d) { return {__shfl_down(a.m, d), __shfl_down(a.e, d)}; }
    static __device__ __forceinline__ El rl(El a, int l) { return {rlane(a.m, l), rlane(a.e, l)}; }
};

__device__ __forceinline__ XF<double> xfrom_small(double c)
{
    return {xmant(c), c == 0.0 ? XF_ZERO_E : xexpo(c)};
}

template <>
struct ET<DXF> {
    using MT = double;
    using El = DXF;
    using P = ET<XF<double>>;
    static __device__ __forceinline__ El zero() { return {xzero<double>(), xzero<double>()}; }
    static __device__ __forceinline__ El one() { return {xone<double>(), xzero<double>()}; }
    static __device__ __forceinline__ El add(El a, El b) { return {xadd(a.v, b.v), xadd(a.w, b.w)}; }
    static __device__ __forceinline__ El scale(El a, XF<double> s) { return {xmul(a.v, s), xmul(a.w, s)}; }
    // crossing p gaps with k(l-k) separated pairs each adds p*k(l-k) times the
    // value to the weighted part, then both parts take the factor g(k)^p
    static __device__ __forceinline__ El disc(El a, XG<double> gp, double pc)
    {
        const XF<double> w = (pc == 0.0) ? a.w : xadd(a.w, xmul(a.v, xfrom_small(pc)));
        return {xmulg(a.v, gp), xmulg(w, gp)};
    }
    static __device__ __forceinline__ El prod(El a, El b)
    {
        return {xmul(a.v, b.v), xadd(xmul(a.v, b.w), xmul(a.w, b.v))};
    }
    static __device__ __forceinline__ El shup(El a, int d) { return {P::shup(a.v, d), P::shup(a.w, d)}; }
    static __device__ __forceinline__ El shdn(El a, int d) { return {P::shdn(a.v, d), P::shdn(a.w, d)}; }
    static __device__ __forceinline__ El rl(El a, int l) { return {P::rl(a.v, l), P::rl(a.w, l)}; }
};

// ---- global memory through global-address-space pointers -------------------------
// A load or store through a generic pointer compiles to a flat instruction, which
// also counts against the LDS wait counter: every LDS read after it would wait for
// the global access to land.  The walks' global accesses go through these.
template <typename T>
__device__ __forceinline__ T gld(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ void gst(T *p, T v)
{
    *(__attribute__((address_space(1))) T *)p = v;
}
// element kinds (XF, DXF) word by word
template <typename E>
__device__ __forceinline__ E gld_e(const E *p)
{
    E v;
    int *d = reinterpret_cast<int *>(&v);
    const __attribute__((address_space(1))) int *q = (const __attribute__((address_space(1))) int *)p;
#pragma unroll
    for (int w = 0; w < (int)(sizeof(E) / 4); ++w) d[w] = q[w];
    return v;
}
template <typename E>
__device__ __forceinline__ void gst_e(E *p, E v)
{
    const int *d = reinterpret_cast<const int *>(&v);
    __attribute__((address_space(1))) int *q = (__attribute__((address_space(1))) int *)p;
#pragma unroll
    for (int w = 0; w < (int)(sizeof(E) / 4); ++w) q[w] = d[w];
}

// Workgroup barrier ordering LDS only (as team_sync, for a whole workgroup).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace mmot
