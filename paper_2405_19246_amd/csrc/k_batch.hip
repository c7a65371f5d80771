// The persistent mixed-l batch kernels and the launch dispatchers.
#include <algorithm>

#include "kernels.hpp"
#include "wide.hpp"

namespace mmot {

__global__ void k_fill_int(int *p, int v) { *p = v; }

__global__ void k_zero_int(int *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// One block per (instance, row): compensated per-thread sums of exp(log u),
// then a tree over the block.
__global__ __launch_bounds__(256) void k_check_marginals(const Inst *I, const Ptrs *P, int count, int *flags)
{
    const int i = blockIdx.x, q = blockIdx.y;
    if (i >= count || q >= I[i].l) return;
    const long N = I[i].N;
    const double *lu = P[i].log_u + (long)q * N;
    __shared__ double red[256];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    double s = 0.0, c = 0.0;
    int b = 0;
    for (long p = threadIdx.x; p < N; p += blockDim.x) {
        const double x = lu[p];
        if (x != x || x == INFINITY) b = 1;
        const double y = exp(x) - c;
        const double t = s + y;
        c = (t - s) - y;
        s = t;
    }
    // the coordinates of a non-uniform grid: finite and non-decreasing
    const double *xs = I[i].x;
    if (q == 0 && xs)
        for (long p = threadIdx.x; p < N; p += blockDim.x) {
            const double x = xs[p];
            if (!(x - x == 0.0) || (p > 0 && !(x >= xs[p - 1]))) b |= 4;
        }
    if (b) atomicOr(&bad, b);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int f = bad;
        if (!(fabs(red[0] - 1.0) <= 1e-12)) f |= 2;
        if (f) atomicOr(&flags[i], f);
    }
}

// All-marginals (Jacobi) sweep, second half: with log J_j of every marginal from
// the potentials at the start of the sweep, a_j <- a_j + (log u_j - a_j - log J_j) / l
// (zero mass keeps a_j = -inf).  n = l N entries, row-major [l][N] like a.
__global__ void k_jacobi_update(double *a, const double *log_u, const double *logJ, long n, double inv_l)
{
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const double lu = log_u[p];
        a[p] = (lu == -INFINITY) ? -INFINITY : a[p] + (lu - a[p] - logJ[p]) * inv_l;
    }
}

__global__ void k_fill_f64(double *a, long n, double v)
{
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) a[p] = v;
}

hipError_t launch_jacobi_update(double *a, const double *log_u, const double *logJ, long n, int l, hipStream_t s)
{
    const int blocks = (int)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_jacobi_update, dim3(blocks), dim3(256), 0, s, a, log_u, logJ, n, 1.0 / (double)l);
    return hipGetLastError();
}

hipError_t launch_fill(double *a, long n, double v, hipStream_t s)
{
    const int blocks = (int)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(256), 0, s, a, n, v);
    return hipGetLastError();
}

hipError_t launch_check_marginals(const Inst *dI, const Ptrs *dP, int count, int *dflags, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_int, dim3(std::min((count + 255) / 256, 1024)), dim3(256), 0, s, dflags, count);
    hipLaunchKernelGGL(k_check_marginals, dim3(count, MAXL), dim3(256), 0, s, dI, dP, count, dflags);
    return hipGetLastError();
}

// phi = 1/N (Alg. 1 initialisation) for the listed instances that do not start warm.
__global__ void k_tile_init(const Inst *I, const Ptrs *P, const int *list, int count, RunOpts o)
{
    if ((int)blockIdx.y >= count) return;
    const int i = list[blockIdx.y];
    if ((o.flags | P[i].flags) & F_WARM) return;
    const long n = (long)I[i].l * I[i].N;
    const double a0 = -log((double)I[i].N);
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) P[i].a[p] = a0;
}

__global__ __launch_bounds__(256) void k_objective_batch(const Inst *I, const Ptrs *P, const int *list, int count,
                                                         Result *R, int *ticket)
{
    const int lane = threadIdx.x & (WAVE - 1);
    for (;;) {
        const int t = wave_ticket(ticket, lane);
        if (t >= count) break;
        const int idx = __builtin_amdgcn_readfirstlane(list[t]);
        switch (I[idx].l) {
            case 2: objective_one<2>(&I[idx], P[idx], &R[idx], lane); break;
            case 3: objective_one<3>(&I[idx], P[idx], &R[idx], lane); break;
            case 4: objective_one<4>(&I[idx], P[idx], &R[idx], lane); break;
            case 5: objective_one<5>(&I[idx], P[idx], &R[idx], lane); break;
            case 6: objective_one<6>(&I[idx], P[idx], &R[idx], lane); break;
            default: break;
        }
    }
}


// Predicted sweeps a solve still needs after a warm-up round of `warmup` sweeps:
// the estimate fell from est_mid to est over the round's second half; at the same
// geometric rate it reaches tol * f after log(est / (tol f)) / rate more sweeps.
// Solves not sweeping come last (-1); an estimate that did not fall ranks first.
__device__ __forceinline__ double remaining_sweeps_dev(const Track &T, double tol, int warmup)
{
    if (T.state != TS_SWEEP) return -1.0;
    const double tgt = tol * T.f;
    if (!(T.est > tgt)) return 0.0;
    if (!(T.est_mid > T.est) || !(T.est > 0.0)) return INFINITY;
    const double rate = log(T.est_mid / T.est) / (double)(warmup / 2);
    return log(T.est / fmax(tgt, 1e-300)) / rate;
}

// One workgroup: bitonic sort of (predicted remaining sweeps, position) in LDS,
// longest first and positions ascending among equal keys (the host's stable
// order), then list rewritten in that order.
__global__ __launch_bounds__(1024) void k_fast_order(const Track *T, int *list, int n, double tol, int warmup)
{
    __shared__ double key[FAST_ORDER_MAX];
    __shared__ int pos[FAST_ORDER_MAX];
    int P = 1;
    while (P < n) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const double r = i < n ? remaining_sweeps_dev(T[list[i]], tol, warmup) : -INFINITY;
        key[i] = r == r ? r : INFINITY;
        pos[i] = i;
    }
    __syncthreads();
    // a comes after b: smaller key, or the same key and a later position
    auto after = [&](int a, int b) { return key[a] < key[b] || (key[a] == key[b] && pos[a] > pos[b]); };
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int x = i ^ j;
                if (x > i) {
                    const bool up = (i & k) == 0;
                    if (up ? after(i, x) : after(x, i)) {
                        const double tk = key[i];
                        key[i] = key[x];
                        key[x] = tk;
                        const int tp = pos[i];
                        pos[i] = pos[x];
                        pos[x] = tp;
                    }
                }
            }
            __syncthreads();
        }
    }
    // every read of the old order before any write (n <= 4 * blockDim.x)
    int v[FAST_ORDER_MAX / 1024];
#pragma unroll
    for (int r = 0; r < FAST_ORDER_MAX / 1024; ++r) {
        const int i = threadIdx.x + r * 1024;
        v[r] = i < n ? list[pos[i]] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < FAST_ORDER_MAX / 1024; ++r) {
        const int i = threadIdx.x + r * 1024;
        if (i < n) list[i] = v[r];
    }
}

hipError_t launch_fast_order(const Track *dT, int *list, int n, double tol, int warmup, hipStream_t s)
{
    if (n < 1 || n > FAST_ORDER_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fast_order, dim3(1), dim3(1024), 0, s, dT, list, n, tol, warmup);
    return hipGetLastError();
}

hipError_t launch_solve_batch(int precision, const Inst *dI, const Ptrs *dP, const int *dorder, int count,
                              const RunOpts &o, Result *dR, int *dticket, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, dticket, 0);
    if (precision == 1)
        hipLaunchKernelGGL((k_solve_batch<float>), dim3(blocks), dim3(256), 0, s, dI, dP, dorder, count, o, dR,
                           dticket);
    else
        hipLaunchKernelGGL((k_solve_batch<double>), dim3(blocks), dim3(256), 0, s, dI, dP, dorder, count, o, dR,
                           dticket);
    return hipGetLastError();
}

#define MMOT_DISPATCH(fn, l, ...)                   \
    switch (l) {                                    \
        case 2: return fn##2(__VA_ARGS__);          \
        case 3: return fn##3(__VA_ARGS__);          \
        case 4: return fn##4(__VA_ARGS__);          \
        case 5: return fn##5(__VA_ARGS__);          \
        case 6: return fn##6(__VA_ARGS__);          \
        default: return hipErrorInvalidValue;       \
    }

hipError_t launch_fast(int kind, int l, int precision, const Inst *dI, const Ptrs *dP, const int *dlist, int count,
                       const RunOpts &o, Track *dT, int *dticket, int blocks, int waves, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, dticket, 0);
    MMOT_DISPATCH(launch_fast_l, l, kind, precision, dI, dP, dlist, count, o, dT, dticket, blocks, waves, s)
}

hipError_t launch_objective_batch(const Inst *dI, const Ptrs *dP, const int *dlist, int count, Result *dR,
                                  int *dticket, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, dticket, 0);
    const int blocks = std::max(1, std::min((count + 3) / 4, 4096));
    hipLaunchKernelGGL(k_objective_batch, dim3(blocks), dim3(256), 0, s, dI, dP, dlist, count, dR, dticket);
    return hipGetLastError();
}

hipError_t launch_pass(int l, int precision, int mode, const Inst *dI, const Ptrs &P, int j, double *dres,
                       hipStream_t s)
{
    switch (l) {
        case 7: return launch_wide_pass_l7(precision, mode, dI, P, j, dres, s);
        case 8: return launch_wide_pass_l8(precision, mode, dI, P, j, dres, s);
        case 9: return launch_wide_pass_l9(precision, mode, dI, P, j, dres, s);
        case 10: return launch_wide_pass_l10(precision, mode, dI, P, j, dres, s);
        default: break;
    }
    MMOT_DISPATCH(launch_pass_l, l, precision, mode, dI, P, j, dres, s)
}

#define MMOT_DISPATCH_T(fn, l, ...)              \
    switch (l) {                                  \
        case 2: return fn##2(__VA_ARGS__);        \
        case 3: return fn##3(__VA_ARGS__);        \
        case 4: return fn##4(__VA_ARGS__);        \
        case 5: return fn##5(__VA_ARGS__);        \
        case 6: return fn##6(__VA_ARGS__);        \
        case 7: return fn##7(__VA_ARGS__);        \
        case 8: return fn##8(__VA_ARGS__);        \
        case 9: return fn##9(__VA_ARGS__);        \
        case 10: return fn##10(__VA_ARGS__);      \
        default: return hipErrorInvalidValue;     \
    }

hipError_t launch_tile_pass(int l, int precision, int mode, const Inst *dI, const Ptrs *dP, const TileInst *dTI,
                            const TileTrack *dTr, const TileJobs &J, int j, int state_need, hipStream_t s)
{
    MMOT_DISPATCH_T(launch_tile_pass_l, l, precision, mode, dI, dP, dTI, dTr, J, j, state_need, s)
}

hipError_t launch_tile_ctrl(int l, int which, const Ptrs *dP, const TileInst *dTI, TileTrack *dTr, int count,
                            const RunOpts &o, hipStream_t s)
{
    MMOT_DISPATCH_T(launch_tile_ctrl_l, l, which, dP, dTI, dTr, count, o, s)
}

hipError_t launch_tile_init(const Inst *dI, const Ptrs *dP, const int *dlist, int count, const RunOpts &o,
                            hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_init, dim3(64, count), dim3(256), 0, s, dI, dP, dlist, count, o);
    return hipGetLastError();
}

hipError_t launch_wide_batch(int l, int precision, const Inst *dI, const Ptrs *dP, const int *dorder, int count,
                             const RunOpts &o, Result *dR, int *dticket, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, dticket, 0);
    switch (l) {
        case 7: return launch_wide_batch_l7(precision, dI, dP, dorder, count, o, dR, dticket, s);
        case 8: return launch_wide_batch_l8(precision, dI, dP, dorder, count, o, dR, dticket, s);
        case 9: return launch_wide_batch_l9(precision, dI, dP, dorder, count, o, dR, dticket, s);
        case 10: return launch_wide_batch_l10(precision, dI, dP, dorder, count, o, dR, dticket, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve_single(int l, int precision, const Inst *dI, const Ptrs &P, const RunOpts &o, Result *dR,
                               hipStream_t s)
{
    MMOT_DISPATCH(launch_single_l, l, precision, dI, P, o, dR, s)
}

}  // namespace mmot
