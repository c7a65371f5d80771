// The marginal product from its definition, on the device: the sum over all
// N^(l-1) index tuples of the other marginals of the Gibbs kernel times their
// scaling factors (Sec. 2, the tensor-vector product of the multi-marginal
// Sinkhorn update; Alg. 1 as written, O(N^l) per product).  It is the
// comparison point for the O(N) scans at small sizes, not part of their path.
//
// Work split: output position y = blockIdx.y; the N^(l-1) terms of y are cut
// into gridDim.x contiguous ranges, one per workgroup.  Each thread keeps a
// running log-sum-exp (m, s) over its terms (s rescaled when m grows), the
// workgroup combines its threads' pairs in LDS, and k_dense_finish combines
// the ranges of each y.  Every value is FP64.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dense.hpp"

namespace mmot {

namespace {

constexpr int DENSE_THREADS = 256;

struct LseAcc {
    double m, s;  // sum = s * exp(m); m = -inf: empty
};

__device__ __forceinline__ LseAcc lse_add(LseAcc a, double v)
{
    if (v == -INFINITY) return a;
    if (v <= a.m) return {a.m, a.s + exp(v - a.m)};
    return {v, a.s * exp(a.m - v) + 1.0};
}

__device__ __forceinline__ LseAcc lse_join(LseAcc a, LseAcc b)
{
    if (b.m == -INFINITY) return a;
    if (a.m == -INFINITY) return b;
    if (b.m <= a.m) return {a.m, a.s + b.s * exp(b.m - a.m)};
    return {b.m, b.s + a.s * exp(a.m - b.m)};
}

}  // namespace

// Rows of a (L x N, row j unused) and the node coordinates in LDS.  Uniform grid
// (x == nullptr): cost = (h / eps) * sum_{p<q} |i_p - i_q| with the integer index
// sum formed first; non-uniform: cost = sum_{p<q} |x_{i_p} - x_{i_q}| / eps.
template <int L>
__global__ __launch_bounds__(DENSE_THREADS) void k_dense_terms(const double *__restrict__ a, int N, int j, double hoe,
                                                              double ieps, const double *__restrict__ x,
                                                              unsigned terms, unsigned chunk,
                                                              double *__restrict__ part)
{
    extern __shared__ double lds[];
    double *rows = lds;              // [L][N]
    double *xs = lds + (long)L * N;  // [N] (non-uniform grid only)
    const int y = blockIdx.y;
    for (int p = threadIdx.x; p < L * N; p += blockDim.x) rows[p] = a[p];
    if (x)
        for (int p = threadIdx.x; p < N; p += blockDim.x) xs[p] = x[p];
    __syncthreads();

    const unsigned t0 = blockIdx.x * chunk;
    const unsigned t1 = t0 + chunk < terms ? t0 + chunk : terms;
    LseAcc acc = {-INFINITY, 0.0};
    for (unsigned t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        // digits of t in base N: the index of marginal q (q != j, in order)
        int idx[L];
        unsigned u = t;
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < L - 1; ++r) {
            const int q = r < j ? r : r + 1;
            const int i = (int)(u % (unsigned)N);
            u /= (unsigned)N;
            idx[r] = i;
            v += rows[q * N + i];
        }
        idx[L - 1] = y;
        if (x) {
            double c = 0.0;
#pragma unroll
            for (int p = 0; p < L; ++p)
#pragma unroll
                for (int q = p + 1; q < L; ++q) c += fabs(xs[idx[p]] - xs[idx[q]]);
            v -= c * ieps;
        } else {
            int e = 0;
#pragma unroll
            for (int p = 0; p < L; ++p)
#pragma unroll
                for (int q = p + 1; q < L; ++q) e += abs(idx[p] - idx[q]);
            v -= hoe * (double)e;
        }
        acc = lse_add(acc, v);
    }
    // workgroup: tree over the threads' pairs
    __shared__ double rm[DENSE_THREADS], rs[DENSE_THREADS];
    rm[threadIdx.x] = acc.m;
    rs[threadIdx.x] = acc.s;
    __syncthreads();
    for (int w = DENSE_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const LseAcc c = lse_join({rm[threadIdx.x], rs[threadIdx.x]}, {rm[threadIdx.x + w], rs[threadIdx.x + w]});
            rm[threadIdx.x] = c.m;
            rs[threadIdx.x] = c.s;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * ((long)y * gridDim.x + blockIdx.x)] = rm[0];
        part[2 * ((long)y * gridDim.x + blockIdx.x) + 1] = rs[0];
    }
}

// Per output y: log J_j(y) from the ranges' pairs.  out != nullptr: out[y] = log J;
// else the update a_j(y) = log u_j(y) - log J (zero mass keeps -inf).
__global__ void k_dense_finish(const double *__restrict__ part, int G, int N, double *out, double *a_j,
                               const double *__restrict__ lu_j)
{
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= N) return;
    LseAcc acc = {-INFINITY, 0.0};
    for (int g = 0; g < G; ++g) acc = lse_join(acc, {part[2 * ((long)y * G + g)], part[2 * ((long)y * G + g) + 1]});
    const double lj = acc.m == -INFINITY ? -INFINITY : acc.m + log(acc.s);
    if (out) {
        out[y] = lj;
    } else {
        const double lu = lu_j[y];
        a_j[y] = lu == -INFINITY ? -INFINITY : lu - lj;
    }
}

int dense_ranges(int N) { return std::max(1, std::min(DENSE_MAX_RANGES, (2048 + N - 1) / N)); }

bool dense_supported(int l, int64_t N)
{
    if (l < 2 || l > DENSE_MAXL || N < 1 || N * (l + 1) > DENSE_MAX_LDS_DOUBLES) return false;
    double terms = 1.0;
    for (int r = 0; r < l - 1; ++r) terms *= (double)N;
    return terms < 2147483648.0;
}

hipError_t launch_dense_product(int l, int N, int j, double hoe, double ieps, const double *x, const double *a,
                                double *out, double *a_j, const double *lu_j, double *part, hipStream_t s)
{
    if (!dense_supported(l, N) || j < 0 || j >= l) return hipErrorInvalidValue;
    unsigned terms = 1;
    for (int r = 0; r < l - 1; ++r) terms *= (unsigned)N;
    const int G = dense_ranges(N);
    const unsigned chunk = (terms + (unsigned)G - 1) / (unsigned)G;
    const size_t lds = sizeof(double) * ((size_t)l * N + (x ? (size_t)N : 0));
    const dim3 g(G, N), b(DENSE_THREADS);
    switch (l) {
        case 2: hipLaunchKernelGGL(k_dense_terms<2>, g, b, lds, s, a, N, j, hoe, ieps, x, terms, chunk, part); break;
        case 3: hipLaunchKernelGGL(k_dense_terms<3>, g, b, lds, s, a, N, j, hoe, ieps, x, terms, chunk, part); break;
        case 4: hipLaunchKernelGGL(k_dense_terms<4>, g, b, lds, s, a, N, j, hoe, ieps, x, terms, chunk, part); break;
        case 5: hipLaunchKernelGGL(k_dense_terms<5>, g, b, lds, s, a, N, j, hoe, ieps, x, terms, chunk, part); break;
        default: hipLaunchKernelGGL(k_dense_terms<6>, g, b, lds, s, a, N, j, hoe, ieps, x, terms, chunk, part); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dense_finish, dim3((N + 255) / 256), dim3(256), 0, s, part, G, N, out, a_j, lu_j);
    return hipGetLastError();
}

}  // namespace mmot
