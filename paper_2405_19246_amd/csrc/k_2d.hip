// Three marginals on an N x M grid with separable L1 cost (Sec. 4.1).
//
// The kernel is K = K_1 (x) K_2.  Along the second axis (index y = i2, M points)
// the gap form of K_2 holds as in 1-D: with l = 3 every gap with one or two of
// the marginals on its left costs g = lambda_2^2.  Walking y with the two summed
// marginals a, b of a product J_j (j the third), the states are N-vectors over
// the first axis (index x = i1):
//   F_y(a) = g F_{y-1}(a) + phi_a(., y)           (a placed at or left of y)
//   H_y(a) = g (H_{y+1}(a) + phi_a(., y))          (a placed at or right of y)
// and the same for b.  The states with both placed are N x N; they are only ever
// needed contracted with K_1 against x_j, which makes them N-vectors again
// (CF with both left, CH with both right).  Writing P(u, v) for the 1-D product
// K_1 x_{i1} u x_{j1} v along the first axis, bilinearity gives
//   CF_y = g CF_{y-1} + P(F_y(a), phi_b) + P(phi_a, g F_{y-1}(b))
//   CH_y = g (CH_{y+1} + P(B_y(a), phi_b) + P(phi_a, H_{y+1}(b))),  B_y(a) = H_{y+1}(a) + phi_a
//   J_j(., y) = CH_{y+1} + P(F_y(a), H_{y+1}(b)) + P(H_{y+1}(a), F_y(b)) + CF_y
// (phi at row y).  So one 2-D product is
//   1. per x, scans along y of the vector states (k2_scan_in);
//   2. 6 M independent 1-D products of length N (rows gathered by k2_gather,
//      then one wavefront each, k2_pass_many -- the one-wavefront scan kernels);
//   3. per x, the scans of CF and CH and the sum (k2_combine).
// Every value is a natural logarithm in FP64; sums are log-add-exp.
//
// The objective W = <C, T> splits as C = h1 E_1 + h2 E_2.  The first-axis part
// moves the y-scans of CF and CH onto the weight: sum_y <phi_j(y), CF_y> =
// sum_y <P_j(y), (terms of CF_y)> with P_j(y) = sum_{y' >= y} g^{y'-y} phi_j(y'),
// and sum_y <phi_j(y), CH_{y+1}> = sum_y <Q_j(y), (terms of CH_y / g)> with
// Q_j(y) = sum_{y' < y} g^{y-y'} phi_j(y'), so it is a sum of 6 M 1-D objectives
// (the DXF scans, h1 <w, (E_1 K_1) x u x v>) with those weights as third row.
// The second-axis part is the same computation on the transposed grid.

#include "kernels.hpp"

namespace mmot {

__device__ __forceinline__ double lae(double x, double y)
{
    const double m = fmax(x, y);
    if (m == -INFINITY) return -INFINITY;
    return m + log1p(exp(-fabs(x - y)));
}

// Per column x: the forward states F(a), F(b), g F_{y-1}(b), and the backward
// B(a), H_{y+1}(a), H_{y+1}(b).  A, B: [M][N] log phi of the two summed marginals.
__global__ void k2_scan_in(const double *__restrict__ A, const double *__restrict__ B, long N, int M, double lg,
                           double *Fa, double *Fb, double *gFbp, double *Ba, double *Hna, double *Hnb)
{
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    double fa = -INFINITY, fb = -INFINITY;
    for (int y = 0; y < M; ++y) {
        const long p = (long)y * N + x;
        gFbp[p] = fb + lg;
        fa = lae(fa + lg, A[p]);
        fb = lae(fb + lg, B[p]);
        Fa[p] = fa;
        Fb[p] = fb;
    }
    double ha = -INFINITY, hb = -INFINITY;
    for (int y = M - 1; y >= 0; --y) {
        const long p = (long)y * N + x;
        Hna[p] = ha;
        Hnb[p] = hb;
        const double ba = lae(ha, A[p]);
        Ba[p] = ba;
        ha = lg + ba;
        hb = lg + lae(hb, B[p]);
    }
}

// Per column x: the objective's weights P_j (inclusive, from the right) and Q_j
// (exclusive, from the left) of the row phi_j C.
__global__ void k2_scan_w(const double *__restrict__ C, long N, int M, double lg, double *Pj, double *Qj)
{
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    double p = -INFINITY;
    for (int y = M - 1; y >= 0; --y) {
        p = lae(p + lg, C[(long)y * N + x]);
        Pj[(long)y * N + x] = p;
    }
    double q = -INFINITY;
    for (int y = 0; y < M; ++y) {
        Qj[(long)y * N + x] = q;
        q = lg + lae(q, C[(long)y * N + x]);
    }
}

// Row sources of the 6 groups of 1-D products: rows 0 and 1 of group g at y are
// src[2 g][y] and src[2 g + 1][y]; row 2 is src[12 + g / 2][y] (the objective's
// weight) or zero.
struct Gather2 {
    const double *src[15];
};

// tri: [6][M][3][N]; instance g M + y holds rows (u, v, w) of one 1-D pass.
__global__ void k2_gather(Gather2 G, long N, int M, int with_weight, double *__restrict__ tri)
{
    const long total = 6L * M * 3 * N;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long x = e % N;
        const long rest = e / N;
        const int r = (int)(rest % 3);
        const long gy = rest / 3;
        const int y = (int)(gy % M), g = (int)(gy / M);
        double v = 0.0;
        if (r < 2) v = G.src[2 * g + r][(long)y * N + x];
        else if (with_weight) v = G.src[12 + g / 2][(long)y * N + x];
        tri[e] = v;
    }
}

// One 1-D three-marginal pass per wavefront: product of rows 0, 1 into out
// (P_PRODUCT), or the objective h1 <row 2, (E_1 K_1) x row 0 x row 1> into res.
template <int V, typename E, int MODE>
__global__ __launch_bounds__(64) void k2_pass_many(const Inst *I, const Ptrs *P, int count, double *res)
{
    const int b = blockIdx.x;
    if (b >= count) return;
    const Disc<typename ET<E>::MT> *K =
        (MODE == P_OBJECTIVE) ? (const Disc<typename ET<E>::MT> *)&I->dob : (const Disc<typename ET<E>::MT> *)&I->d64;
    const double r = marginal_pass<3, V, E, MODE>(I, K, 2, P[b].a, P[b].log_u, P[b].out, P[b].scratch, threadIdx.x);
    if (threadIdx.x == 0 && res) res[b] = r;
}

// Per column x: CF forward, then CH backward and J.  T: [6][M][N] log products.
// mode 0: out = log J; mode 1: a_j = log u_j - log J (zero mass keeps -inf).
__global__ void k2_combine(const double *__restrict__ T, long N, int M, double lg, double *CF, int mode,
                           double *out, const double *__restrict__ lu)
{
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    const long S = (long)M * N;
    double cf = -INFINITY;
    for (int y = 0; y < M; ++y) {
        const long p = (long)y * N + x;
        cf = lae(cf + lg, lae(T[p], T[S + p]));
        CF[p] = cf;
    }
    double ch = -INFINITY;  // CH_{y+1}
    for (int y = M - 1; y >= 0; --y) {
        const long p = (long)y * N + x;
        const double J = lae(lae(ch, T[4 * S + p]), lae(T[5 * S + p], CF[p]));
        if (mode == 0) out[p] = J;
        else out[p] = (lu[p] == -INFINITY) ? -INFINITY : lu[p] - J;
        ch = lg + lae(ch, lae(T[2 * S + p], T[3 * S + p]));
    }
}

// Block sums of |exp(a + logJ) - u| (u = exp(log u)); one partial per block.
__global__ __launch_bounds__(256) void k2_err(const double *__restrict__ a, const double *__restrict__ logJ,
                                              const double *__restrict__ lu, long n, double *partial)
{
    __shared__ double red[256];
    double s = 0.0;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x)
        s += fabs(exp(a[p] + logJ[p]) - exp(lu[p]));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[q][x][y] = in[q][y][x] for the three marginals.
__global__ void k2_transpose(const double *__restrict__ in, long N, int M, double *__restrict__ out)
{
    const long total = 3L * M * N;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long q = e / ((long)M * N), r = e % ((long)M * N);
        const long y = r / N, x = r % N;
        out[q * M * N + x * M + y] = in[e];
    }
}

static int cols(long N) { return (int)((N + 127) / 128); }

hipError_t launch2_scan_in(const double *A, const double *B, long N, int M, double lg, double *const bufs[6],
                           hipStream_t s)
{
    hipLaunchKernelGGL(k2_scan_in, dim3(cols(N)), dim3(128), 0, s, A, B, N, M, lg, bufs[0], bufs[1], bufs[2], bufs[3],
                       bufs[4], bufs[5]);
    return hipGetLastError();
}

hipError_t launch2_scan_w(const double *C, long N, int M, double lg, double *Pj, double *Qj, hipStream_t s)
{
    hipLaunchKernelGGL(k2_scan_w, dim3(cols(N)), dim3(128), 0, s, C, N, M, lg, Pj, Qj);
    return hipGetLastError();
}

hipError_t launch2_gather(const double *const src[15], long N, int M, int with_weight, double *tri, hipStream_t s)
{
    Gather2 G;
    for (int k = 0; k < 15; ++k) G.src[k] = src[k];
    const long total = 6L * M * 3 * N;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k2_gather, dim3(blocks), dim3(256), 0, s, G, N, M, with_weight, tri);
    return hipGetLastError();
}

hipError_t launch2_passes(int mode, const Inst *dI, const Ptrs *dP, int count, double *dres, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (mode == P_OBJECTIVE)
        hipLaunchKernelGGL((k2_pass_many<vsel(3, 2), DXF, P_OBJECTIVE>), dim3(count), dim3(WAVE), 0, s, dI, dP, count,
                           dres);
    else
        hipLaunchKernelGGL((k2_pass_many<vsel(3, 1), XF<double>, P_PRODUCT>), dim3(count), dim3(WAVE), 0, s, dI, dP,
                           count, dres);
    return hipGetLastError();
}

hipError_t launch2_combine(const double *T, long N, int M, double lg, double *CF, int mode, double *out,
                           const double *lu, hipStream_t s)
{
    hipLaunchKernelGGL(k2_combine, dim3(cols(N)), dim3(128), 0, s, T, N, M, lg, CF, mode, out, lu);
    return hipGetLastError();
}

hipError_t launch2_err(const double *a, const double *logJ, const double *lu, long n, double *partial, int blocks,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k2_err, dim3(blocks), dim3(256), 0, s, a, logJ, lu, n, partial);
    return hipGetLastError();
}

hipError_t launch2_transpose(const double *in, long N, int M, double *out, hipStream_t s)
{
    const long total = 3L * M * N;
    const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k2_transpose, dim3(blocks), dim3(256), 0, s, in, N, M, out);
    return hipGetLastError();
}

}  // namespace mmot
