// The dense (O(N^l)) marginal product on the device, for comparison with the
// O(N) scans (k_dense.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace mmot {

constexpr int DENSE_MAXL = 6;                // largest l of the dense product
constexpr int DENSE_MAX_RANGES = 64;         // workgroups per output position at most
constexpr int DENSE_MAX_LDS_DOUBLES = 6144;  // rows and coordinates staged in LDS: (l + 1) N doubles

// True if the dense product takes (l, N): l <= DENSE_MAXL, (l + 1) N doubles fit
// the LDS stage, N^(l-1) < 2^31 terms per output.
bool dense_supported(int l, int64_t N);
// Workgroups per output position (ranges of its terms).
int dense_ranges(int N);
// log J_j = log sum over the N^(l-1) index tuples of the other marginals of
// exp(sum_q a_q(i_q) - C / eps): into out[N] if out is not null, else the
// update a_j = lu_j - log J_j (zero mass keeps -inf).  a: device [l][N];
// x: device node coordinates or null (uniform grid, step h: hoe = h / eps);
// part: device workspace of 2 N dense_ranges(N) doubles.
hipError_t launch_dense_product(int l, int N, int j, double hoe, double ieps, const double *x, const double *a,
                                double *out, double *a_j, const double *lu_j, double *part, hipStream_t s);

}  // namespace mmot
