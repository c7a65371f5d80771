// Per-l instantiation of the team-layout kernels (compiled once per l with
// -DMMOT_L=<l>) and their launchers.
#include <algorithm>

#include "launch.hpp"
#include "wide.hpp"

#ifndef MMOT_L
#error "compile with -DMMOT_L=<number of marginals>"
#endif

namespace mmot {

static __global__ void k_fill_int1(int *p, int v) { *p = v; }

template <int L>
static hipError_t wide_pass_t(int precision, int mode, const Inst *dI, const Ptrs &P, int j, double *dres,
                              hipStream_t s)
{
    const dim3 g(1), b(WAVE);
    switch (mode) {
        case P_PRODUCT:
            if (precision == 1)
                hipLaunchKernelGGL((k_wide_pass<L, XF<float>, P_PRODUCT>), g, b, 0, s, dI, P, j, dres);
            else
                hipLaunchKernelGGL((k_wide_pass<L, XF<double>, P_PRODUCT>), g, b, 0, s, dI, P, j, dres);
            break;
        case P_OBJECTIVE:
            hipLaunchKernelGGL((k_wide_pass<L, DXF, P_OBJECTIVE>), g, b, 0, s, dI, P, L - 1, dres);
            break;
        case P_CHECK:
            hipLaunchKernelGGL((k_wide_check_all<L>), g, b, 0, s, dI, P, dres);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
static hipError_t wide_batch_t(int precision, const Inst *dI, const Ptrs *dP, const int *dorder, int count,
                               const RunOpts &o, Result *dR, int *dticket, hipStream_t s)
{
    constexpr int tpw = WAVE / wide_tl(L);
    const int blocks = std::max(1, std::min((count + tpw - 1) / tpw, 8192));
    if (precision == 1)
        hipLaunchKernelGGL((k_wide_batch<L, float>), dim3(blocks), dim3(WAVE), 0, s, dI, dP, dorder, count, o, dR,
                           dticket);
    else
        hipLaunchKernelGGL((k_wide_batch<L, double>), dim3(blocks), dim3(WAVE), 0, s, dI, dP, dorder, count, o, dR,
                           dticket);
    // the objective of the solves that ended cleanly, in a launch of its own
    hipLaunchKernelGGL(k_fill_int1, dim3(1), dim3(1), 0, s, dticket, 0);
    hipLaunchKernelGGL((k_wide_objective<L>), dim3(blocks), dim3(WAVE), 0, s, dI, dP, dorder, count, o, dR, dticket);
    return hipGetLastError();
}

#define MMOT_CAT2(a, b) a##b
#define MMOT_CAT(a, b) MMOT_CAT2(a, b)

hipError_t MMOT_CAT(launch_wide_pass_l, MMOT_L)(int precision, int mode, const Inst *dI, const Ptrs &P, int j,
                                                 double *dres, hipStream_t s)
{
    return wide_pass_t<MMOT_L>(precision, mode, dI, P, j, dres, s);
}

hipError_t MMOT_CAT(launch_wide_batch_l, MMOT_L)(int precision, const Inst *dI, const Ptrs *dP, const int *dorder,
                                                  int count, const RunOpts &o, Result *dR, int *dticket, hipStream_t s)
{
    return wide_batch_t<MMOT_L>(precision, dI, dP, dorder, count, o, dR, dticket, s);
}

}  // namespace mmot
