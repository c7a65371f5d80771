// Per-l instantiation of the single-instance kernels (compiled once per l with
// -DMMOT_L=<l>) and their launchers.
#include "kernels.hpp"

#ifndef MMOT_L
#error "compile with -DMMOT_L=<number of marginals>"
#endif

namespace mmot {

template <int L>
static hipError_t launch_pass_t(int precision, int mode, const Inst *dI, const Ptrs &P, int j, double *dres,
                                hipStream_t s)
{
    const dim3 g(1), b(WAVE);
    switch (mode) {
        case P_PRODUCT:
            if (precision == 1)
                hipLaunchKernelGGL((k_pass<L, vsel(L, 0), XF<float>, P_PRODUCT>), g, b, 0, s, dI, P, j, dres);
            else
                hipLaunchKernelGGL((k_pass<L, vsel(L, 1), XF<double>, P_PRODUCT>), g, b, 0, s, dI, P, j, dres);
            break;
        case P_OBJECTIVE:
            hipLaunchKernelGGL((k_pass<L, vsel(L, 2), DXF, P_OBJECTIVE>), g, b, 0, s, dI, P, L - 1, dres);
            break;
        case P_CHECK:
            hipLaunchKernelGGL((k_check_all<L>), g, b, 0, s, dI, P, dres);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
static hipError_t launch_single_t(int precision, const Inst *dI, const Ptrs &P, const RunOpts &o, Result *dR,
                                  hipStream_t s)
{
    if (precision == 1)
        hipLaunchKernelGGL((k_solve_single<L, float>), dim3(1), dim3(WAVE), 0, s, dI, P, o, dR);
    else
        hipLaunchKernelGGL((k_solve_single<L, double>), dim3(1), dim3(WAVE), 0, s, dI, P, o, dR);
    return hipGetLastError();
}

template <int L>
static hipError_t launch_fast_t(int kind, int precision, const Inst *dI, const Ptrs *dP, const int *dlist,
                                int count, const RunOpts &o, Track *dT, int *dticket, int blocks, int waves,
                                hipStream_t s)
{
    if constexpr (L > FAST_MAXL) {
        return hipErrorInvalidValue;
    } else {
    const dim3 g(blocks), b(WAVE * waves);
    if (kind == 1)
        hipLaunchKernelGGL((k_fast_check<L, fast_v(L, 0)>), g, b, 0, s, dI, dP, dlist, count, o, dT, dticket);
    else if (precision == 1)
        hipLaunchKernelGGL((k_fast_sweep<L, fast_v(L, 1), float>), g, b, 0, s, dI, dP, dlist, count, o, dT, dticket);
    else
        hipLaunchKernelGGL((k_fast_sweep<L, fast_v(L, 0), double>), g, b, 0, s, dI, dP, dlist, count, o, dT,
                           dticket);
    return hipGetLastError();
    }
}

#define MMOT_CAT2(a, b) a##b
#define MMOT_CAT(a, b) MMOT_CAT2(a, b)

hipError_t MMOT_CAT(launch_pass_l, MMOT_L)(int precision, int mode, const Inst *dI, const Ptrs &P, int j,
                                            double *dres, hipStream_t s)
{
    return launch_pass_t<MMOT_L>(precision, mode, dI, P, j, dres, s);
}

hipError_t MMOT_CAT(launch_single_l, MMOT_L)(int precision, const Inst *dI, const Ptrs &P, const RunOpts &o,
                                              Result *dR, hipStream_t s)
{
    return launch_single_t<MMOT_L>(precision, dI, P, o, dR, s);
}

hipError_t MMOT_CAT(launch_fast_l, MMOT_L)(int kind, int precision, const Inst *dI, const Ptrs *dP,
                                            const int *dlist, int count, const RunOpts &o, Track *dT, int *dticket,
                                            int blocks, int waves, hipStream_t s)
{
    return launch_fast_t<MMOT_L>(kind, precision, dI, dP, dlist, count, o, dT, dticket, blocks, waves, s);
}

}  // namespace mmot
