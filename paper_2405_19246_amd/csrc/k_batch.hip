// The persistent mixed-l batch kernels and the launch dispatchers.
#include "kernels.hpp"

namespace mmot {

__global__ void k_fill_int(int *p, int v) { *p = v; }

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

hipError_t launch_pass(int l, int precision, int mode, const Inst *dI, const Ptrs &P, int j, double *dres,
                       hipStream_t s)
{
    MMOT_DISPATCH(launch_pass_l, l, precision, mode, dI, P, j, dres, s)
}

hipError_t launch_solve_single(int l, int precision, const Inst *dI, const Ptrs &P, const RunOpts &o, Result *dR,
                               hipStream_t s)
{
    MMOT_DISPATCH(launch_single_l, l, precision, dI, P, o, dR, s)
}

}  // namespace mmot
