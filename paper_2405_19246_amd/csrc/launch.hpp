// Host-side entry points into the device code (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

#ifndef MMOT_BUILD_MAXL
#define MMOT_BUILD_MAXL 6
#endif

namespace mmot {

// mode: 0 product (plan precision), 2 FP64 errors of all marginals, 3 objective.
hipError_t launch_pass(int l, int precision, int mode, const Inst *dI, const Ptrs &P, int j, double *dres,
                       hipStream_t s);

hipError_t launch_solve_single(int l, int precision, const Inst *dI, const Ptrs &P, const RunOpts &o, Result *dR,
                               hipStream_t s);

#define MMOT_DECL_L(l)                                                                                  \
    hipError_t launch_pass_l##l(int precision, int mode, const Inst *dI, const Ptrs &P, int j, double *dres, \
                                hipStream_t s);                                                        \
    hipError_t launch_single_l##l(int precision, const Inst *dI, const Ptrs &P, const RunOpts &o, Result *dR, \
                                  hipStream_t s);
MMOT_DECL_L(2)
MMOT_DECL_L(3)
MMOT_DECL_L(4)
MMOT_DECL_L(5)
MMOT_DECL_L(6)
#undef MMOT_DECL_L

hipError_t launch_solve_batch(int precision, const Inst *dI, const Ptrs *dP, const int *dorder, int count,
                              const RunOpts &o, Result *dR, int *dticket, int blocks, hipStream_t s);

}  // namespace mmot
