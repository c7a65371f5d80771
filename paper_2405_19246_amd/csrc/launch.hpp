// Host-side entry points into the device code (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

#ifndef MMOT_BUILD_MAXL
#define MMOT_BUILD_MAXL 10
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
                                  hipStream_t s);                                                        \
    hipError_t launch_fast_l##l(int kind, int precision, const Inst *dI, const Ptrs *dP, const int *dlist,    \
                                int count, const RunOpts &o, Track *dT, int *dticket, int blocks, int waves,   \
                                hipStream_t s);
MMOT_DECL_L(2)
MMOT_DECL_L(3)
MMOT_DECL_L(4)
MMOT_DECL_L(5)
MMOT_DECL_L(6)
#undef MMOT_DECL_L

// Job lists of the tiled launches (device arrays): agg (instance, tile, m,
// direction), chain (instance, direction), fin (instance, tile).
struct TileJobs {
    const int4 *agg;
    int n1;
    const int2 *chain;
    int n2;
    const int2 *fin;
    int n3;
};

#define MMOT_DECL_T(l)                                                                                          \
    hipError_t launch_tile_pass_l##l(int precision, int mode, const Inst *dI, const Ptrs *dP, const TileInst *dTI, \
                                     const TileTrack *dTr, const TileJobs &J, int j, int state_need,            \
                                     hipStream_t s);                                                            \
    hipError_t launch_tile_ctrl_l##l(int which, const Ptrs *dP, const TileInst *dTI, TileTrack *dTr, int count,   \
                                     const RunOpts &o, hipStream_t s);
MMOT_DECL_T(2)
MMOT_DECL_T(3)
MMOT_DECL_T(4)
MMOT_DECL_T(5)
MMOT_DECL_T(6)
MMOT_DECL_T(7)
MMOT_DECL_T(8)
MMOT_DECL_T(9)
MMOT_DECL_T(10)
#undef MMOT_DECL_T

// Tiled passes of marginal j (mode P_PRODUCT / P_UPDATE in the given precision,
// P_CHECK and P_OBJECTIVE in FP64) over the jobs of instances with this l; jobs
// of instances whose TileTrack.state differs from state_need do nothing
// (dTr NULL: every job runs).
hipError_t launch_tile_pass(int l, int precision, int mode, const Inst *dI, const Ptrs *dP, const TileInst *dTI,
                            const TileTrack *dTr, const TileJobs &J, int j, int state_need, hipStream_t s);
// which 0: estimate and check decision after a sweep; 1: residual and stop decision after a check.
hipError_t launch_tile_ctrl(int l, int which, const Ptrs *dP, const TileInst *dTI, TileTrack *dTr, int count,
                            const RunOpts &o, hipStream_t s);
// Marginal checks of `count` instances: flags[i] |= 1 if a log u entry of
// instance i is NaN or +inf, |= 2 if a row's mass differs from 1 by more than
// 1e-12 (FP64).  flags must be zero on entry.
hipError_t launch_check_marginals(const Inst *dI, const Ptrs *dP, int count, int *dflags, hipStream_t s);
// All-marginals sweep update from the l products of the sweep's starting potentials,
// and a constant fill (potentials phi = 1/N).
hipError_t launch_jacobi_update(double *a, const double *log_u, const double *logJ, long n, int l, hipStream_t s);
hipError_t launch_fill(double *a, long n, double v, hipStream_t s);
// Reorders list[0..n) (n <= FAST_ORDER_MAX) by the sweeps each solve is predicted to
// still need after a warm-up of `warmup` sweeps, longest first (ties keep their
// order); one workgroup, so the batch host needs no copy of the states for it.
hipError_t launch_fast_order(const Track *dT, int *list, int n, double tol, int warmup, hipStream_t s);

// phi = 1/N for the listed instances that do not start warm.
hipError_t launch_tile_init(const Inst *dI, const Ptrs *dP, const int *dlist, int count, const RunOpts &o,
                            hipStream_t s);

// Team-layout kernels (wide.hpp), l = WIDE_MINL .. WIDE_MAXL.
#define MMOT_DECL_W(l)                                                                                      \
    hipError_t launch_wide_pass_l##l(int precision, int mode, const Inst *dI, const Ptrs &P, int j, double *dres, \
                                     hipStream_t s);                                                        \
    hipError_t launch_wide_batch_l##l(int precision, const Inst *dI, const Ptrs *dP, const int *dorder, int count, \
                                      const RunOpts &o, Result *dR, int *dticket, hipStream_t s);
MMOT_DECL_W(7)
MMOT_DECL_W(8)
MMOT_DECL_W(9)
MMOT_DECL_W(10)
#undef MMOT_DECL_W

// Persistent batch of instances that all have l (>= WIDE_MINL): one team of
// lanes per instance, whole solves.  Resets *dticket first.
hipError_t launch_wide_batch(int l, int precision, const Inst *dI, const Ptrs *dP, const int *dorder, int count,
                             const RunOpts &o, Result *dR, int *dticket, hipStream_t s);

// Fast path over a list of instances that all have l and N <= waves * 64 * V:
// kind 0 runs the sweeps (V = fast_v(l, precision)), kind 1 the FP64 residual
// checks (V = fast_v(l, 0)).  Resets *dticket first.
hipError_t launch_fast(int kind, int l, int precision, const Inst *dI, const Ptrs *dP, const int *dlist, int count,
                       const RunOpts &o, Track *dT, int *dticket, int blocks, int waves, hipStream_t s);

// FP64 objective of each listed instance (Result.W only).  Resets *dticket first.
hipError_t launch_objective_batch(const Inst *dI, const Ptrs *dP, const int *dlist, int count, Result *dR,
                                  int *dticket, hipStream_t s);

hipError_t launch_solve_batch(int precision, const Inst *dI, const Ptrs *dP, const int *dorder, int count,
                              const RunOpts &o, Result *dR, int *dticket, int blocks, hipStream_t s);

}  // namespace mmot
