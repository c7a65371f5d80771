// Device kernels of libmmot (templates; instantiated by k_single.hip and k_batch.hip).
//
// One wavefront works on one problem instance at a time (scan.hpp); a block of
// 256 threads is four independent wavefronts.  The solve kernels run the whole
// Gauss-Seidel iteration on the device: the l marginal updates of a sweep
// (Alg. 1 update lines, Sec. 4.2 update formulas), the FP64 residual every
// check_every sweeps (Alg. 1 Res line) and the FP64 objective at the end
// (Sec. 2 Eq. mmot distance).  The batch kernel is persistent: each wavefront
// takes the next instance from an atomic ticket until the list is exhausted.
#pragma once
#include <type_traits>

#include "fast.hpp"
#include "launch.hpp"
#include "scan.hpp"

namespace mmot {

// Whole solve of one instance on one wavefront.
template <int L, typename M>
__device__ void solve_one(const Inst *__restrict__ I, const Ptrs P, const RunOpts o, Result *__restrict__ R, int lane)
{
    constexpr int KU = std::is_same<M, float>::value ? 0 : 1;
    constexpr int VU = vsel(L, KU);
    constexpr int VC = vsel(L, 3);
    constexpr int VO = vsel(L, 2);
    const long N = I->N;
    double *a = P.a;
    const double *lu = P.log_u;
    const int flags = o.flags | P.flags;
    const long itr_max = P.itr_cap > 0 ? P.itr_cap : o.itr_max;

    if (!(flags & F_WARM) && P.it0 == 0) {
        // phi = 1/N (Alg. 1 initialisation)
        const double a0 = -log((double)N);
        for (long p = lane; p < (long)L * N; p += WAVE) a[p] = a0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    // a resumed solve finishes sweep it0 from marginal j0 first (j0 = l: only its check)
    long it = P.it0;
    int jr = P.j0;
    double res = INFINITY, f = 1.0;
    int status = ST_OK;
    bool checked = false;
    while (it < itr_max || jr > 0) {
        const bool resumed = jr > 0;
        if (!resumed) ++it;
        // est: marginal errors the updates of this sweep removed (j < l-1)
        double est = 0.0;
        for (int j = jr; j < L; ++j) {
            const double e =
                marginal_pass<L, VU, XF<M>, P_UPDATE>(I, upd_disc<L, M>(I), j, a, lu, nullptr, P.scratch, lane);
            if (j < L - 1) est += e;
        }
        jr = 0;
        const bool trig = !resumed && o.tol >= 0.0 && est <= o.tol * f;
        const bool chk = !(flags & F_NO_CHECK) &&
                         ((resumed && P.j0 == L) || (o.check_every > 0 && it % o.check_every == 0) ||
                          it >= itr_max || trig);
        if (chk) {
            checked = true;
            res = 0.0;
            for (int j = 0; j < L - 1; ++j)
                res += marginal_pass<L, VC, XF<double>, P_CHECK>(I, &I->dck, j, a, lu, nullptr, P.scratch, lane);
            if (!(res == res)) {
                status = ST_NUMERIC;
                break;
            }
            if (res <= o.tol) break;
            if (trig) f *= 0.5;
        }
    }
    double W = 0.0;
    if (status == ST_OK && !(flags & F_NO_OBJ)) {
        W = marginal_pass<L, VO, DXF, P_OBJECTIVE>(I, &I->dob, L - 1, a, lu, nullptr, P.scratch, lane);
        if (!(W == W) || W == INFINITY) status = ST_NUMERIC;
    }
    if (status == ST_OK && checked && o.tol >= 0.0 && !(res <= o.tol)) status = ST_NOT_CONVERGED;
    if (lane == 0) {
        R->W = W;
        R->marg_err = res;
        R->iters = it;
        R->status = status;
        R->l = L;
        R->N = N;
    }
}

template <int L, typename M>
__global__ __launch_bounds__(64, 2) void k_solve_single(const Inst *I, Ptrs P, RunOpts o, Result *R)
{
    solve_one<L, M>(I, P, o, R, threadIdx.x);
}

template <typename M>
__device__ void solve_dispatch(const Inst *I, const Ptrs P, const RunOpts o, Result *R, int lane)
{
    switch (I->l) {
        case 2: solve_one<2, M>(I, P, o, R, lane); break;
        case 3: solve_one<3, M>(I, P, o, R, lane); break;
        case 4: solve_one<4, M>(I, P, o, R, lane); break;
        case 5: solve_one<5, M>(I, P, o, R, lane); break;
        case 6: solve_one<6, M>(I, P, o, R, lane); break;
        default: break;  // l >= 7 runs on the team layout (wide.hpp)
    }
}

// Next instance ticket of a wavefront, the same value in every lane.  Every
// lane takes part in one atomic (lane 0 adds 1, the others 0) and the value
// lane 0 got is broadcast: no branch on the lane index precedes the
// broadcast.  (With the atomic under `if (lane == 0)` and a shuffle
// broadcast, the optimizer can send the other lanes round the loop past the
// atomic with a constant 0 as their shuffle input; they then take ticket 0
// forever and the wavefront never leaves the loop.)
__device__ __forceinline__ int wave_ticket(int *ticket, int lane)
{
    return __builtin_amdgcn_readfirstlane(atomicAdd(ticket, lane == 0 ? 1 : 0));
}

// Persistent batch: wavefronts pull instance tickets until none is left.
template <typename M>
__global__ __launch_bounds__(256, 2) void k_solve_batch(const Inst *I, const Ptrs *P, const int *order, int count,
                                                     RunOpts o, Result *R, int *ticket)
{
    const int lane = threadIdx.x & (WAVE - 1);
    for (;;) {
        const int t = wave_ticket(ticket, lane);
        if (t >= count) break;
        const int idx = __builtin_amdgcn_readfirstlane(order[t]);
        solve_dispatch<M>(&I[idx], P[idx], o, &R[idx], lane);
    }
}


template <int L, int V, typename E, int MODE>
__global__ __launch_bounds__(64) void k_pass(const Inst *I, Ptrs P, int j, double *result)
{
    const Disc<typename ET<E>::MT> *K;
    if constexpr (MODE == P_OBJECTIVE)
        K = &I->dob;
    else if constexpr (std::is_same<typename ET<E>::MT, float>::value)
        K = (const Disc<typename ET<E>::MT> *)&I->d32;
    else
        K = (const Disc<typename ET<E>::MT> *)&I->d64;
    const double r = marginal_pass<L, V, E, MODE>(I, K, j, P.a, P.log_u, P.out, P.scratch, threadIdx.x);
    if (threadIdx.x == 0 && result) result[0] = r;
}

template <int L>
__global__ __launch_bounds__(64) void k_check_all(const Inst *I, Ptrs P, double *err)
{
    constexpr int VC = vsel(L, 3);
    for (int j = 0; j < L; ++j) {
        const double r = marginal_pass<L, VC, XF<double>, P_CHECK>(I, &I->dck, j, P.a, P.log_u, nullptr, P.scratch,
                                                                  threadIdx.x);
        if (threadIdx.x == 0) err[j] = r;
    }
}

// Fast path, sweeps: each workgroup takes the next instance of the list (all
// have l = L and N <= blockDim.x * V) and, if its state is TS_SWEEP, runs
// fast_sweeps on it.
template <int L, int V, typename M>
__global__ __launch_bounds__(fast_threads(L, sizeof(M) == 4 ? 1 : 0))
__attribute__((amdgpu_waves_per_eu(fast_waves_per_eu(sizeof(M) == 4 ? 1 : 0)))) void k_fast_sweep(
    const Inst *I, const Ptrs *P, const int *list, int count, RunOpts o, Track *Tr, int *ticket)
{
    __shared__ FastShared<L, V, M> sh;
    __shared__ int tk;
    for (;;) {
        if (threadIdx.x == 0) tk = atomicAdd(ticket, 1);
        __syncthreads();
        const int t = tk;
        __syncthreads();
        if (t >= count) break;
        const int idx = list[t];
        if (Tr[idx].state == TS_SWEEP) fast_sweeps<L, V, M>(&I[idx], P[idx], o, &Tr[idx], sh);
        __syncthreads();
    }
}

// Fast path, FP64 residual checks of the instances in state TS_CHECK.
template <int L, int V>
__global__ __launch_bounds__(fast_threads(L, 0)) void k_fast_check(const Inst *I, const Ptrs *P, const int *list,
                                                                int count, RunOpts o, Track *Tr, int *ticket)
{
    __shared__ FastShared<L, V, double> sh;
    __shared__ int tk;
    for (;;) {
        if (threadIdx.x == 0) tk = atomicAdd(ticket, 1);
        __syncthreads();
        const int t = tk;
        __syncthreads();
        if (t >= count) break;
        const int idx = list[t];
        if (Tr[idx].state == TS_CHECK) fast_check<L, V>(&I[idx], P[idx], o, &Tr[idx], sh);
        __syncthreads();
    }
}

// FP64 objective (Sec. 2 Eq. mmot distance) of each listed instance, one
// wavefront per instance; writes Result.W only.
template <int L>
__device__ void objective_one(const Inst *I, const Ptrs P, Result *R, int lane)
{
    constexpr int VO = vsel(L, 2);
    const double W = marginal_pass<L, VO, DXF, P_OBJECTIVE>(I, &I->dob, L - 1, P.a, P.log_u, nullptr, P.scratch, lane);
    if (lane == 0) R->W = W;
}

}  // namespace mmot
