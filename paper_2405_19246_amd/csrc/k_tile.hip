// Per-l instantiation of the tiled kernels (compiled once per l with
// -DMMOT_L=<l>) and their launchers.
#include <algorithm>

#include "launch.hpp"
#include "wide.hpp"

#ifndef MMOT_L
#error "compile with -DMMOT_L=<number of marginals>"
#endif

namespace mmot {

template <int L, typename E, int MODE>
static hipError_t tile_pass_t(const Inst *dI, const Ptrs *dP, const TileInst *dTI, const TileTrack *dTr,
                              const TileJobs &J, int j, int state_need, hipStream_t s)
{
    constexpr int tpw = WAVE / wide_tl(L);
    if (J.n1 > 0)
        hipLaunchKernelGGL((k_tile_agg<L, E>), dim3((J.n1 + tpw - 1) / tpw), dim3(WAVE), 0, s, dI, dP, dTI, dTr,
                           J.agg, J.n1, j, state_need);
    if (J.n2 > 0)
        hipLaunchKernelGGL((k_tile_chain<L, E>), dim3(J.n2), dim3(CHAIN_THREADS), 0, s, dTI, dTr, J.chain, J.n2,
                           state_need);
    if (J.n3 > 0)
        hipLaunchKernelGGL((k_tile_final<L, E, MODE>), dim3((J.n3 + tpw - 1) / tpw), dim3(WAVE), 0, s, dI, dP, dTI,
                           dTr, J.fin, J.n3, j, state_need);
    return hipGetLastError();
}

template <int L>
static hipError_t tile_pass_l(int precision, int mode, const Inst *dI, const Ptrs *dP, const TileInst *dTI,
                              const TileTrack *dTr, const TileJobs &J, int j, int state_need, hipStream_t s)
{
    switch (mode) {
        case P_PRODUCT:
            return precision == 1 ? tile_pass_t<L, XF<float>, P_PRODUCT>(dI, dP, dTI, dTr, J, j, state_need, s)
                                  : tile_pass_t<L, XF<double>, P_PRODUCT>(dI, dP, dTI, dTr, J, j, state_need, s);
        case P_UPDATE:
            return precision == 1 ? tile_pass_t<L, XF<float>, P_UPDATE>(dI, dP, dTI, dTr, J, j, state_need, s)
                                  : tile_pass_t<L, XF<double>, P_UPDATE>(dI, dP, dTI, dTr, J, j, state_need, s);
        case P_CHECK:
            return tile_pass_t<L, XF<double>, P_CHECK>(dI, dP, dTI, dTr, J, j, state_need, s);
        case P_OBJECTIVE:
            return tile_pass_t<L, DXF, P_OBJECTIVE>(dI, dP, dTI, dTr, J, L - 1, state_need, s);
        default:
            return hipErrorInvalidValue;
    }
}

template <int L>
static hipError_t tile_ctrl_l(int which, const Ptrs *dP, const TileInst *dTI, TileTrack *dTr, int count,
                              const RunOpts &o, hipStream_t s)
{
    const dim3 g((count + 255) / 256), b(256);
    if (which == 0)
        hipLaunchKernelGGL((k_tile_ctrl_sweep<L>), g, b, 0, s, dP, dTI, dTr, count, o);
    else
        hipLaunchKernelGGL((k_tile_ctrl_check<L>), g, b, 0, s, dP, dTI, dTr, count, o);
    return hipGetLastError();
}

#define MMOT_CAT2(a, b) a##b
#define MMOT_CAT(a, b) MMOT_CAT2(a, b)

hipError_t MMOT_CAT(launch_tile_pass_l, MMOT_L)(int precision, int mode, const Inst *dI, const Ptrs *dP,
                                                 const TileInst *dTI, const TileTrack *dTr, const TileJobs &J, int j,
                                                 int state_need, hipStream_t s)
{
    return tile_pass_l<MMOT_L>(precision, mode, dI, dP, dTI, dTr, J, j, state_need, s);
}

hipError_t MMOT_CAT(launch_tile_ctrl_l, MMOT_L)(int which, const Ptrs *dP, const TileInst *dTI, TileTrack *dTr,
                                                 int count, const RunOpts &o, hipStream_t s)
{
    return tile_ctrl_l<MMOT_L>(which, dP, dTI, dTr, count, o, s);
}

}  // namespace mmot
