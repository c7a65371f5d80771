// Host side of the tiled solver (wide.hpp): tile shapes, scratch layout, job
// lists, and the sweep loop of instances whose N is cut into tiles that run on
// many teams at once.
//
// A sweep of a group of instances with the same l is, for each marginal j, the
// three tiled launches of the update (aggregates, carry chain, final pass),
// then a controller launch that turns the per-tile sums into each instance's
// stopping estimate and decides whether a residual check is due; the check is
// the same three launches per j < l - 1 in FP64, then a controller that decides
// whether the instance stops.  Instances that stopped skip their jobs, so the
// host only looks at the states after a block of sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "launch.hpp"
#include "serve.hpp"
#include "tables.hpp"

namespace mmot {

namespace {
size_t r256(size_t n) { return (n + 255) & ~(size_t)255; }
}  // namespace

using namespace rt;

#define TCHK(call)                                                                                      \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return fail(MMOT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipError_t tile_buffers_reserve(BatchBuffers *bb, size_t jobs_bytes)
{
    if (jobs_bytes <= bb->jobs_cap) return hipSuccess;
    if (bb->djobs) (void)hipFree(bb->djobs);
    bb->djobs = nullptr;
    bb->jobs_cap = 0;
    const size_t cap = std::max<size_t>(jobs_bytes, 4096);
    hipError_t e = hipMalloc((void **)&bb->djobs, cap);
    if (e == hipSuccess) bb->jobs_cap = cap;
    return e;
}

// Job lists of the instances in g (all with the same l) laid out in one device
// buffer; returns the lists' device pointers.
hipError_t upload_jobs(const std::vector<int> &g, const std::vector<TileInst> &hTI, int l, BatchBuffers *bb,
                       hipStream_t s, std::vector<char> &host, TileJobs *J)
{
    std::vector<int4> j1;
    std::vector<int2> j2, j3;
    for (int i : g) {
        const int nt = hTI[i].ntile;
        if (nt > 1)
            for (int t = 0; t < nt; ++t)
                for (int m = 0; m < l; ++m)
                    for (int d = 0; d < 2; ++d) j1.push_back(make_int4(i, t, m, d));
        // the chain also writes the starting carries of a single tile
        j2.push_back(make_int2(i, 0));
        j2.push_back(make_int2(i, 1));
        for (int t = 0; t < nt; ++t) j3.push_back(make_int2(i, t));
    }
    const size_t b1 = r256(j1.size() * sizeof(int4)), b2 = r256(j2.size() * sizeof(int2)),
                 b3 = r256(j3.size() * sizeof(int2)) + 256;
    hipError_t e = tile_buffers_reserve(bb, b1 + b2 + b3 + g.size() * sizeof(int) + 256);
    if (e != hipSuccess) return e;
    host.assign(b1 + b2 + b3 + r256(g.size() * sizeof(int)), 0);
    std::memcpy(host.data(), j1.data(), j1.size() * sizeof(int4));
    std::memcpy(host.data() + b1, j2.data(), j2.size() * sizeof(int2));
    std::memcpy(host.data() + b1 + b2, j3.data(), j3.size() * sizeof(int2));
    std::memcpy(host.data() + b1 + b2 + b3, g.data(), g.size() * sizeof(int));
    e = hipMemcpyAsync(bb->djobs, host.data(), host.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    J->agg = reinterpret_cast<const int4 *>(bb->djobs);
    J->n1 = (int)j1.size();
    J->chain = reinterpret_cast<const int2 *>(bb->djobs + b1);
    J->n2 = (int)j2.size();
    J->fin = reinterpret_cast<const int2 *>(bb->djobs + b1 + b2);
    J->n3 = (int)j3.size();
    return hipSuccess;
}

const int *tile_group_list(const BatchBuffers *bb, const TileJobs &J)
{
    const size_t b1 = r256((size_t)J.n1 * sizeof(int4)), b2 = r256((size_t)J.n2 * sizeof(int2)),
                 b3 = r256((size_t)J.n3 * sizeof(int2)) + 256;
    return reinterpret_cast<const int *>(bb->djobs + b1 + b2 + b3);
}



// Autotuner of the tile length.  For an instance whose (l, ceil(log2 N)) class
// has no measured length yet: its potentials are initialised as the solve would
// (phi = 1/N unless warm), then one tiled FP64 check pass of marginal 0 runs at
// each candidate length (an eighth, a quarter, half, once and twice the rule's; warm-up run, then a run
// timed with HIP events on the stream), and the fastest is kept for the class.
static int tune_tile_length(int l, int i, int count, const Inst *hI, const Ptrs *hP, const RunOpts &o, int flags,
                            hipStream_t s, BatchBuffers *bb)
{
    int cand[5];
    const int k = tile_candidates(l, hI[i].N, flags | hP[i].flags, cand);
    if (k <= 1) {
        if (k == 1) tile_set_tuned(l, hI[i].N, cand[0]);
        return MMOT_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TCHK(hipEventCreate(&e0));
    TCHK(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } eg{e0, e1};
    std::vector<TileInst> hti(count);
    std::vector<char> jh;
    int best = cand[0];
    float best_ms = INFINITY;
    for (int c = 0; c < k; ++c) {
        const int B = cand[c];
        const int nt = (int)((hI[i].N + B - 1) / B);
        hti[i] = tile_inst(l, nt, B, reinterpret_cast<char *>(hP[i].scratch));
        TCHK(hipMemcpyAsync(bb->dTI + i, &hti[i], sizeof(TileInst), hipMemcpyHostToDevice, s));
        TileJobs J;
        TCHK(upload_jobs(std::vector<int>{i}, hti, l, bb, s, jh, &J));
        if (c == 0) TCHK(launch_tile_init(bb->dI, bb->dP, tile_group_list(bb, J), 1, o, s));
        TCHK(launch_tile_pass(l, 0, P_CHECK, bb->dI, bb->dP, bb->dTI, nullptr, J, 0, 0, s));
        TCHK(hipEventRecord(e0, s));
        TCHK(launch_tile_pass(l, 0, P_CHECK, bb->dI, bb->dP, bb->dTI, nullptr, J, 0, 0, s));
        TCHK(hipEventRecord(e1, s));
        TCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        TCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = B;
        }
    }
    tile_set_tuned(l, hI[i].N, best);
    return MMOT_OK;
}

static int tiled_group_solve_on(int l, const std::vector<int> &g, int count, const Inst *hI, const Ptrs *hP,
                                int precision, const RunOpts &o, int flags, hipStream_t s, BatchBuffers *bb,
                                Result *hR);

// The legacy default stream cannot be captured into a graph, so the tiled loop
// runs on a stream of the library's own (one per host thread, non-blocking,
// default priority), ordered after the caller's stream by an event and before
// its later work by another.
int tiled_group_solve(int l, const std::vector<int> &g, int count, const Inst *hI, const Ptrs *hP, int precision,
                      const RunOpts &o, int flags, hipStream_t s, BatchBuffers *bb, Result *hR, hipEvent_t start)
{
    if (g.empty()) return MMOT_OK;
    thread_local hipStream_t side = nullptr;
    thread_local hipEvent_t ev_in = nullptr, ev_out = nullptr;
    if (!side) {
        TCHK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        TCHK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
        TCHK(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
    }
    if (!start) {
        TCHK(hipEventRecord(ev_in, s));
        start = ev_in;
    }
    TCHK(hipStreamWaitEvent(side, start, 0));
    const int rc = tiled_group_solve_on(l, g, count, hI, hP, precision, o, flags, side, bb, hR);
    TCHK(hipEventRecord(ev_out, side));
    TCHK(hipStreamWaitEvent(s, ev_out, 0));
    return rc;
}

static int tiled_group_solve_on(int l, const std::vector<int> &g, int count, const Inst *hI, const Ptrs *hP,
                                int precision, const RunOpts &o, int flags, hipStream_t s, BatchBuffers *bb,
                                Result *hR)
{
    for (int i : g)
        if (!((flags | hP[i].flags) & F_TILES) && !tile_tuned(l, hI[i].N)) {
            const int rc = tune_tile_length(l, i, count, hI, hP, o, flags, s, bb);
            if (rc) return rc;
        }
    std::vector<TileInst> hTI(count);
    std::vector<TileTrack> hTT(count);
    for (int i = 0; i < count; ++i) {
        std::memset(&hTI[i], 0, sizeof(TileInst));
        hTT[i] = {1.0, INFINITY, INFINITY, 0, TS_DONE, 0, 0, 0};
    }
    for (int i : g) {
        int nt = 1, B = (int)hI[i].N;
        if (!tile_shape(l, hI[i].N, flags | hP[i].flags, &nt, &B))
            return fail(MMOT_ERR_STATE, "instance routed to the tiled solver without a tile shape");
        hTI[i] = tile_inst(l, nt, B, reinterpret_cast<char *>(hP[i].scratch));
        const int64_t itr = hP[i].itr_cap > 0 ? hP[i].itr_cap : o.itr_max;
        hTT[i].state = itr > 0 ? TS_SWEEP : TS_DONE;
    }
    TCHK(hipMemcpyAsync(bb->dTI, hTI.data(), sizeof(TileInst) * count, hipMemcpyHostToDevice, s));
    TCHK(hipMemcpyAsync(bb->dTT, hTT.data(), sizeof(TileTrack) * count, hipMemcpyHostToDevice, s));
    std::vector<char> jh;
    TileJobs J;
    TCHK(upload_jobs(g, hTI, l, bb, s, jh, &J));
    const int *dlist = tile_group_list(bb, J);
    TCHK(launch_tile_init(bb->dI, bb->dP, dlist, (int)g.size(), o, s));

    // One sweep: l tiled updates, the estimate controller, l - 1 tiled FP64 checks (their jobs
    // return at once unless the controller asked for a check), the stopping controller.
    auto sweep = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int j = 0; j < l && e == hipSuccess; ++j)
            e = launch_tile_pass(l, precision, P_UPDATE, bb->dI, bb->dP, bb->dTI, bb->dTT, J, j, TS_SWEEP, s);
        if (e == hipSuccess) e = launch_tile_ctrl(l, 0, bb->dP, bb->dTI, bb->dTT, count, o, s);
        for (int j = 0; j < l - 1 && e == hipSuccess; ++j)
            e = launch_tile_pass(l, 0, P_CHECK, bb->dI, bb->dP, bb->dTI, bb->dTT, J, j, TS_CHECK, s);
        if (e == hipSuccess) e = launch_tile_ctrl(l, 1, bb->dP, bb->dTI, bb->dTT, count, o, s);
        return e;
    };
    // Sweeps in blocks of TILE_GRAPH_SWEEPS, captured once as a HIP graph and replayed (every
    // launch of a block has the same arguments); the host reads the states after each block.
    // Stopped instances' jobs return at once, so a block may run past an instance's stop.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const bool use_graph = !(flags & F_NO_GRAPH);
    if (use_graph) {
        TCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int rep = 0; rep < TILE_GRAPH_SWEEPS && e == hipSuccess; ++rep) e = sweep();
        hipGraph_t gcap = nullptr;
        const hipError_t e2 = hipStreamEndCapture(s, &gcap);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (gcap) (void)hipGraphDestroy(gcap);
            return fail(MMOT_ERR_HIP, std::string("capture of a sweep block: ") +
                                          hipGetErrorString(e != hipSuccess ? e : e2));
        }
        graph = gcap;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(MMOT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
    }
    struct GraphGuard {
        hipGraph_t g;
        hipGraphExec_t x;
        ~GraphGuard()
        {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
        }
    } guard{graph, exec};
    for (;;) {
        if (use_graph) {
            TCHK(hipGraphLaunch(exec, s));
        } else {
            for (int rep = 0; rep < TILE_GRAPH_SWEEPS; ++rep) TCHK(sweep());
        }
        TCHK(hipMemcpyAsync(hTT.data(), bb->dTT, sizeof(TileTrack) * count, hipMemcpyDeviceToHost, s));
        TCHK(hipStreamSynchronize(s));
        bool any = false;
        for (int i : g) any |= hTT[i].state == TS_SWEEP || hTT[i].state == TS_CHECK;
        if (!any) break;
    }

    // objective of the instances that finished cleanly
    bool anyobj = false;
    for (int i : g) {
        if (hTT[i].status == MMOT_OK && !((o.flags | hP[i].flags) & F_NO_OBJ)) {
            hTT[i].state = TS_OBJ;
            anyobj = true;
        }
    }
    std::vector<std::vector<double>> parts(count);
    if (anyobj) {
        TCHK(hipMemcpyAsync(bb->dTT, hTT.data(), sizeof(TileTrack) * count, hipMemcpyHostToDevice, s));
        TCHK(launch_tile_pass(l, 0, P_OBJECTIVE, bb->dI, bb->dP, bb->dTI, bb->dTT, J, l - 1, TS_OBJ, s));
        for (int i : g) {
            if (hTT[i].state != TS_OBJ) continue;
            parts[i].resize(hTI[i].ntile);
            TCHK(hipMemcpyAsync(parts[i].data(), hTI[i].part + (size_t)(l - 1) * hTI[i].ntile,
                                sizeof(double) * hTI[i].ntile, hipMemcpyDeviceToHost, s));
        }
    }
    TCHK(hipStreamSynchronize(s));
    for (int i : g) {
        Result &R = hR[i];
        const TileTrack &T = hTT[i];
        double W = 0.0;
        for (double v : parts[i]) W += v;
        R.W = W;
        R.marg_err = T.res;
        R.iters = T.it;
        R.status = T.status;
        R.l = l;
        R.N = hI[i].N;
        if (R.status == MMOT_OK && T.state == TS_OBJ && !std::isfinite(W)) R.status = MMOT_ERR_NUMERIC;
        if (R.status == MMOT_OK && T.checked && o.tol >= 0.0 && !(T.res <= o.tol)) R.status = MMOT_NOT_CONVERGED;
    }
    return MMOT_OK;
}

}  // namespace mmot
