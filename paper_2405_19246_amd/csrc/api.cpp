// Host runtime of libmmot: argument checks, discount tables, device workspace,
// launches, and the C ABI declared in include/mmot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "launch.hpp"
#include "mmot.h"
#include "serve.hpp"
#include "tables.hpp"

using namespace mmot;

namespace mmot {
namespace rt {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(MMOT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int check_shape(int l, int64_t N, double h, double eps)
{
    if (l < 2 || l > MMOT_MAX_L) return fail(MMOT_ERR_INVALID, "l must be in [2, " + std::to_string(MMOT_MAX_L) + "]");
    if (l > MMOT_BUILD_MAXL)
        return fail(MMOT_ERR_UNSUPPORTED, "this build solves l <= " + std::to_string(MMOT_BUILD_MAXL));
    if (N < 1) return fail(MMOT_ERR_INVALID, "N must be >= 1");
    if (N > (int64_t(1) << 31) / l) return fail(MMOT_ERR_INVALID, "l * N too large");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(MMOT_ERR_INVALID, "eps must be finite and > 0");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(MMOT_ERR_INVALID, "h must be finite and > 0");
    return MMOT_OK;
}

int check_opts(const mmot_opts *o)
{
    if (!o) return fail(MMOT_ERR_INVALID, "opts is NULL");
    if (o->itr_max < 0) return fail(MMOT_ERR_INVALID, "itr_max must be >= 0");
    if (o->check_every < 0) return fail(MMOT_ERR_INVALID, "check_every must be >= 0");
    if (std::isnan(o->tol)) return fail(MMOT_ERR_INVALID, "tol is NaN");
    return MMOT_OK;
}

}  // namespace rt
}  // namespace mmot

using namespace mmot::rt;

struct mmot_plan {
    mmot_problem p;
    mmot_opts o;
    hipStream_t s;
    Inst *dI = nullptr;
    void *scratch = nullptr;
    size_t scratch_size = 0;
    Result *dR = nullptr;
    double *dtmp = nullptr;
};

extern "C" {

const char *mmot_last_error(void) { return g_err.c_str(); }

int mmot_plan(const mmot_problem *p, const mmot_opts *o, void *hip_stream, mmot_plan_t **out)
{
    if (!p || !out) return fail(MMOT_ERR_INVALID, "problem or out is NULL");
    *out = nullptr;
    int rc = check_shape(p->l, p->N, p->h, p->eps);
    if (rc) return rc;
    if (p->precision != MMOT_FP64 && p->precision != MMOT_FP32)
        return fail(MMOT_ERR_INVALID, "precision must be MMOT_FP64 or MMOT_FP32");
    mmot_opts oo = {1e-8, 1000, 10, 0};
    if (o) {
        rc = check_opts(o);
        if (rc) return rc;
        oo = *o;
    }
    mmot_plan_t *pl = new mmot_plan_t();
    pl->p = *p;
    pl->o = oo;
    pl->s = (hipStream_t)hip_stream;
    const Inst I = make_inst(p->l, p->N, p->h, p->eps);
    pl->scratch_size = scratch_bytes(p->l, p->N, p->precision);
    hipError_t e = hipMalloc((void **)&pl->dI, sizeof(Inst));
    if (e == hipSuccess) e = hipMalloc(&pl->scratch, std::max<size_t>(pl->scratch_size, 256));
    if (e == hipSuccess) e = hipMalloc((void **)&pl->dR, sizeof(Result));
    if (e == hipSuccess) e = hipMalloc((void **)&pl->dtmp, sizeof(double) * MAXL);
    if (e == hipSuccess) e = hipMemcpy(pl->dI, &I, sizeof(Inst), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        mmot_plan_destroy(pl);
        return fail(e == hipErrorOutOfMemory ? MMOT_ERR_NOMEM : MMOT_ERR_HIP,
                    std::string("plan allocation: ") + hipGetErrorString(e));
    }
    *out = pl;
    return MMOT_OK;
}

int mmot_plan_footprint(const mmot_plan_t *pl, size_t *device_bytes)
{
    if (!pl || !device_bytes) return fail(MMOT_ERR_INVALID, "NULL argument");
    *device_bytes = sizeof(Inst) + pl->scratch_size + sizeof(Result) + sizeof(double) * MAXL +
                    2 * sizeof(double) * (size_t)pl->p.l * (size_t)pl->p.N;
    return MMOT_OK;
}

int mmot_plan_destroy(mmot_plan_t *pl)
{
    if (!pl) return MMOT_OK;
    if (pl->dI) (void)hipFree(pl->dI);
    if (pl->scratch) (void)hipFree(pl->scratch);
    if (pl->dR) (void)hipFree(pl->dR);
    if (pl->dtmp) (void)hipFree(pl->dtmp);
    delete pl;
    return MMOT_OK;
}

int mmot_marginal_product(const mmot_plan_t *pl, int32_t j, const double *log_phi, double *log_J)
{
    if (!pl || !log_phi || !log_J) return fail(MMOT_ERR_INVALID, "NULL argument");
    if (j < 0 || j >= pl->p.l) return fail(MMOT_ERR_INVALID, "j out of range");
    Ptrs P = {nullptr, const_cast<double *>(log_phi), log_J, pl->scratch, 0, 0, 0};
    HIPCHK(launch_pass(pl->p.l, pl->p.precision, 0, pl->dI, P, j, nullptr, pl->s));
    return MMOT_OK;
}

static int read_result(const mmot_plan_t *pl, Result *R)
{
    HIPCHK(hipMemcpyAsync(R, pl->dR, sizeof(Result), hipMemcpyDeviceToHost, pl->s));
    HIPCHK(hipStreamSynchronize(pl->s));
    return MMOT_OK;
}

int mmot_marginal_errors(const mmot_plan_t *pl, const double *log_u, const double *log_phi, double *err)
{
    if (!pl || !log_u || !log_phi || !err) return fail(MMOT_ERR_INVALID, "NULL argument");
    Ptrs P = {log_u, const_cast<double *>(log_phi), nullptr, pl->scratch, 0, 0, 0};
    HIPCHK(launch_pass(pl->p.l, MMOT_FP64, 2, pl->dI, P, 0, pl->dtmp, pl->s));
    HIPCHK(hipMemcpyAsync(err, pl->dtmp, sizeof(double) * pl->p.l, hipMemcpyDeviceToHost, pl->s));
    HIPCHK(hipStreamSynchronize(pl->s));
    return MMOT_OK;
}

int mmot_sinkhorn_iter(const mmot_plan_t *pl, const double *log_u, double *log_phi, int64_t n_sweeps,
                       double *marg_err)
{
    if (!pl || !log_u || !log_phi) return fail(MMOT_ERR_INVALID, "NULL argument");
    if (n_sweeps < 0) return fail(MMOT_ERR_INVALID, "n_sweeps must be >= 0");
    if (n_sweeps > 0) {
        RunOpts o = {-1.0, n_sweeps, 0, F_WARM | F_NO_OBJ | (marg_err ? 0 : F_NO_CHECK)};
        Ptrs P = {log_u, log_phi, nullptr, pl->scratch, 0, 0, 0};
        HIPCHK(launch_solve_single(pl->p.l, pl->p.precision, pl->dI, P, o, pl->dR, pl->s));
        if (!marg_err) return MMOT_OK;
        Result R;
        int rc = read_result(pl, &R);
        if (rc) return rc;
        *marg_err = R.marg_err;
        if (R.status == MMOT_ERR_NUMERIC || !std::isfinite(R.marg_err)) return fail(MMOT_ERR_NUMERIC, "non-finite residual");
        return MMOT_OK;
    }
    if (!marg_err) return MMOT_OK;
    double err[MAXL];
    int rc = mmot_marginal_errors(pl, log_u, log_phi, err);
    if (rc) return rc;
    double r = 0.0;
    for (int j = 0; j < pl->p.l - 1; ++j) r += err[j];
    *marg_err = r;
    return std::isfinite(r) ? MMOT_OK : fail(MMOT_ERR_NUMERIC, "non-finite residual");
}

int mmot_solve(const mmot_plan_t *pl, const double *log_u, double *log_phi, mmot_result *res)
{
    if (!pl || !log_u || !log_phi || !res) return fail(MMOT_ERR_INVALID, "NULL argument");
    RunOpts o = {pl->o.tol, pl->o.itr_max, pl->o.check_every, (pl->o.flags & MMOT_FLAG_WARM_START) ? F_WARM : 0};
    Ptrs P = {log_u, log_phi, nullptr, pl->scratch, 0, 0, 0};
    HIPCHK(launch_solve_single(pl->p.l, pl->p.precision, pl->dI, P, o, pl->dR, pl->s));
    Result R;
    int rc = read_result(pl, &R);
    if (rc) return rc;
    static_assert(sizeof(Result) == sizeof(mmot_result), "result layout");
    std::memcpy(res, &R, sizeof R);
    if (R.status == MMOT_ERR_NUMERIC) return fail(MMOT_ERR_NUMERIC, "non-finite potentials, residual or objective");
    if (R.status == MMOT_NOT_CONVERGED) {
        g_err = "itr_max reached before tol";
        return MMOT_NOT_CONVERGED;
    }
    return MMOT_OK;
}

int mmot_objective(const mmot_plan_t *pl, const double *log_phi, double *W)
{
    if (!pl || !log_phi || !W) return fail(MMOT_ERR_INVALID, "NULL argument");
    Ptrs P = {nullptr, const_cast<double *>(log_phi), nullptr, pl->scratch, 0, 0, 0};
    HIPCHK(launch_pass(pl->p.l, MMOT_FP64, 3, pl->dI, P, pl->p.l - 1, pl->dtmp, pl->s));
    HIPCHK(hipMemcpyAsync(W, pl->dtmp, sizeof(double), hipMemcpyDeviceToHost, pl->s));
    HIPCHK(hipStreamSynchronize(pl->s));
    return std::isfinite(*W) ? MMOT_OK : fail(MMOT_ERR_NUMERIC, "non-finite objective");
}

}  // extern "C"

// ---------------- batch ----------------

namespace {

// Grow-only device arena for batch launches (one per process, serialised).
struct BatchArena {
    std::mutex mu;
    Inst *dI = nullptr;
    Ptrs *dP = nullptr;
    int *dorder = nullptr;
    Result *dR = nullptr;
    int *dticket = nullptr;
    char *scratch = nullptr;
    size_t cap_inst = 0, cap_scratch = 0;

    int reserve(size_t count, size_t scratch_total)
    {
        if (count > cap_inst) {
            if (dI) (void)hipFree(dI);
            if (dP) (void)hipFree(dP);
            if (dorder) (void)hipFree(dorder);
            if (dR) (void)hipFree(dR);
            dI = nullptr; dP = nullptr; dorder = nullptr; dR = nullptr;
            cap_inst = 0;
            size_t c = std::max<size_t>(count, 64);
            if (hipMalloc((void **)&dI, sizeof(Inst) * c) != hipSuccess ||
                hipMalloc((void **)&dP, sizeof(Ptrs) * c) != hipSuccess ||
                hipMalloc((void **)&dorder, sizeof(int) * c) != hipSuccess ||
                hipMalloc((void **)&dR, sizeof(Result) * c) != hipSuccess)
                return fail(MMOT_ERR_NOMEM, "batch descriptor allocation failed");
            cap_inst = c;
        }
        if (!dticket && hipMalloc((void **)&dticket, sizeof(int)) != hipSuccess)
            return fail(MMOT_ERR_NOMEM, "ticket allocation failed");
        if (scratch_total > cap_scratch) {
            if (scratch) (void)hipFree(scratch);
            scratch = nullptr;
            cap_scratch = 0;
            if (hipMalloc((void **)&scratch, scratch_total) != hipSuccess)
                return fail(MMOT_ERR_NOMEM, "batch scratch allocation failed (" + std::to_string(scratch_total) + " B)");
            cap_scratch = scratch_total;
        }
        return MMOT_OK;
    }
};

BatchArena g_batch;

// HIP-event timing of the last persistent batch kernel (stream-ordered).
std::mutex g_time_mu;
hipEvent_t g_ev0 = nullptr, g_ev1 = nullptr;
double g_last_kernel_ms = -1.0;

// Estimated work of one solve: scan cost per position grows like l 2^(l-1),
// sweeps grow as eps shrinks.  Only used to order the work queue.
double est_cost(int l, int64_t N, double eps)
{
    return (double)l * (double)l * std::ldexp(1.0, l - 1) * (double)N / std::sqrt(eps);
}

}  // namespace

namespace mmot {

// Shared by mmot_solve_batch and the server: enqueue one persistent launch.
int batch_launch(const Inst *hI, const Ptrs *hP, int count, int precision, const RunOpts &o, hipStream_t s,
                 Result *hR, BatchBuffers *bb)
{
    if (count <= 0) return MMOT_OK;
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) cost[i] = est_cost(hI[i].l, hI[i].N, hI[i].h / hI[i].hoe);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    HIPCHK(hipMemcpyAsync(bb->dI, hI, sizeof(Inst) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bb->dP, hP, sizeof(Ptrs) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bb->dorder, order.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    const int waves = count;
    const int blocks = std::max(1, std::min((waves + 3) / 4, 4096));
    std::lock_guard<std::mutex> lk(g_time_mu);
    if (!g_ev0) {
        HIPCHK(hipEventCreate(&g_ev0));
        HIPCHK(hipEventCreate(&g_ev1));
    }
    HIPCHK(hipEventRecord(g_ev0, s));
    HIPCHK(launch_solve_batch(precision, bb->dI, bb->dP, bb->dorder, count, o, bb->dR, bb->dticket, blocks, s));
    HIPCHK(hipEventRecord(g_ev1, s));
    HIPCHK(hipMemcpyAsync(hR, bb->dR, sizeof(Result) * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, g_ev0, g_ev1));
    g_last_kernel_ms = ms;
    return MMOT_OK;
}

}  // namespace mmot

extern "C" int mmot_last_batch_kernel_ms(double *ms)
{
    if (!ms) return fail(MMOT_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(g_time_mu);
    if (g_last_kernel_ms < 0) return fail(MMOT_ERR_STATE, "no batch launch yet");
    *ms = g_last_kernel_ms;
    return MMOT_OK;
}

extern "C" int mmot_solve_batch(const mmot_instance *inst, int32_t count, int32_t precision, const mmot_opts *o,
                                void *hip_stream, mmot_result *res)
{
    if (count < 0 || (count > 0 && (!inst || !res))) return fail(MMOT_ERR_INVALID, "bad instance list");
    if (precision != MMOT_FP64 && precision != MMOT_FP32) return fail(MMOT_ERR_INVALID, "bad precision");
    int rc = check_opts(o);
    if (rc) return rc;
    if (count == 0) return MMOT_OK;
    std::vector<Inst> hI(count);
    std::vector<Ptrs> hP(count);
    size_t off = 0;
    std::vector<size_t> offs(count);
    for (int i = 0; i < count; ++i) {
        rc = check_shape(inst[i].l, inst[i].N, inst[i].h, inst[i].eps);
        if (rc) return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
        if (!inst[i].log_u || !inst[i].log_phi) return fail(MMOT_ERR_INVALID, "instance " + std::to_string(i) + ": NULL buffer");
        hI[i] = make_inst(inst[i].l, inst[i].N, inst[i].h, inst[i].eps);
        offs[i] = off;
        off += scratch_bytes(inst[i].l, inst[i].N, precision);
    }
    std::lock_guard<std::mutex> lk(g_batch.mu);
    rc = g_batch.reserve((size_t)count, std::max<size_t>(off, 256));
    if (rc) return rc;
    for (int i = 0; i < count; ++i)
        hP[i] = {inst[i].log_u, inst[i].log_phi, nullptr, g_batch.scratch + offs[i], 0,
                 (o->flags & MMOT_FLAG_WARM_START) ? F_WARM : 0, 0};
    RunOpts ro = {o->tol, o->itr_max, o->check_every, 0};
    BatchBuffers bb = {g_batch.dI, g_batch.dP, g_batch.dorder, g_batch.dR, g_batch.dticket};
    std::vector<Result> hR(count);
    rc = batch_launch(hI.data(), hP.data(), count, precision, ro, (hipStream_t)hip_stream, hR.data(), &bb);
    if (rc) return rc;
    int worst = MMOT_OK;
    for (int i = 0; i < count; ++i) {
        std::memcpy(&res[i], &hR[i], sizeof(Result));
        if (hR[i].status == MMOT_ERR_NUMERIC) worst = MMOT_ERR_NUMERIC;
        else if (hR[i].status == MMOT_NOT_CONVERGED && worst == MMOT_OK) worst = MMOT_NOT_CONVERGED;
    }
    if (worst == MMOT_ERR_NUMERIC) return fail(MMOT_ERR_NUMERIC, "some instances produced non-finite values");
    if (worst == MMOT_NOT_CONVERGED) g_err = "some instances reached itr_max";
    return worst;
}
