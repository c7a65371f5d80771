// Host runtime of libmmot: argument checks, discount tables, device workspace,
// launches, and the C ABI declared in include/mmot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dense.hpp"
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

int guard_fail()
{
    try {
        throw;
    } catch (const std::bad_alloc &) {
        return fail(MMOT_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(MMOT_ERR_INTERNAL, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(MMOT_ERR_INTERNAL, "internal error");
    }
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
        return fail(MMOT_ERR_UNSUPPORTED, "the library solves l <= " + std::to_string(MMOT_BUILD_MAXL));
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
    Inst hI;
    mutable BatchBuffers bb = {};  // one-instance batch for the solve entry points
    Inst *dI = nullptr;
    void *scratch = nullptr;
    size_t scratch_size = 0;
    Result *dR = nullptr;
    double *dtmp = nullptr;
    // tiled plans (long N): tile shape, host copies kept alive for async uploads
    bool tiled = false;
    int ntile = 1, B = 0;
    double *dx = nullptr;  // non-uniform grid: device copy of the coordinates (tiled kernels)
    double *djac = nullptr;  // MMOT_FLAG_JACOBI: [l][N] products of one all-marginals sweep
    double *ddense = nullptr;  // dense products: per-range partial sums (small problems only)
    TileInst hTI;
    mutable Ptrs hP;
    mutable std::vector<char> jobs_host;
};

static int plan_flags(const mmot_opts &o, bool grid)
{
    // a non-uniform grid runs on the tiled kernels only
    return ((o.flags & MMOT_FLAG_TILES) || grid ? F_TILES : 0) | ((o.flags & MMOT_FLAG_NO_GRAPH) ? F_NO_GRAPH : 0);
}

// Host-side check of non-uniform grid coordinates: finite and non-decreasing.
static int check_grid_host(const double *x, int64_t N)
{
    for (int64_t p = 0; p < N; ++p)
        if (!std::isfinite(x[p]) || (p > 0 && !(x[p] >= x[p - 1])))
            return fail(MMOT_ERR_INVALID, "grid coordinates must be finite and non-decreasing (index " +
                                              std::to_string(p) + ")");
    return MMOT_OK;
}

extern "C" {

const char *mmot_last_error(void) { return g_err.c_str(); }

int mmot_plan(const mmot_problem *p, const mmot_opts *o, void *hip_stream, mmot_plan_t **out)
{
    try {
        if (!p || !out) return fail(MMOT_ERR_INVALID, "problem or out is NULL");
        *out = nullptr;
        const bool grid = p->x != nullptr;
        int rc = check_shape(p->l, p->N, grid ? 1.0 : p->h, p->eps);
        if (rc) return rc;
        if (grid && (rc = check_grid_host(p->x, p->N))) return rc;
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
        // on a non-uniform grid the gap lengths enter the factors and the objective's
        // weights, so the objective takes no factor h (h = 1)
        Inst I = make_inst(p->l, p->N, grid ? 1.0 : p->h, p->eps);
        pl->tiled = tile_shape(p->l, p->N, plan_flags(oo, grid), &pl->ntile, &pl->B);
        pl->scratch_size = scratch_bytes(p->l, p->N, p->precision, plan_flags(oo, grid));
        hipError_t e = hipSuccess;
        if (grid) {
            e = hipMalloc((void **)&pl->dx, sizeof(double) * (size_t)p->N);
            if (e == hipSuccess) e = hipMemcpy(pl->dx, p->x, sizeof(double) * (size_t)p->N, hipMemcpyHostToDevice);
            I.x = pl->dx;
        }
        pl->p.x = nullptr;  // the caller's host array is not kept
        pl->hI = I;
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dI, sizeof(Inst));
        if (e == hipSuccess && (oo.flags & MMOT_FLAG_JACOBI))
            e = hipMalloc((void **)&pl->djac, sizeof(double) * (size_t)p->l * (size_t)p->N);
        if (e == hipSuccess && dense_supported(p->l, p->N))
            e = hipMalloc((void **)&pl->ddense, sizeof(double) * 2 * (size_t)p->N * (size_t)dense_ranges((int)p->N));
        if (e == hipSuccess) e = hipMalloc(&pl->scratch, std::max<size_t>(pl->scratch_size, 256));
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dR, sizeof(Result));
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dtmp, sizeof(double) * MAXL);
        if (e == hipSuccess) e = batch_buffers_alloc(&pl->bb, 1);
        if (e == hipSuccess) e = hipMemcpy(pl->dI, &I, sizeof(Inst), hipMemcpyHostToDevice);
        if (e == hipSuccess && pl->tiled) {
            pl->hTI = tile_inst(p->l, pl->ntile, pl->B, reinterpret_cast<char *>(pl->scratch));
            e = hipMemcpy(pl->bb.dTI, &pl->hTI, sizeof(TileInst), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(pl->bb.dI, &I, sizeof(Inst), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            mmot_plan_destroy(pl);
            return fail(e == hipErrorOutOfMemory ? MMOT_ERR_NOMEM : MMOT_ERR_HIP,
                        std::string("plan allocation: ") + hipGetErrorString(e));
        }
        *out = pl;
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_plan_footprint(const mmot_plan_t *pl, size_t *device_bytes)
{
    try {
        if (!pl || !device_bytes) return fail(MMOT_ERR_INVALID, "NULL argument");
        *device_bytes = 2 * sizeof(Inst) + pl->scratch_size + 2 * sizeof(Result) + sizeof(double) * MAXL +
                        sizeof(Ptrs) + 3 * sizeof(int) + sizeof(Track) +
                        2 * sizeof(double) * (size_t)pl->p.l * (size_t)pl->p.N +
                        (pl->dx ? sizeof(double) * (size_t)pl->p.N : 0) +
                        (pl->djac ? sizeof(double) * (size_t)pl->p.l * (size_t)pl->p.N : 0) +
                        (pl->ddense ? sizeof(double) * 2 * (size_t)pl->p.N * (size_t)dense_ranges((int)pl->p.N) : 0);
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_plan_destroy(mmot_plan_t *pl)
{
    try {
        if (!pl) return MMOT_OK;
        if (pl->dI) (void)hipFree(pl->dI);
        batch_buffers_free(&pl->bb);
        if (pl->scratch) (void)hipFree(pl->scratch);
        if (pl->dR) (void)hipFree(pl->dR);
        if (pl->dtmp) (void)hipFree(pl->dtmp);
        if (pl->dx) (void)hipFree(pl->dx);
        if (pl->djac) (void)hipFree(pl->djac);
        if (pl->ddense) (void)hipFree(pl->ddense);
        delete pl;
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

// One tiled pass (product, FP64 errors of every marginal, or objective) of a
// tiled plan; per-tile sums land in the plan's scratch (TileInst.part).
static int plan_tile_pass(const mmot_plan_t *pl, int mode, int j, const double *log_u, const double *log_phi,
                          double *out)
{
    pl->hP = {log_u, const_cast<double *>(log_phi), out, pl->scratch, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(pl->bb.dP, &pl->hP, sizeof(Ptrs), hipMemcpyHostToDevice, pl->s));
    TileJobs J;
    std::vector<TileInst> hti(1, pl->hTI);
    HIPCHK(upload_jobs(std::vector<int>{0}, hti, pl->p.l, &pl->bb, pl->s, pl->jobs_host, &J));
    if (mode == P_CHECK) {
        for (int jj = 0; jj < pl->p.l; ++jj)
            HIPCHK(launch_tile_pass(pl->p.l, MMOT_FP64, P_CHECK, pl->bb.dI, pl->bb.dP, pl->bb.dTI, nullptr, J, jj, 0,
                                    pl->s));
    } else {
        HIPCHK(launch_tile_pass(pl->p.l, pl->p.precision, mode, pl->bb.dI, pl->bb.dP, pl->bb.dTI, nullptr, J, j, 0,
                                pl->s));
    }
    return MMOT_OK;
}

// Sums of the per-tile results of rows [j0, j1) of a tiled plan (synchronises).
static int plan_tile_sums(const mmot_plan_t *pl, int j0, int j1, double *sums)
{
    std::vector<double> part((size_t)(j1 - j0) * pl->ntile);
    HIPCHK(hipMemcpyAsync(part.data(), pl->hTI.part + (size_t)j0 * pl->ntile, sizeof(double) * part.size(),
                          hipMemcpyDeviceToHost, pl->s));
    HIPCHK(hipStreamSynchronize(pl->s));
    for (int j = j0; j < j1; ++j) {
        double r = 0.0;
        for (int t = 0; t < pl->ntile; ++t) r += part[(size_t)(j - j0) * pl->ntile + t];
        sums[j - j0] = r;
    }
    return MMOT_OK;
}

int mmot_marginal_product(const mmot_plan_t *pl, int32_t j, const double *log_phi, double *log_J)
{
    try {
        if (!pl || !log_phi || !log_J) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (j < 0 || j >= pl->p.l) return fail(MMOT_ERR_INVALID, "j out of range");
        if (pl->tiled) return plan_tile_pass(pl, P_PRODUCT, j, nullptr, log_phi, log_J);
        Ptrs P = {nullptr, const_cast<double *>(log_phi), log_J, pl->scratch, 0, 0, 0, 0};
        HIPCHK(launch_pass(pl->p.l, pl->p.precision, 0, pl->dI, P, j, nullptr, pl->s));
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_dense_marginal_product(const mmot_plan_t *pl, int32_t j, const double *log_phi, double *log_J)
{
    try {
        if (!pl || !log_phi || !log_J) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (j < 0 || j >= pl->p.l) return fail(MMOT_ERR_INVALID, "j out of range");
        if (!pl->ddense) return fail(MMOT_ERR_UNSUPPORTED, "the dense product takes l <= 6, (l + 1) N <= 6144 and N^(l-1) < 2^31");
        HIPCHK(launch_dense_product(pl->p.l, (int)pl->p.N, j, pl->hI.hoe, pl->hI.ieps, pl->dx, log_phi, log_J,
                                    nullptr, nullptr, pl->ddense, pl->s));
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_dense_sinkhorn_iter(const mmot_plan_t *pl, const double *log_u, double *log_phi, int64_t n_sweeps)
{
    try {
        if (!pl || !log_u || !log_phi) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (n_sweeps < 0) return fail(MMOT_ERR_INVALID, "n_sweeps must be >= 0");
        if (!pl->ddense) return fail(MMOT_ERR_UNSUPPORTED, "the dense product takes l <= 6, (l + 1) N <= 6144 and N^(l-1) < 2^31");
        const long N = (long)pl->p.N;
        for (int64_t it = 0; it < n_sweeps; ++it)
            for (int j = 0; j < pl->p.l; ++j)
                HIPCHK(launch_dense_product(pl->p.l, (int)N, j, pl->hI.hoe, pl->hI.ieps, pl->dx, log_phi, nullptr,
                                            log_phi + (long)j * N, log_u + (long)j * N, pl->ddense, pl->s));
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_marginal_errors(const mmot_plan_t *pl, const double *log_u, const double *log_phi, double *err)
{
    try {
        if (!pl || !log_u || !log_phi || !err) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (pl->tiled) {
            const int rc = plan_tile_pass(pl, P_CHECK, 0, log_u, log_phi, nullptr);
            return rc ? rc : plan_tile_sums(pl, 0, pl->p.l, err);
        }
        Ptrs P = {log_u, const_cast<double *>(log_phi), nullptr, pl->scratch, 0, 0, 0, 0};
        HIPCHK(launch_pass(pl->p.l, MMOT_FP64, 2, pl->dI, P, 0, pl->dtmp, pl->s));
        HIPCHK(hipMemcpyAsync(err, pl->dtmp, sizeof(double) * pl->p.l, hipMemcpyDeviceToHost, pl->s));
        HIPCHK(hipStreamSynchronize(pl->s));
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

static int plan_path(const mmot_plan_t *pl)
{
    return ((pl->o.flags & MMOT_FLAG_NO_FAST) ? F_NO_FAST : 0) | plan_flags(pl->o, pl->dx != nullptr);
}

// The marginals of one plan call must be probability vectors (checked on the device).
static int plan_validate(const mmot_plan_t *pl, const double *log_u, const double *log_phi)
{
    Ptrs P = {log_u, const_cast<double *>(log_phi), nullptr, pl->scratch, 0, 0, 0, 0};
    int bad = 0;
    HIPCHK(hipMemcpyAsync(pl->bb.dI, &pl->hI, sizeof(Inst), hipMemcpyHostToDevice, pl->s));
    HIPCHK(hipMemcpyAsync(pl->bb.dP, &P, sizeof(Ptrs), hipMemcpyHostToDevice, pl->s));
    HIPCHK(launch_check_marginals(pl->bb.dI, pl->bb.dP, 1, pl->bb.dflags, pl->s));
    HIPCHK(hipMemcpyAsync(&bad, pl->bb.dflags, sizeof(int), hipMemcpyDeviceToHost, pl->s));
    HIPCHK(hipStreamSynchronize(pl->s));
    if (bad & 1) return fail(MMOT_ERR_INVALID, "a marginal entry is NaN or negative");
    if (bad & 2) return fail(MMOT_ERR_INVALID, "a marginal's mass differs from 1 by more than 1e-12");
    if (bad & 4) return fail(MMOT_ERR_INVALID, "grid coordinates must be finite and non-decreasing");
    return MMOT_OK;
}

// MMOT_FLAG_JACOBI: up to max_sweeps all-marginals sweeps (l products from the
// sweep's starting potentials into djac, then the damped update of every row),
// the FP64 residual over all l marginals every check_every sweeps and after the
// last, stopping once it is <= tol (tol < 0: never early).  Potentials start at
// phi = 1/N unless warm.
static int jacobi_run(const mmot_plan_t *pl, const double *log_u, double *log_phi, int64_t max_sweeps, double tol,
                      int check_every, bool warm, bool want_res, int64_t *iters, double *res)
{
    const int l = pl->p.l;
    const int64_t N = pl->p.N;
    int rc = plan_validate(pl, log_u, log_phi);
    if (rc) return rc;
    if (!warm) HIPCHK(launch_fill(log_phi, (long)l * N, -std::log((double)N), pl->s));
    const int every = check_every > 0 ? check_every : 10;
    double r = INFINITY;
    int64_t it = 0;
    while (it < max_sweeps) {
        ++it;
        for (int j = 0; j < l; ++j) {
            double *out = pl->djac + (size_t)j * (size_t)N;
            if (pl->tiled) {
                rc = plan_tile_pass(pl, P_PRODUCT, j, nullptr, log_phi, out);
                if (rc) return rc;
            } else {
                Ptrs P = {nullptr, log_phi, out, pl->scratch, 0, 0, 0, 0};
                HIPCHK(launch_pass(l, pl->p.precision, P_PRODUCT, pl->dI, P, j, nullptr, pl->s));
            }
        }
        HIPCHK(launch_jacobi_update(log_phi, log_u, pl->djac, (long)l * N, l, pl->s));
        if (want_res && (it % every == 0 || it == max_sweeps)) {
            double err[MAXL];
            rc = mmot_marginal_errors(pl, log_u, log_phi, err);
            if (rc) return rc;
            r = 0.0;
            for (int j = 0; j < l; ++j) r += err[j];
            if (!std::isfinite(r)) return fail(MMOT_ERR_NUMERIC, "non-finite residual");
            if (tol >= 0.0 && r <= tol) break;
        }
    }
    *iters = it;
    *res = r;
    return MMOT_OK;
}

int mmot_sinkhorn_iter(const mmot_plan_t *pl, const double *log_u, double *log_phi, int64_t n_sweeps,
                       double *marg_err)
{
    try {
        if (!pl || !log_u || !log_phi) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (n_sweeps < 0) return fail(MMOT_ERR_INVALID, "n_sweeps must be >= 0");
        if (pl->djac && n_sweeps > 0) {
            int64_t it = 0;
            double r = 0.0;
            // only the sweep count's last residual is computed (check_every = n_sweeps)
            const int rc = jacobi_run(pl, log_u, log_phi, n_sweeps, -1.0, (int)std::min<int64_t>(n_sweeps, INT32_MAX),
                                      true, marg_err != nullptr, &it, &r);
            if (rc) return rc;
            if (marg_err) *marg_err = r;
            return MMOT_OK;
        }
        if (n_sweeps > 0) {
            RunOpts o = {-1.0, n_sweeps, 0, F_WARM | F_NO_OBJ | F_VALIDATE | (marg_err ? 0 : F_NO_CHECK) | plan_path(pl)};
            Ptrs P = {log_u, log_phi, nullptr, pl->scratch, 0, 0, F_WARM, 0};
            Result R;
            int rc = batch_launch(&pl->hI, &P, 1, pl->p.precision, o, pl->s, &R, &pl->bb);
            if (rc) return rc;
            if (!marg_err) return MMOT_OK;
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
    } catch (...) {
        return guard_fail();
    }
}

int mmot_solve(const mmot_plan_t *pl, const double *log_u, double *log_phi, mmot_result *res)
{
    try {
        if (pl && pl->djac && log_u && log_phi && res) {
            const bool warm = (pl->o.flags & MMOT_FLAG_WARM_START) != 0;
            int64_t it = 0;
            double r = INFINITY;
            int rc = jacobi_run(pl, log_u, log_phi, pl->o.itr_max, pl->o.tol, pl->o.check_every, warm, true, &it, &r);
            if (rc) return rc;
            double W = 0.0;
            rc = mmot_objective(pl, log_phi, &W);
            if (rc) return rc;
            res->W = W;
            res->marg_err = r;
            res->iters = it;
            res->l = pl->p.l;
            res->N = pl->p.N;
            const bool conv = pl->o.tol < 0.0 || r <= pl->o.tol;
            res->status = !std::isfinite(W) ? MMOT_ERR_NUMERIC : conv ? MMOT_OK : MMOT_NOT_CONVERGED;
            if (res->status == MMOT_ERR_NUMERIC) return fail(MMOT_ERR_NUMERIC, "non-finite objective");
            if (res->status == MMOT_NOT_CONVERGED) g_err = "itr_max reached before tol";
            return res->status;
        }
        if (!pl || !log_u || !log_phi || !res) return fail(MMOT_ERR_INVALID, "NULL argument");
        const int warm = (pl->o.flags & MMOT_FLAG_WARM_START) ? F_WARM : 0;
        RunOpts o = {pl->o.tol, pl->o.itr_max, pl->o.check_every, plan_path(pl) | F_VALIDATE};
        Ptrs P = {log_u, log_phi, nullptr, pl->scratch, 0, 0, warm, 0};
        Result R;
        int rc = batch_launch(&pl->hI, &P, 1, pl->p.precision, o, pl->s, &R, &pl->bb);
        if (rc) return rc;
        static_assert(sizeof(Result) == sizeof(mmot_result), "result layout");
        std::memcpy(res, &R, sizeof R);
        if (R.status == MMOT_ERR_NUMERIC) return fail(MMOT_ERR_NUMERIC, "non-finite potentials, residual or objective");
        if (R.status == MMOT_NOT_CONVERGED) {
            g_err = "itr_max reached before tol";
            return MMOT_NOT_CONVERGED;
        }
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_objective(const mmot_plan_t *pl, const double *log_phi, double *W)
{
    try {
        if (!pl || !log_phi || !W) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (pl->tiled) {
            int rc = plan_tile_pass(pl, P_OBJECTIVE, pl->p.l - 1, nullptr, log_phi, nullptr);
            if (!rc) rc = plan_tile_sums(pl, pl->p.l - 1, pl->p.l, W);
            if (rc) return rc;
            return std::isfinite(*W) ? MMOT_OK : fail(MMOT_ERR_NUMERIC, "non-finite objective");
        }
        Ptrs P = {nullptr, const_cast<double *>(log_phi), nullptr, pl->scratch, 0, 0, 0, 0};
        HIPCHK(launch_pass(pl->p.l, MMOT_FP64, 3, pl->dI, P, pl->p.l - 1, pl->dtmp, pl->s));
        HIPCHK(hipMemcpyAsync(W, pl->dtmp, sizeof(double), hipMemcpyDeviceToHost, pl->s));
        HIPCHK(hipStreamSynchronize(pl->s));
        return std::isfinite(*W) ? MMOT_OK : fail(MMOT_ERR_NUMERIC, "non-finite objective");
    } catch (...) {
        return guard_fail();
    }
}

}  // extern "C"

// ---------------- batch ----------------

namespace {

// Grow-only device arena for batch launches (one per process, serialised).
struct BatchArena {
    std::mutex mu;
    BatchBuffers bb = {};
    char *scratch = nullptr;
    size_t cap_inst = 0, cap_scratch = 0;
    Inst *hI = nullptr;  // pinned host descriptors (the source of the descriptor upload)
    size_t cap_host = 0;

    int reserve_host(size_t count)
    {
        if (count <= cap_host) return MMOT_OK;
        if (hI) (void)hipHostFree(hI);
        hI = nullptr;
        cap_host = 0;
        const size_t c = std::max<size_t>(count, 64);
        if (hipHostMalloc((void **)&hI, c * sizeof(Inst), hipHostMallocDefault) != hipSuccess) {
            hI = nullptr;
            return fail(MMOT_ERR_NOMEM, "pinned batch descriptor allocation failed");
        }
        cap_host = c;
        return MMOT_OK;
    }

    int reserve(size_t count, size_t scratch_total)
    {
        if (count > cap_inst) {
            batch_buffers_free(&bb);
            cap_inst = 0;
            const size_t c = std::max<size_t>(count, 64);
            if (batch_buffers_alloc(&bb, c) != hipSuccess) {
                batch_buffers_free(&bb);
                return fail(MMOT_ERR_NOMEM, "batch descriptor allocation failed");
            }
            cap_inst = c;
        }
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
mmot_batch_timing g_last_timing = {};

// Events around individual launches of one timed batch (grow-only pool).
struct LaunchTimer {
    std::vector<hipEvent_t> pool;
    struct Span {
        int kind;  // 0 sweep, 1 check, 2 other
        int e0, e1;
    };
    std::vector<Span> spans;
    bool on = false;

    hipError_t begin(int kind, hipStream_t s, int *slot)
    {
        *slot = -1;
        if (!on) return hipSuccess;
        const int need = 2 * ((int)spans.size() + 1);
        while ((int)pool.size() < need) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            pool.push_back(e);
        }
        const int i = 2 * (int)spans.size();
        spans.push_back({kind, i, i + 1});
        *slot = (int)spans.size() - 1;
        return hipEventRecord(pool[i], s);
    }
    hipError_t end(int slot, hipStream_t s) { return slot < 0 ? hipSuccess : hipEventRecord(pool[spans[slot].e1], s); }
};
LaunchTimer g_timer;

constexpr int ST_OK_HOST = 0;

// Estimated work of one solve: scan cost per position grows like l 2^(l-1),
// sweeps grow as eps shrinks.  Only used to order the work queue.
double est_cost(int l, int64_t N, double eps)
{
    return (double)l * (double)l * std::ldexp(1.0, l - 1) * (double)N / std::sqrt(eps);
}

}  // namespace

namespace mmot {

hipError_t batch_buffers_alloc(BatchBuffers *bb, size_t c)
{
    *bb = {};
    hipError_t e = hipMalloc((void **)&bb->dI, sizeof(Inst) * c);
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dP, sizeof(Ptrs) * c);
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dorder, sizeof(int) * 2 * c);
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dR, sizeof(Result) * c);
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dticket, sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dT, sizeof(Track) * c);
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dTI, sizeof(TileInst) * c);
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dTT, sizeof(TileTrack) * c);
    if (e == hipSuccess) e = hipMalloc((void **)&bb->dflags, sizeof(int) * c);
    return e;
}

void batch_buffers_free(BatchBuffers *bb)
{
    if (bb->dI) (void)hipFree(bb->dI);
    if (bb->dP) (void)hipFree(bb->dP);
    if (bb->dorder) (void)hipFree(bb->dorder);
    if (bb->dR) (void)hipFree(bb->dR);
    if (bb->dticket) (void)hipFree(bb->dticket);
    if (bb->dT) (void)hipFree(bb->dT);
    if (bb->dTI) (void)hipFree(bb->dTI);
    if (bb->dTT) (void)hipFree(bb->dTT);
    if (bb->djobs) (void)hipFree(bb->djobs);
    if (bb->dflags) (void)hipFree(bb->dflags);
    *bb = {};
}

// Shared by mmot_solve_batch, the plan entry points and the server.
//   1. instances the register-resident path does not take: one persistent
//      launch of the extended-range solver (one wavefront per instance);
//   2. the others, grouped by l: rounds of the sweep kernel (runs each solve
//      until a residual check is due) and the FP64 check kernel, until no
//      solve is left sweeping; solves handed to the extended-range solver
//      mid-way resume there in one more persistent launch;
//   3. the objective of the fast-path solves, one wavefront each.
// Predicted sweeps an instance still needs after a warm-up round of `warmup`
// sweeps: the estimate fell from est_mid to est over the round's second half;
// assuming the same geometric rate, it reaches tol * f after log(est / (tol f))
// / rate more sweeps.  Instances not sweeping come last; an estimate that did
// not fall ranks first.
static double remaining_sweeps(const Track &T, double tol, int warmup)
{
    if (T.state != TS_SWEEP) return -1.0;
    const double tgt = tol * T.f;
    if (!(T.est > tgt)) return 0.0;
    if (!(T.est_mid > T.est) || !(T.est > 0.0)) return INFINITY;
    const double rate = std::log(T.est_mid / T.est) / (double)(warmup / 2);
    return std::log(T.est / std::max(tgt, 1e-300)) / rate;
}

int batch_launch(const Inst *hI, const Ptrs *hP, int count, int precision, const RunOpts &o, hipStream_t s,
                 Result *hR, BatchBuffers *bb, bool timed)
{
    if (count <= 0) return MMOT_OK;
    int flags = o.flags;
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) cost[i] = est_cost(hI[i].l, hI[i].N, hI[i].h / hI[i].hoe);
    auto by_cost = [&](std::vector<int> &v) {
        std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    };
    // Paths: tiled (long N), one team per instance (l >= WIDE_MINL), register-resident
    // (l <= 4, N fits a workgroup), one wavefront per instance (the rest).  Index p
    // of robust / wide / tiled is the precision of the instance's scans: FP32 mode
    // keeps FP32 mantissas only where the scan window is short (scan_precision).
    // A batch with few instances that the register-resident path does not take cannot fill the
    // GPU with one team or wavefront per instance: then every such instance from N = 256 up is
    // tiled (its scratch always has room for both layouts, scratch_bytes).
    {
        int n_slow = 0;
        for (int i = 0; i < count; ++i)
            if ((flags & F_NO_FAST) || !fast_eligible(hI[i], precision)) ++n_slow;
        // (MMOT_FLAG_NO_FAST asks for the one-wavefront solver: no small-batch tiling then)
        if (n_slow < SMALL_BATCH && !(flags & F_NO_FAST)) flags |= F_TILE_SMALL;
    }
    std::vector<int> robust[2], group[MAXL + 1], wide[MAXL + 1][2], tiled[MAXL + 1][2];
    for (int i = 0; i < count; ++i) {
        int nt = 0, tb = 0;
        const int fl = flags | hP[i].flags;
        const bool fast = !(fl & F_NO_FAST) && !(fl & F_TILES) && fast_eligible(hI[i], precision);
        if (fast) group[hI[i].l].push_back(i);
        else if (tile_shape(hI[i].l, hI[i].N, fl, &nt, &tb)) tiled[hI[i].l][scan_precision(hI[i], precision, true)].push_back(i);
        else if (hI[i].l >= WIDE_MINL) wide[hI[i].l][scan_precision(hI[i], precision, true)].push_back(i);
        else robust[scan_precision(hI[i], precision, false)].push_back(i);
    }
    // dorder: [robust FP64 | robust FP32 | wide (l, p) ... | group 2 | group 3 | ...], then the second
    // half for resumed and objective lists
    std::vector<int> order;
    order.reserve(2 * (size_t)count);
    int roff[2] = {0, 0};
    for (int p = 0; p < 2; ++p) {
        by_cost(robust[p]);
        roff[p] = (int)order.size();
        order.insert(order.end(), robust[p].begin(), robust[p].end());
    }
    int woff[MAXL + 1][2] = {};
    for (int l = WIDE_MINL; l <= MAXL; ++l)
        for (int p = 0; p < 2; ++p) {
            by_cost(wide[l][p]);
            woff[l][p] = (int)order.size();
            order.insert(order.end(), wide[l][p].begin(), wide[l][p].end());
        }
    int goff[MAXL + 1] = {0}, gmaxN[MAXL + 1] = {0};
    for (int l = 2; l <= MAXL; ++l) {
        by_cost(group[l]);
        goff[l] = (int)order.size();
        order.insert(order.end(), group[l].begin(), group[l].end());
        for (int i : group[l]) gmaxN[l] = std::max<int>(gmaxN[l], (int)hI[i].N);
    }
    HIPCHK(hipMemcpyAsync(bb->dI, hI, sizeof(Inst) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bb->dP, hP, sizeof(Ptrs) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bb->dorder, order.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    if (flags & F_VALIDATE) {
        // the marginals must be probability vectors (checked on the device, before any sweep)
        std::vector<int> bad(count);
        HIPCHK(launch_check_marginals(bb->dI, bb->dP, count, bb->dflags, s));
        HIPCHK(hipMemcpyAsync(bad.data(), bb->dflags, sizeof(int) * count, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < count; ++i) {
            if (bad[i] & 1) return fail(MMOT_ERR_INVALID, "instance " + std::to_string(i) + ": a marginal entry is NaN or negative");
            if (bad[i] & 2)
                return fail(MMOT_ERR_INVALID, "instance " + std::to_string(i) + ": a marginal's mass differs from 1 by more than 1e-12");
            if (bad[i] & 4)
                return fail(MMOT_ERR_INVALID, "instance " + std::to_string(i) + ": grid coordinates must be finite and non-decreasing");
        }
    }
    size_t nother = robust[0].size() + robust[1].size();
    for (int l = 2; l <= MAXL; ++l) nother += wide[l][0].size() + wide[l][1].size() + tiled[l][0].size() + tiled[l][1].size();
    const bool any_fast = nother < (size_t)count;
    std::vector<Track> hT;
    if (any_fast) {
        hT.resize(count);
        for (int i = 0; i < count; ++i) {
            const int64_t itr = hP[i].itr_cap > 0 ? hP[i].itr_cap : o.itr_max;
            hT[i] = {1.0, INFINITY, INFINITY, 0, itr > 0 ? TS_SWEEP : TS_DONE, 0, 0, 0, 0.0};
        }
        HIPCHK(hipMemcpyAsync(bb->dT, hT.data(), sizeof(Track) * count, hipMemcpyHostToDevice, s));
    }
    std::unique_lock<std::mutex> lk(g_time_mu, std::defer_lock);
    int slot = -1;
    double sweep_units = 0.0;
    int rounds = 0;
    if (timed) {
        lk.lock();
        if (!g_ev0) {
            HIPCHK(hipEventCreate(&g_ev0));
            HIPCHK(hipEventCreate(&g_ev1));
        }
        g_timer.spans.clear();
        g_timer.on = true;
        HIPCHK(hipEventRecord(g_ev0, s));
    }
    // the tiled groups need only the uploads above: their launches (on a stream
    // of their own) overlap the persistent launches enqueued below
    thread_local hipEvent_t ev_ready = nullptr;
    if (!ev_ready) HIPCHK(hipEventCreateWithFlags(&ev_ready, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev_ready, s));
    LaunchTimer &tm = g_timer;
    const bool tmon = timed;
    auto tbegin = [&](int kind) { return tmon ? tm.begin(kind, s, &slot) : hipSuccess; };
    auto tend = [&]() { return tmon ? tm.end(slot, s) : hipSuccess; };
    for (int p = 0; p < 2; ++p) {
        if (robust[p].empty()) continue;
        const int n = (int)robust[p].size();
        const int blocks = std::max(1, std::min((n + 3) / 4, 4096));
        HIPCHK(tbegin(2));
        HIPCHK(launch_solve_batch(p, bb->dI, bb->dP, bb->dorder + roff[p], n, o, bb->dR, bb->dticket, blocks, s));
        HIPCHK(tend());
    }
    for (int l = WIDE_MINL; l <= MAXL; ++l)
        for (int p = 0; p < 2; ++p) {
            if (wide[l][p].empty()) continue;
            HIPCHK(tbegin(2));
            HIPCHK(launch_wide_batch(l, p, bb->dI, bb->dP, bb->dorder + woff[l][p], (int)wide[l][p].size(), o,
                                     bb->dR, bb->dticket, s));
            HIPCHK(tend());
        }
    // tiled instances: host-driven blocks of sweeps per (l, precision), results straight into hR
    std::vector<Result> tiled_res;
    for (int l = 2; l <= MAXL; ++l)
        for (int p = 0; p < 2; ++p) {
            if (tiled[l][p].empty()) continue;
            if (tiled_res.empty()) tiled_res.resize(count);
            HIPCHK(tbegin(2));
            const int rc =
                tiled_group_solve(l, tiled[l][p], count, hI, hP, p, o, flags, s, bb, tiled_res.data(), ev_ready);
            if (rc) return rc;
            HIPCHK(tend());
        }
    std::vector<int> resumed, objective;
    std::vector<char> handed(count, 0);  // handed to the extended-range solver
    if (any_fast) {
        bool sweeping[MAXL + 1];
        for (int l = 0; l <= MAXL; ++l) sweeping[l] = !group[l].empty();
        std::vector<int64_t> it_before(count, 0);
        // Longest first: a group larger than the device holds at once starts with
        // a round of o.warmup sweeps for every instance; from the estimate's decay
        // over its second half each instance's remaining sweeps are predicted,
        // and the later rounds take the group in that order, longest first, so
        // that the slowest solves do not start last (reordered on the device up
        // to FAST_ORDER_MAX instances, else by the host).  Rounds are pairs of a
        // sweep and a check launch; for such groups FAST_PAIRS of them are
        // enqueued back to back before the host reads the states (a solve whose
        // check fails goes on in the next pair).  Iterates are unchanged.
        bool warm[MAXL + 1];
        for (int l = 0; l <= MAXL; ++l)
            warm[l] = o.warmup >= 2 && o.tol >= 0.0 && (int)group[l].size() > FAST_RESIDENT;
        for (;;) {
            bool any = false;
            int pairs_max = 0;
            for (int l = 2; l <= MAXL; ++l) {
                if (!sweeping[l]) continue;
                any = true;
                const int n = (int)group[l].size();
                const int cap = 256 * 8;  // persistent workgroups: a few per CU
                auto pair = [&](int budget) -> hipError_t {
                    RunOpts so = o;
                    so.budget = budget;
                    hipError_t e = tbegin(0);
                    if (e == hipSuccess)
                        e = launch_fast(0, l, precision, bb->dI, bb->dP, bb->dorder + goff[l], n, so, bb->dT,
                                        bb->dticket, std::min(n, cap), fast_waves(l, gmaxN[l], 0, precision), s);
                    if (e == hipSuccess) e = tend();
                    if (e == hipSuccess) e = tbegin(1);
                    if (e == hipSuccess)
                        e = launch_fast(1, l, precision, bb->dI, bb->dP, bb->dorder + goff[l], n, o, bb->dT,
                                        bb->dticket, std::min(n, cap), fast_waves(l, gmaxN[l], 1, precision), s);
                    if (e == hipSuccess) e = tend();
                    return e;
                };
                int pairs = 0;
                if (warm[l]) {
                    HIPCHK(pair(o.warmup));
                    ++pairs;
                    if (n <= FAST_ORDER_MAX) {
                        HIPCHK(launch_fast_order(bb->dT, bb->dorder + goff[l], n, o.tol, o.warmup, s));
                        warm[l] = false;
                        for (int k = 0; k < FAST_PAIRS; ++k, ++pairs) HIPCHK(pair(0));
                    }
                } else {
                    // after a reordering (large groups) several pairs, else one
                    const int np = (int)group[l].size() > FAST_RESIDENT ? FAST_PAIRS : 1;
                    for (int k = 0; k < np; ++k, ++pairs) HIPCHK(pair(0));
                }
                pairs_max = std::max(pairs_max, pairs);
            }
            if (!any) break;
            rounds += pairs_max;
            HIPCHK(hipMemcpyAsync(hT.data(), bb->dT, sizeof(Track) * count, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int l = 2; l <= MAXL; ++l) {
                if (!sweeping[l]) continue;
                sweeping[l] = false;
                for (int i : group[l]) {
                    sweep_units += (double)l * (double)hI[i].N * (double)(hT[i].it - it_before[i]);
                    it_before[i] = hT[i].it;
                    if (hT[i].state == TS_SWEEP) sweeping[l] = true;
                    if (hT[i].state == TS_ROBUST && !handed[i]) {
                        handed[i] = 1;
                        resumed.push_back(i);
                    }
                }
                if (warm[l]) {
                    warm[l] = false;
                    std::vector<int> &g = group[l];
                    std::vector<double> pr(count, 0.0);
                    for (int i : g) pr[i] = remaining_sweeps(hT[i], o.tol, o.warmup);
                    std::stable_sort(g.begin(), g.end(), [&](int x, int y) { return pr[x] > pr[y]; });
                    std::copy(g.begin(), g.end(), order.begin() + goff[l]);
                    HIPCHK(hipMemcpyAsync(bb->dorder + goff[l], order.data() + goff[l], sizeof(int) * g.size(),
                                          hipMemcpyHostToDevice, s));
                }
            }
        }
        for (int l = 2; l <= MAXL; ++l)
            for (int i : group[l])
                if (!handed[i] && hT[i].status == ST_OK_HOST && !((flags | hP[i].flags) & F_NO_OBJ))
                    objective.push_back(i);
    }
    if (!resumed.empty()) {
        // the extended-range solver picks these up where the fast path stopped
        std::vector<Ptrs> rp(resumed.size());
        for (size_t k = 0; k < resumed.size(); ++k) {
            const int i = resumed[k];
            Ptrs P = hP[i];
            P.it0 = hT[i].it;
            P.j0 = hT[i].j0;
            P.flags |= F_WARM;
            rp[k] = P;
            HIPCHK(hipMemcpyAsync(bb->dP + i, &rp[k], sizeof(Ptrs), hipMemcpyHostToDevice, s));
        }
        HIPCHK(hipMemcpyAsync(bb->dorder + count, resumed.data(), sizeof(int) * resumed.size(), hipMemcpyHostToDevice,
                              s));
        RunOpts ro = o;
        if (ro.check_every <= 0) ro.check_every = 10;
        const int n = (int)resumed.size();
        HIPCHK(tbegin(2));
        HIPCHK(launch_solve_batch(precision, bb->dI, bb->dP, bb->dorder + count, n, ro, bb->dR, bb->dticket,
                                  std::max(1, std::min((n + 3) / 4, 4096)), s));
        HIPCHK(tend());
        HIPCHK(hipStreamSynchronize(s));  // rp and resumed stay alive until the copies ran
    }
    if (!objective.empty()) {
        HIPCHK(hipMemcpyAsync(bb->dorder + count, objective.data(), sizeof(int) * objective.size(),
                              hipMemcpyHostToDevice, s));
        HIPCHK(tbegin(2));
        HIPCHK(launch_objective_batch(bb->dI, bb->dP, bb->dorder + count, (int)objective.size(), bb->dR,
                                      bb->dticket, s));
        HIPCHK(tend());
    }
    if (timed) HIPCHK(hipEventRecord(g_ev1, s));
    HIPCHK(hipMemcpyAsync(hR, bb->dR, sizeof(Result) * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int l = 2; l <= MAXL; ++l)
        for (int p = 0; p < 2; ++p)
            for (int i : tiled[l][p]) hR[i] = tiled_res[i];
    if (timed) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g_ev0, g_ev1));
        g_last_kernel_ms = ms;
        mmot_batch_timing t = {};
        t.total_ms = ms;
        for (const auto &sp : tm.spans) {
            float d = 0.f;
            HIPCHK(hipEventElapsedTime(&d, tm.pool[sp.e0], tm.pool[sp.e1]));
            if (sp.kind == 0) {
                t.sweep_ms += d;
                ++t.sweep_launches;
            } else if (sp.kind == 1) {
                t.check_ms += d;
            } else {
                t.other_ms += d;
            }
        }
        t.sweep_units = sweep_units;
        t.rounds = rounds;
        g_last_timing = t;
        tm.on = false;
    }
    if (any_fast) {
        std::vector<char> has_w(count, 0);
        for (int i : objective) has_w[i] = 1;
        for (int l = 2; l <= MAXL; ++l)
            for (int i : group[l]) {
                if (handed[i]) continue;  // the extended-range solver wrote its own result
                Result &R = hR[i];
                const Track &T = hT[i];
                R.W = has_w[i] ? R.W : 0.0;
                R.marg_err = T.res;
                R.iters = T.it;
                R.status = T.status;
                R.l = hI[i].l;
                R.N = hI[i].N;
                if (R.status == ST_OK_HOST && has_w[i] && !std::isfinite(R.W)) R.status = MMOT_ERR_NUMERIC;
                if (R.status == ST_OK_HOST && T.checked && o.tol >= 0.0 && !(T.res <= o.tol))
                    R.status = MMOT_NOT_CONVERGED;
            }
    }
    return MMOT_OK;
}

}  // namespace mmot

extern "C" int mmot_last_batch_kernel_ms(double *ms)
{
    try {
        if (!ms) return fail(MMOT_ERR_INVALID, "NULL argument");
        std::lock_guard<std::mutex> lk(g_time_mu);
        if (g_last_kernel_ms < 0) return fail(MMOT_ERR_STATE, "no batch launch yet");
        *ms = g_last_kernel_ms;
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

extern "C" int mmot_last_batch_timing(mmot_batch_timing *t)
{
    try {
        if (!t) return fail(MMOT_ERR_INVALID, "NULL argument");
        std::lock_guard<std::mutex> lk(g_time_mu);
        if (g_last_kernel_ms < 0) return fail(MMOT_ERR_STATE, "no batch launch yet");
        *t = g_last_timing;
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

extern "C" int mmot_solve_batch(const mmot_instance *inst, int32_t count, int32_t precision, const mmot_opts *o,
                                void *hip_stream, mmot_result *res)
{
    try {
        if (count < 0 || (count > 0 && (!inst || !res))) return fail(MMOT_ERR_INVALID, "bad instance list");
        if (precision != MMOT_FP64 && precision != MMOT_FP32) return fail(MMOT_ERR_INVALID, "bad precision");
        int rc = check_opts(o);
        if (rc) return rc;
        if (o->flags & MMOT_FLAG_JACOBI) return fail(MMOT_ERR_UNSUPPORTED, "MMOT_FLAG_JACOBI is a plan option");
        if (count == 0) return MMOT_OK;
        std::vector<Ptrs> hP(count);
        size_t off = 0;
        std::vector<size_t> offs(count);
        for (int i = 0; i < count; ++i) {
            const bool grid = inst[i].x != nullptr;
            rc = check_shape(inst[i].l, inst[i].N, grid ? 1.0 : inst[i].h, inst[i].eps);
            if (rc) return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
            if (!inst[i].log_u || !inst[i].log_phi) return fail(MMOT_ERR_INVALID, "instance " + std::to_string(i) + ": NULL buffer");
            offs[i] = off;
            off += scratch_bytes(inst[i].l, inst[i].N, precision, (o->flags & MMOT_FLAG_TILES) || grid ? F_TILES : 0);
        }
        std::lock_guard<std::mutex> lk(g_batch.mu);
        rc = g_batch.reserve((size_t)count, std::max<size_t>(off, 256));
        if (rc) return rc;
        rc = g_batch.reserve_host((size_t)count);
        if (rc) return rc;
        // Descriptors, written into pinned memory.  The discount tables depend on l
        // and h / eps only: they are computed once per distinct pair and copied.
        Inst *hI = g_batch.hI;
        std::map<std::pair<int, uint64_t>, int> owner;
        for (int i = 0; i < count; ++i) {
            // non-uniform grid: tiled kernels, no factor h on the objective (as mmot_plan)
            const double he = inst[i].x ? 1.0 : inst[i].h;
            const double hoe = he / inst[i].eps;
            uint64_t bits;
            std::memcpy(&bits, &hoe, sizeof bits);
            const auto key = std::make_pair((int)inst[i].l, bits);
            const auto it = owner.find(key);
            if (it == owner.end()) {
                hI[i] = make_inst(inst[i].l, inst[i].N, he, inst[i].eps);
                owner.emplace(key, i);
            } else {
                std::memcpy(&hI[i], &hI[it->second], sizeof(Inst));
                hI[i].N = inst[i].N;
                hI[i].h = he;
                hI[i].hoe = hoe;
                hI[i].ieps = 1.0 / inst[i].eps;
            }
            hI[i].x = inst[i].x;
        }
        for (int i = 0; i < count; ++i)
            hP[i] = {inst[i].log_u, inst[i].log_phi, nullptr, g_batch.scratch + offs[i], 0, 0,
                     ((o->flags & MMOT_FLAG_WARM_START) ? F_WARM : 0) | (inst[i].x ? F_TILES : 0), 0};
        RunOpts ro = {o->tol, o->itr_max, o->check_every,
                      ((o->flags & MMOT_FLAG_NO_FAST) ? F_NO_FAST : 0) | ((o->flags & MMOT_FLAG_TILES) ? F_TILES : 0) |
                          ((o->flags & MMOT_FLAG_NO_GRAPH) ? F_NO_GRAPH : 0) |
                          F_VALIDATE, 0,
                      FAST_WARMUP_SWEEPS};
        BatchBuffers bb = g_batch.bb;
        std::vector<Result> hR(count);
        rc = batch_launch(hI, hP.data(), count, precision, ro, (hipStream_t)hip_stream, hR.data(), &bb, true);
        if (rc) {
            // the descriptor upload reads the pinned buffer asynchronously: let it
            // finish before a later call rewrites the buffer
            (void)hipStreamSynchronize((hipStream_t)hip_stream);
            return rc;
        }
        int worst = MMOT_OK;
        for (int i = 0; i < count; ++i) {
            std::memcpy(&res[i], &hR[i], sizeof(Result));
            if (hR[i].status == MMOT_ERR_NUMERIC) worst = MMOT_ERR_NUMERIC;
            else if (hR[i].status == MMOT_NOT_CONVERGED && worst == MMOT_OK) worst = MMOT_NOT_CONVERGED;
        }
        if (worst == MMOT_ERR_NUMERIC) return fail(MMOT_ERR_NUMERIC, "some instances produced non-finite values");
        if (worst == MMOT_NOT_CONVERGED) g_err = "some instances reached itr_max";
        return worst;
    } catch (...) {
        return guard_fail();
    }
}
