// Host side of the 2-D three-marginal problem (Sec. 4.1): plans, the product
// pipeline of k_2d.hip, Gauss-Seidel solves, FP64 errors and the objective.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "launch.hpp"
#include "mmot.h"
#include "serve.hpp"
#include "tables.hpp"

namespace mmot {
hipError_t launch2_scan_in(const double *A, const double *B, long N, int M, double lg, double *const bufs[6],
                           hipStream_t s);
hipError_t launch2_scan_w(const double *C, long N, int M, double lg, double *Pj, double *Qj, hipStream_t s);
hipError_t launch2_gather(const double *const src[15], long N, int M, int with_weight, double *tri, hipStream_t s);
hipError_t launch2_passes(int mode, const Inst *dI, const Ptrs *dP, int count, double *dres, hipStream_t s);
hipError_t launch2_combine(const double *T, long N, int M, double lg, double *CF, int mode, double *out,
                           const double *lu, hipStream_t s);
hipError_t launch2_err(const double *a, const double *logJ, const double *lu, long n, double *partial, int blocks,
                       hipStream_t s);
hipError_t launch2_transpose(const double *in, long N, int M, double *out, hipStream_t s);
}  // namespace mmot

using namespace mmot;
using namespace mmot::rt;

#define H2CHK(call)                                                                                    \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(MMOT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {
constexpr int ERR_BLOCKS = 256;
}

struct mmot_plan_2d {
    mmot_problem_2d p;
    mmot_opts o;
    hipStream_t s = nullptr;
    Inst hI[2];                 // 1-D passes along the first axis (length N, h1) and the second (M, h2)
    Inst *dI = nullptr;         // [2]
    Inst *dIv = nullptr;        // validation view: l = 3 rows of N M entries
    size_t cnt = 0;             // 6 max(N, M) passes
    double *buf = nullptr;      // one allocation, carved below
    double *st[6] = {};         // F(a), F(b), g F_{y-1}(b), B(a), H_{y+1}(a), H_{y+1}(b): [M][N] each
    double *cf = nullptr, *pj = nullptr, *qj = nullptr, *jt = nullptr;
    double *tri = nullptr;      // [6][m][3][n] rows of the passes (n m = N M on either axis)
    double *T = nullptr;        // [6][M][N] pass outputs
    double *aT = nullptr;       // [3][N][M] transposed potentials
    double *res = nullptr;      // per-pass objective terms
    double *part = nullptr;     // error partial sums
    char *scratch = nullptr;    // per-pass scan checkpoints
    size_t scr_each = 0;
    Ptrs *dP = nullptr;
    std::vector<Ptrs> hP;
    int ptr_axis = -1;          // axis whose pass pointers dP holds
    int *dflags = nullptr;
    Ptrs *dPv = nullptr;
};

static int check_2d(const mmot_problem_2d *p)
{
    if (!p) return fail(MMOT_ERR_INVALID, "problem is NULL");
    if (p->N < 1 || p->M < 1) return fail(MMOT_ERR_INVALID, "N and M must be >= 1");
    if (p->N * p->M > (int64_t(1) << 31) / 3) return fail(MMOT_ERR_INVALID, "N * M too large");
    if (p->M > (int64_t(1) << 24) || p->N > (int64_t(1) << 24)) return fail(MMOT_ERR_INVALID, "N or M too large");
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(MMOT_ERR_INVALID, "eps must be finite and > 0");
    if (!(p->h1 > 0.0) || !std::isfinite(p->h1) || !(p->h2 > 0.0) || !std::isfinite(p->h2))
        return fail(MMOT_ERR_INVALID, "h1 and h2 must be finite and > 0");
    return MMOT_OK;
}

// One 1-D pass set along an axis of length n (rows of the other axis: m): Ptrs of
// pass b read tri + 3 n b and write T + n b (product) or res[b] (objective).
static int upload_ptrs(mmot_plan_2d_t *pl, int ax, long n, int m)
{
    if (pl->ptr_axis == ax) return MMOT_OK;
    const int count = 6 * m;
    for (int b = 0; b < count; ++b)
        pl->hP[b] = {nullptr, pl->tri + (size_t)3 * n * b, pl->T + (size_t)n * b, pl->scratch + pl->scr_each * b, 0, 0, 0, 0};
    H2CHK(hipMemcpyAsync(pl->dP, pl->hP.data(), sizeof(Ptrs) * count, hipMemcpyHostToDevice, pl->s));
    H2CHK(hipStreamSynchronize(pl->s));
    pl->ptr_axis = ax;
    return MMOT_OK;
}

// The product pipeline for target j on potentials a ([3][m][n], axis parameters
// ax): mode 0 writes log J_j to out, mode 1 writes a_j = log u_j - log J_j; or,
// with obj, the first-axis part of the objective of target j into *W.
static int pipeline(mmot_plan_2d_t *pl, int ax, const double *a, long n, int m, int j, int mode, double *out,
                    const double *lu, bool obj, double *W)
{
    const double h2 = ax == 0 ? pl->p.h2 : pl->p.h1;
    const double lg = -2.0 * h2 / pl->p.eps;  // log g: l = 3, one or two marginals left of a gap
    const int qa = j == 0 ? 1 : 0, qb = j == 2 ? 1 : 2;
    const size_t S = (size_t)n * m;
    const double *A = a + qa * S, *B = a + qb * S;
    H2CHK(launch2_scan_in(A, B, n, m, lg, pl->st, pl->s));
    const double *src[15] = {pl->st[0], B, A, pl->st[2], pl->st[3], B, A, pl->st[5], pl->st[0], pl->st[5],
                             pl->st[4], pl->st[1], pl->pj, pl->qj, a + (size_t)j * S};
    if (obj) H2CHK(launch2_scan_w(a + (size_t)j * S, n, m, lg, pl->pj, pl->qj, pl->s));
    H2CHK(launch2_gather(src, n, m, obj ? 1 : 0, pl->tri, pl->s));
    int rc = upload_ptrs(pl, ax, n, m);
    if (rc) return rc;
    const Inst *dI = pl->dI + ax;
    if (obj) {
        const int count = 6 * m;
        H2CHK(launch2_passes(P_OBJECTIVE, dI, pl->dP, count, pl->res, pl->s));
        std::vector<double> r(count);
        H2CHK(hipMemcpyAsync(r.data(), pl->res, sizeof(double) * count, hipMemcpyDeviceToHost, pl->s));
        H2CHK(hipStreamSynchronize(pl->s));
        double w = 0.0;
        for (double v : r) w += v;
        *W = w;
        return MMOT_OK;
    }
    H2CHK(launch2_passes(P_PRODUCT, dI, pl->dP, 6 * m, nullptr, pl->s));
    H2CHK(launch2_combine(pl->T, n, m, lg, pl->cf, mode, out, lu, pl->s));
    return MMOT_OK;
}

static int errors_2d(mmot_plan_2d_t *pl, const double *log_u, const double *a, double *err, int nj)
{
    const long n = pl->p.N;
    const int m = (int)pl->p.M;
    const size_t S = (size_t)n * m;
    std::vector<double> part(ERR_BLOCKS);
    for (int j = 0; j < nj; ++j) {
        int rc = pipeline(pl, 0, a, n, m, j, 0, pl->jt, nullptr, false, nullptr);
        if (rc) return rc;
        H2CHK(launch2_err(a + j * S, pl->jt, log_u + j * S, (long)S, pl->part, ERR_BLOCKS, pl->s));
        H2CHK(hipMemcpyAsync(part.data(), pl->part, sizeof(double) * ERR_BLOCKS, hipMemcpyDeviceToHost, pl->s));
        H2CHK(hipStreamSynchronize(pl->s));
        double e = 0.0;
        for (double v : part) e += v;
        err[j] = e;
    }
    return MMOT_OK;
}

extern "C" {

int mmot_plan_2d(const mmot_problem_2d *p, const mmot_opts *o, void *hip_stream, mmot_plan_2d_t **out)
{
    try {
        if (!out) return fail(MMOT_ERR_INVALID, "out is NULL");
        *out = nullptr;
        int rc = check_2d(p);
        if (rc) return rc;
        mmot_opts oo = {1e-8, 1000, 10, 0};
        if (o) {
            rc = check_opts(o);
            if (rc) return rc;
            oo = *o;
        }
        if (oo.flags & ~MMOT_FLAG_WARM_START)
            return fail(MMOT_ERR_UNSUPPORTED, "2-D plans take MMOT_FLAG_WARM_START only");
        mmot_plan_2d_t *pl = new mmot_plan_2d_t();
        pl->p = *p;
        pl->o = oo;
        pl->s = (hipStream_t)hip_stream;
        const long N = p->N, M = p->M, L = std::max(N, M);  // passes per pipeline: 6 M, or 6 N transposed
        pl->hI[0] = make_inst(3, N, p->h1, p->eps);
        pl->hI[1] = make_inst(3, M, p->h2, p->eps);
        const Inst iv = make_inst(3, N * M, 1.0, p->eps);
        pl->cnt = (size_t)6 * L;
        pl->scr_each = std::max(pass_scratch_bytes(3, N, MMOT_FP64), pass_scratch_bytes(3, M, MMOT_FP64));
        pl->scr_each = (pl->scr_each + 255) & ~(size_t)255;
        const size_t S = (size_t)N * M;
        // st[6], cf, pj, qj, jt: 10 S; tri: 18 S; T: 6 S; aT: 3 S; res: cnt; part
        const size_t nd = 10 * S + 18 * S + 6 * S + 3 * S + pl->cnt + ERR_BLOCKS;
        hipError_t e = hipMalloc((void **)&pl->buf, sizeof(double) * nd);
        if (e == hipSuccess) e = hipMalloc((void **)&pl->scratch, std::max<size_t>(pl->scr_each * pl->cnt, 256));
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dI, 2 * sizeof(Inst));
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dIv, sizeof(Inst));
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dP, sizeof(Ptrs) * pl->cnt);
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dPv, sizeof(Ptrs));
        if (e == hipSuccess) e = hipMalloc((void **)&pl->dflags, sizeof(int));
        if (e == hipSuccess) e = hipMemcpy(pl->dI, pl->hI, 2 * sizeof(Inst), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl->dIv, &iv, sizeof(Inst), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            mmot_plan_2d_destroy(pl);
            return fail(e == hipErrorOutOfMemory ? MMOT_ERR_NOMEM : MMOT_ERR_HIP,
                        std::string("2-D plan allocation: ") + hipGetErrorString(e));
        }
        double *q = pl->buf;
        for (int k = 0; k < 6; ++k, q += S) pl->st[k] = q;
        pl->cf = q; q += S;
        pl->pj = q; q += S;
        pl->qj = q; q += S;
        pl->jt = q; q += S;
        pl->tri = q; q += 18 * S;
        pl->T = q; q += 6 * S;
        pl->aT = q; q += 3 * S;
        pl->res = q; q += pl->cnt;
        pl->part = q;
        pl->hP.resize(pl->cnt);
        *out = pl;
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_plan_2d_destroy(mmot_plan_2d_t *pl)
{
    try {
        if (!pl) return MMOT_OK;
        if (pl->buf) (void)hipFree(pl->buf);
        if (pl->scratch) (void)hipFree(pl->scratch);
        if (pl->dI) (void)hipFree(pl->dI);
        if (pl->dIv) (void)hipFree(pl->dIv);
        if (pl->dP) (void)hipFree(pl->dP);
        if (pl->dPv) (void)hipFree(pl->dPv);
        if (pl->dflags) (void)hipFree(pl->dflags);
        delete pl;
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_marginal_product_2d(const mmot_plan_2d_t *pl, int32_t j, const double *log_phi, double *log_J)
{
    try {
        if (!pl || !log_phi || !log_J) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (j < 0 || j > 2) return fail(MMOT_ERR_INVALID, "j out of range");
        auto *p = const_cast<mmot_plan_2d_t *>(pl);
        return pipeline(p, 0, log_phi, pl->p.N, (int)pl->p.M, j, 0, log_J, nullptr, false, nullptr);
    } catch (...) {
        return guard_fail();
    }
}

int mmot_marginal_errors_2d(const mmot_plan_2d_t *pl, const double *log_u, const double *log_phi, double *err)
{
    try {
        if (!pl || !log_u || !log_phi || !err) return fail(MMOT_ERR_INVALID, "NULL argument");
        return errors_2d(const_cast<mmot_plan_2d_t *>(pl), log_u, log_phi, err, 3);
    } catch (...) {
        return guard_fail();
    }
}

int mmot_objective_2d(const mmot_plan_2d_t *pl, const double *log_phi, double *W)
{
    try {
        if (!pl || !log_phi || !W) return fail(MMOT_ERR_INVALID, "NULL argument");
        auto *p = const_cast<mmot_plan_2d_t *>(pl);
        const long N = pl->p.N, M = pl->p.M;
        double wx = 0.0, wy = 0.0;
        int rc = pipeline(p, 0, log_phi, N, (int)M, 2, 0, nullptr, nullptr, true, &wx);
        if (rc) return rc;
        // the second-axis part: the same on the transposed grid
        H2CHK(launch2_transpose(log_phi, N, (int)M, p->aT, p->s));
        rc = pipeline(p, 1, p->aT, M, (int)N, 2, 0, nullptr, nullptr, true, &wy);
        if (rc) return rc;
        *W = wx + wy;
        return std::isfinite(*W) ? MMOT_OK : fail(MMOT_ERR_NUMERIC, "non-finite objective");
    } catch (...) {
        return guard_fail();
    }
}

int mmot_solve_2d(const mmot_plan_2d_t *pl, const double *log_u, double *log_phi, mmot_result *res)
{
    try {
        if (!pl || !log_u || !log_phi || !res) return fail(MMOT_ERR_INVALID, "NULL argument");
        auto *p = const_cast<mmot_plan_2d_t *>(pl);
        const long N = pl->p.N;
        const int M = (int)pl->p.M;
        const size_t S = (size_t)N * M;
        // the marginals must be probability vectors (device check, as for the 1-D solves)
        const Ptrs Pv = {log_u, log_phi, nullptr, nullptr, 0, 0, 0, 0};
        int bad = 0;
        H2CHK(hipMemcpyAsync(p->dPv, &Pv, sizeof(Ptrs), hipMemcpyHostToDevice, p->s));
        H2CHK(launch_check_marginals(p->dIv, p->dPv, 1, p->dflags, p->s));
        H2CHK(hipMemcpyAsync(&bad, p->dflags, sizeof(int), hipMemcpyDeviceToHost, p->s));
        H2CHK(hipStreamSynchronize(p->s));
        if (bad & 1) return fail(MMOT_ERR_INVALID, "a marginal entry is NaN or negative");
        if (bad & 2) return fail(MMOT_ERR_INVALID, "a marginal's mass differs from 1 by more than 1e-12");
        if (!(pl->o.flags & MMOT_FLAG_WARM_START)) H2CHK(launch_fill(log_phi, (long)(3 * S), -std::log((double)S), p->s));
        const int every = pl->o.check_every > 0 ? pl->o.check_every : 10;
        double r = INFINITY;
        int64_t it = 0;
        while (it < pl->o.itr_max) {
            ++it;
            for (int j = 0; j < 3; ++j) {
                int rc = pipeline(p, 0, log_phi, N, M, j, 1, log_phi + j * S, log_u + j * S, false, nullptr);
                if (rc) return rc;
            }
            if (it % every == 0 || it == pl->o.itr_max) {
                double err[3];
                int rc = errors_2d(p, log_u, log_phi, err, 2);
                if (rc) return rc;
                r = err[0] + err[1];
                if (!std::isfinite(r)) return fail(MMOT_ERR_NUMERIC, "non-finite residual");
                if (pl->o.tol >= 0.0 && r <= pl->o.tol) break;
            }
        }
        double W = 0.0;
        int rc = mmot_objective_2d(pl, log_phi, &W);
        if (rc) return rc;
        res->W = W;
        res->marg_err = r;
        res->iters = it;
        res->l = 3;
        res->N = (int64_t)S;
        const bool conv = pl->o.tol < 0.0 || r <= pl->o.tol;
        res->status = conv ? MMOT_OK : MMOT_NOT_CONVERGED;
        if (!conv) g_err = "itr_max reached before tol";
        return res->status;
    } catch (...) {
        return guard_fail();
    }
}

}  // extern "C"
