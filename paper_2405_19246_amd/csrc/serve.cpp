// Serving loop of libmmot: continuous batching of MMOT solves.
//
// A server thread owns a HIP stream and one device arena sized by the HBM
// budget.  Requests wait in a host queue; at every device-round boundary the
// thread admits waiting requests (in arrival order) into free slots while their
// footprint -- log marginals, potentials, scan checkpoints -- fits the arena.
// It then runs one persistent batch launch in which every resident solve
// advances up to block_sweeps sweeps, stopping early once its FP64 residual
// meets tol.  Potentials stay on the device between rounds.  Finished solves
// get their FP64 objective in one more launch, are copied out, and free their
// slot and arena space for the next admissions.
//
// A solve's arithmetic does not depend on which other solves share a round:
// each runs on its own wavefront with its own buffers, and its residual is
// checked at the same sweep counts as long as block_sweeps is a multiple of
// check_every.  So a request gives the same result alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "serve.hpp"

using namespace mmot;
using namespace mmot::rt;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over offsets of one device arena.
class Arena {
public:
    void init(size_t size)
    {
        free_.clear();
        free_[0] = size;
    }
    static size_t round_up(size_t n) { return (n + 255) & ~(size_t)255; }
    bool alloc(size_t n, size_t *off)
    {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round_up(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t ticket = 0;
    int l = 0;
    int64_t N = 0;
    double h = 0, eps = 0;
    std::vector<double> log_u;  // host copy, [l][N]
    double t_submit = 0;
};

struct Slot {
    std::unique_ptr<Request> req;
    size_t off = 0, bytes = 0;
    Inst I;
    Ptrs P;
    int64_t iters = 0;
    double t_admit = 0;
    bool started = false;
};

struct Done {
    mmot_request_record rec;
    std::vector<double> log_phi;
};

size_t request_bytes(int l, int64_t N, int precision, int flags)
{
    const size_t rows = Arena::round_up(sizeof(double) * (size_t)l * (size_t)N);
    return 2 * rows + scratch_bytes(l, N, precision, flags);
}

}  // namespace

struct mmot_server {
    mmot_serve_cfg cfg;
    hipStream_t s = nullptr;
    char *base = nullptr;
    Arena arena;
    BatchBuffers bb = {};
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<Request>> queue;
    std::map<uint64_t, Done> done;
    uint64_t next_ticket = 1;
    bool stopping = false;
    bool cancel = false;  // mmot_serve_cancel: running solves end after the current round
    int error = MMOT_OK;
    std::string error_msg;

    void loop();
    int finish(std::vector<Slot> &slots, const std::vector<int> &fin, const std::vector<Result> &hR);
    int tile_flag() const
    {
        return ((cfg.opts.flags & MMOT_FLAG_TILES) ? F_TILES : 0) | ((cfg.opts.flags & MMOT_FLAG_NO_GRAPH) ? F_NO_GRAPH : 0);
    }
    int path_flag() const { return ((cfg.opts.flags & MMOT_FLAG_NO_FAST) ? F_NO_FAST : 0) | tile_flag(); }
};

int mmot_server::finish(std::vector<Slot> &slots, const std::vector<int> &fin, const std::vector<Result> &hR)
{
    // objective of the finished solves, one launch, no sweeps
    const int n = (int)fin.size();
    std::vector<Inst> hI(n);
    std::vector<Ptrs> hP(n);
    std::vector<Result> hW(n);
    for (int k = 0; k < n; ++k) {
        hI[k] = slots[fin[k]].I;
        hP[k] = slots[fin[k]].P;
        hP[k].itr_cap = 0;
        hP[k].flags = F_WARM;
    }
    RunOpts ro = {cfg.opts.tol, 0, cfg.opts.check_every, path_flag()};
    int rc = batch_launch(hI.data(), hP.data(), n, cfg.precision, ro, s, hW.data(), &bb);
    if (rc) return rc;
    const double t = now_s();
    std::vector<Done> out(n);
    for (int k = 0; k < n; ++k) {
        Slot &sl = slots[fin[k]];
        Done &d = out[k];
        std::memset(&d.rec, 0, sizeof d.rec);
        Result R = hR[fin[k]];
        R.iters = sl.iters;
        R.W = hW[k].W;
        if (R.status == 0 && hW[k].status == MMOT_ERR_NUMERIC) R.status = MMOT_ERR_NUMERIC;
        if (R.status == 0 && cfg.opts.tol >= 0 && !(R.marg_err <= cfg.opts.tol)) R.status = MMOT_NOT_CONVERGED;
        std::memcpy(&d.rec.result, &R, sizeof R);
        d.rec.t_submit = sl.req->t_submit;
        d.rec.t_admit = sl.t_admit;
        d.rec.t_done = t;
        d.log_phi.resize((size_t)sl.req->l * sl.req->N);
        if (hipMemcpy(d.log_phi.data(), sl.P.a, sizeof(double) * d.log_phi.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(MMOT_ERR_HIP, "copy of potentials failed");
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        for (int k = 0; k < n; ++k) {
            Slot &sl = slots[fin[k]];
            done[sl.req->ticket] = std::move(out[k]);
            arena.release(sl.off, sl.bytes);
        }
    }
    cv.notify_all();
    // drop finished slots (descending index keeps the others valid)
    std::vector<int> idx(fin);
    std::sort(idx.rbegin(), idx.rend());
    for (int i : idx) slots.erase(slots.begin() + i);
    return MMOT_OK;
}

void mmot_server::loop()
{
    std::vector<Slot> slots;
    for (;;) {
        std::vector<int> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stopping || !queue.empty() || !slots.empty(); });
            if (stopping && queue.empty() && slots.empty()) break;
            // admit in arrival order while a slot and arena space are free
            while (!queue.empty() && (int)slots.size() < cfg.max_slots) {
                Request &r = *queue.front();
                const size_t need = request_bytes(r.l, r.N, cfg.precision, tile_flag());
                size_t off = 0;
                if (!arena.alloc(need, &off)) break;
                Slot sl;
                sl.req = std::move(queue.front());
                queue.pop_front();
                sl.off = off;
                sl.bytes = need;
                sl.t_admit = now_s();
                fresh.push_back((int)slots.size());
                slots.push_back(std::move(sl));
            }
        }
        for (int i : fresh) {
            Slot &sl = slots[i];
            const Request &r = *sl.req;
            const size_t rows = Arena::round_up(sizeof(double) * (size_t)r.l * (size_t)r.N);
            char *p = base + sl.off;
            sl.I = make_inst(r.l, r.N, r.h, r.eps);
            sl.P = {(const double *)p, (double *)(p + rows), nullptr, p + 2 * rows, 0, 0, 0, 0};
            if (hipMemcpyAsync(p, r.log_u.data(), sizeof(double) * r.log_u.size(), hipMemcpyHostToDevice, s) !=
                hipSuccess) {
                error = MMOT_ERR_HIP;
                error_msg = "upload of marginals failed";
            }
        }
        if (slots.empty()) continue;
        // one device round over every resident solve
        const int n = (int)slots.size();
        std::vector<Inst> hI(n);
        std::vector<Ptrs> hP(n);
        std::vector<Result> hR(n);
        for (int i = 0; i < n; ++i) {
            hI[i] = slots[i].I;
            hP[i] = slots[i].P;
            const int64_t left = cfg.opts.itr_max - slots[i].iters;
            hP[i].itr_cap = std::max<int64_t>(1, std::min<int64_t>(cfg.block_sweeps, left));
            hP[i].flags = slots[i].started ? F_WARM : 0;
        }
        RunOpts ro = {cfg.opts.tol, cfg.block_sweeps, cfg.opts.check_every, F_NO_OBJ | path_flag()};
        int rc = batch_launch(hI.data(), hP.data(), n, cfg.precision, ro, s, hR.data(), &bb);
        if (rc) {
            std::lock_guard<std::mutex> lk(mu);
            error = rc;
            error_msg = g_err;
            stopping = true;
            queue.clear();
            break;
        }
        std::vector<int> fin;
        for (int i = 0; i < n; ++i) {
            Slot &sl = slots[i];
            sl.started = true;
            sl.iters += hR[i].iters;
            const bool conv = cfg.opts.tol >= 0 && hR[i].marg_err <= cfg.opts.tol;
            if (conv || hR[i].status == MMOT_ERR_NUMERIC || sl.iters >= cfg.opts.itr_max || cancel) fin.push_back(i);
        }
        if (!fin.empty()) {
            rc = finish(slots, fin, hR);
            if (rc) {
                std::lock_guard<std::mutex> lk(mu);
                error = rc;
                error_msg = g_err;
                stopping = true;
                queue.clear();
                break;
            }
        }
    }
    cv.notify_all();
}

extern "C" {

int mmot_serve_start(const mmot_serve_cfg *cfg, mmot_server_t **out)
{
    try {
        if (!cfg || !out) return fail(MMOT_ERR_INVALID, "NULL argument");
        *out = nullptr;
        if (cfg->precision != MMOT_FP64 && cfg->precision != MMOT_FP32) return fail(MMOT_ERR_INVALID, "bad precision");
        int rc = check_opts(&cfg->opts);
        if (rc) return rc;
        if (cfg->opts.flags & MMOT_FLAG_JACOBI)
            return fail(MMOT_ERR_UNSUPPORTED, "MMOT_FLAG_JACOBI is a plan option");
        if (cfg->max_slots < 1) return fail(MMOT_ERR_INVALID, "max_slots must be >= 1");
        if (cfg->block_sweeps < 1) return fail(MMOT_ERR_INVALID, "block_sweeps must be >= 1");
        if (cfg->hbm_budget_bytes < 4096) return fail(MMOT_ERR_INVALID, "hbm_budget_bytes too small");
        std::unique_ptr<mmot_server> srv(new mmot_server());
        srv->cfg = *cfg;
        if (srv->cfg.opts.itr_max < 1) srv->cfg.opts.itr_max = 1;
        hipError_t e = hipStreamCreate(&srv->s);
        if (e == hipSuccess) e = hipMalloc((void **)&srv->base, cfg->hbm_budget_bytes);
        const size_t c = (size_t)cfg->max_slots;
        if (e == hipSuccess) e = batch_buffers_alloc(&srv->bb, c);
        if (e != hipSuccess) {
            mmot_server *p = srv.release();
            if (p->base) (void)hipFree(p->base);
            batch_buffers_free(&p->bb);
            if (p->s) (void)hipStreamDestroy(p->s);
            delete p;
            return fail(e == hipErrorOutOfMemory ? MMOT_ERR_NOMEM : MMOT_ERR_HIP,
                        std::string("server allocation: ") + hipGetErrorString(e));
        }
        srv->arena.init(cfg->hbm_budget_bytes);
        int dev = 0;
        (void)hipGetDevice(&dev);
        mmot_server *raw = srv.get();
        raw->th = std::thread([raw, dev] {
            (void)hipSetDevice(dev);
            raw->loop();
        });
        *out = srv.release();
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_serve_submit(mmot_server_t *srv, const mmot_request *req, uint64_t *ticket)
{
    try {
        if (!srv || !req || !ticket || !req->u) return fail(MMOT_ERR_INVALID, "NULL argument");
        int rc = check_shape(req->l, req->N, req->h, req->eps);
        if (rc) return rc;
        const size_t n = (size_t)req->l * (size_t)req->N;
        std::unique_ptr<Request> r(new Request());
        r->l = req->l;
        r->N = req->N;
        r->h = req->h;
        r->eps = req->eps;
        r->log_u.resize(n);
        for (int q = 0; q < req->l; ++q) {
            double mass = 0.0, comp = 0.0;  // compensated sum: long rows stay well inside 1e-12
            for (int64_t i = 0; i < req->N; ++i) {
                const double v = req->u[(size_t)q * req->N + i];
                if (!(v >= 0.0) || !std::isfinite(v)) return fail(MMOT_ERR_INVALID, "marginal entries must be finite and >= 0");
                const double y = v - comp, t = mass + y;
                comp = (t - mass) - y;
                mass = t;
                r->log_u[(size_t)q * req->N + i] = std::log(v);
            }
            if (!(std::fabs(mass - 1.0) <= 1e-12)) return fail(MMOT_ERR_INVALID, "each marginal must sum to 1");
        }
        if (request_bytes(req->l, req->N, srv->cfg.precision, srv->tile_flag()) > srv->cfg.hbm_budget_bytes)
            return fail(MMOT_ERR_NOMEM, "request footprint exceeds the server's HBM budget");
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) return fail(MMOT_ERR_STATE, "server is stopping");
        r->ticket = srv->next_ticket++;
        r->t_submit = now_s();
        *ticket = r->ticket;
        srv->queue.push_back(std::move(r));
        srv->cv.notify_all();
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_serve_poll(mmot_server_t *srv, uint64_t ticket, mmot_request_record *rec, double *log_phi_out)
{
    try {
        if (!srv || !rec) return fail(MMOT_ERR_INVALID, "NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->error) return fail(srv->error, srv->error_msg);
        auto it = srv->done.find(ticket);
        if (it == srv->done.end()) {
            if (ticket == 0 || ticket >= srv->next_ticket) return fail(MMOT_ERR_STATE, "unknown ticket");
            return 0;
        }
        *rec = it->second.rec;
        if (log_phi_out) std::memcpy(log_phi_out, it->second.log_phi.data(), sizeof(double) * it->second.log_phi.size());
        return 1;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_serve_cancel(mmot_server_t *srv)
{
    try {
        if (!srv) return fail(MMOT_ERR_INVALID, "NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        const double t = now_s();
        for (auto &r : srv->queue) {
            Done d;
            std::memset(&d.rec, 0, sizeof d.rec);
            d.rec.result.status = MMOT_ERR_STATE;
            d.rec.result.l = r->l;
            d.rec.result.N = r->N;
            d.rec.result.marg_err = INFINITY;
            d.rec.t_submit = r->t_submit;
            d.rec.t_admit = t;
            d.rec.t_done = t;
            srv->done[r->ticket] = std::move(d);
        }
        srv->queue.clear();
        srv->cancel = true;
        srv->stopping = true;
        srv->cv.notify_all();
        return MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_serve_stop(mmot_server_t *srv)
{
    try {
        if (!srv) return MMOT_OK;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stopping = true;
        }
        srv->cv.notify_all();
        if (srv->th.joinable()) srv->th.join();
        const int err = srv->error;
        const std::string msg = srv->error_msg;
        (void)hipFree(srv->base);
        batch_buffers_free(&srv->bb);
        (void)hipStreamDestroy(srv->s);
        delete srv;
        return err ? fail(err, msg) : MMOT_OK;
    } catch (...) {
        return guard_fail();
    }
}

int mmot_serve(const mmot_serve_cfg *cfg, mmot_request_fn next, void *user, mmot_serve_stats *stats,
               mmot_request_record *records, int64_t max_records)
{
    try {
        if (!cfg || !next || !stats) return fail(MMOT_ERR_INVALID, "NULL argument");
        mmot_server_t *srv = nullptr;
        int rc = mmot_serve_start(cfg, &srv);
        if (rc) return rc;
        std::vector<uint64_t> tickets;
        int64_t rejected = 0;
        const double t0 = now_s();
        for (int64_t idx = 0;; ++idx) {
            mmot_request req;
            double t_arr = 0.0;
            if (next(user, idx, &req, &t_arr) != 0) break;
            const double wait = t0 + t_arr - now_s();
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            uint64_t tk = 0;
            rc = mmot_serve_submit(srv, &req, &tk);
            if (rc == MMOT_ERR_NOMEM || rc == MMOT_ERR_INVALID || rc == MMOT_ERR_UNSUPPORTED) {
                // footprint above the whole budget, or a request the library does not take:
                // counted as rejected, the others are served
                ++rejected;
                continue;
            }
            if (rc) {
                mmot_serve_stop(srv);
                return rc;
            }
            tickets.push_back(tk);
        }
        std::vector<double> lat;
        double units = 0.0, t_last = t0;
        int64_t k = 0;
        for (uint64_t tk : tickets) {
            mmot_request_record rec;
            for (;;) {
                rc = mmot_serve_poll(srv, tk, &rec, nullptr);
                if (rc == 1) break;
                if (rc < 0) {
                    mmot_serve_stop(srv);
                    return rc;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(200));
            }
            lat.push_back(rec.t_done - rec.t_submit);
            units += (double)rec.result.l * (double)rec.result.N * (double)rec.result.iters;
            t_last = std::max(t_last, rec.t_done);
            if (records && k < max_records) records[k] = rec;
            ++k;
        }
        rc = mmot_serve_stop(srv);
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double q) {
            if (lat.empty()) return 0.0;
            const size_t i = std::min(lat.size() - 1, (size_t)std::ceil(q * (double)lat.size()) - (q > 0 ? 1 : 0));
            return lat[i];
        };
        stats->completed = (int64_t)lat.size();
        stats->rejected = rejected;
        stats->wall_seconds = t_last - t0;
        stats->p50_latency = pct(0.50);
        stats->p99_latency = pct(0.99);
        stats->units_per_second = stats->wall_seconds > 0 ? units / stats->wall_seconds : 0.0;
        return rc;
    } catch (...) {
        return guard_fail();
    }
}

}  // extern "C"
