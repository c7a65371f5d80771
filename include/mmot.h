/*
 * mmot.h -- C ABI of libmmot, entropic multi-marginal optimal transport with
 * L1 cost on a uniform 1-D grid, solved by Gauss-Seidel Sinkhorn whose
 * tensor-vector products run in O(N) per marginal on an MI355X (gfx950).
 *
 * Problem (Sec. 2 and Sec. 4.2 of arXiv:2405.19246).  l probability vectors
 * u_1..u_l of common length N live on a uniform grid of step h.  The cost of an
 * index tuple is c(i_1..i_l) = h * sum_{p<q} |i_p - i_q|, the Gibbs kernel is
 * K = exp(-c / eps) = lambda^{sum |i_p - i_q|} with lambda = exp(-h / eps), and
 * the entropic plan has the Gibbs form t = K * prod_q phi_q(i_q).  Sinkhorn
 * updates phi_j <- u_j / (K x_{q != j} phi_q) for j = 1..l in order, each
 * product using the newest phi's (Gauss-Seidel, Sec. 4.2 update formulas).
 *
 * Conventions shared by every entry point:
 *  - Scaling vectors are passed as log-potentials a_q = log phi_q (natural
 *    log, FP64), row-major [l][N]; marginals as log u_q, FP64 [l][N].  A zero
 *    marginal entry is log u = -inf and gives a = -inf (phi = 0).
 *  - "device" pointers are HIP device memory on the current device (e.g. the
 *    data pointer of a torch CUDA tensor); "host" pointers are CPU memory.
 *    The caller owns every buffer it passes; the library never frees them.
 *  - Work is enqueued on the plan's HIP stream (NULL = default stream).
 *    Entry points that return host values synchronise that stream first.
 *  - Return value: MMOT_OK (0) or a negative MMOT_ERR_* code; the message of
 *    the last error on the calling thread is mmot_last_error().  No C++
 *    exception crosses this interface.
 *  - precision MMOT_FP64: every scan runs in FP64 mantissas.  MMOT_FP32: the
 *    scans of the Sinkhorn updates run in FP32 mantissas with exact integer
 *    power-of-two exponents per value; potentials, the marginal-error check and
 *    the objective stay FP64.
 */
#ifndef MMOT_H
#define MMOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MMOT_OK 0
#define MMOT_ERR_INVALID (-1)     /* bad argument: l < 2, l > MMOT_MAX_L, N < 1, eps <= 0, h <= 0, j out of range, NULL */
#define MMOT_ERR_NOMEM (-2)       /* device or host allocation failed */
#define MMOT_ERR_NUMERIC (-3)     /* a NaN or infinity appeared in a potential, the residual or the objective */
#define MMOT_NOT_CONVERGED (-4)   /* itr_max reached with residual > tol; outputs are still written */
#define MMOT_ERR_UNSUPPORTED (-5) /* valid request the library does not implement */
#define MMOT_ERR_HIP (-6)         /* a HIP runtime call failed (message names it) */
#define MMOT_ERR_STATE (-7)       /* server stopped, unknown ticket, or call out of order */
#define MMOT_ERR_INTERNAL (-8)    /* unexpected failure inside the library (host resources; message names it) */

#define MMOT_MAX_L 10             /* largest number of marginals per problem */

#define MMOT_FP64 0
#define MMOT_FP32 1

/* One problem shape: l marginals of length N on a grid of step h, entropic eps. */
typedef struct {
    int32_t l;
    int64_t N;
    double h;
    double eps;
    int32_t precision; /* MMOT_FP64 or MMOT_FP32 */
    const double *x;   /* NULL: the uniform grid of step h.  Otherwise a non-uniform grid shared by
                          the l marginals (Sec. 3 remarks that the method carries over to one): host
                          [N] coordinates, finite and non-decreasing (MMOT_ERR_INVALID otherwise),
                          copied by mmot_plan; h is then ignored.  The cost becomes
                          sum_{p<q} |x[i_p] - x[i_q]| and gap k's factor exp(-(x[k+1] - x[k])
                          m (l - m) / eps).  Marginals with different supports are given on the
                          union of the supports with zero mass off their own.  Such problems run
                          on the tiled kernels (any N) in the plan's precision. */
} mmot_problem;

/* Marginals passed to the solving calls (mmot_sinkhorn_iter, mmot_solve,
 * mmot_solve_batch, mmot_serve_submit) must be probability vectors: no NaN,
 * no negative mass (in log form: no NaN and no +inf), and each row's mass
 * sum_i exp(log_u[q][i]) within 1e-12 of 1 in FP64; otherwise the call returns
 * MMOT_ERR_INVALID naming the instance and row, before any sweep runs (the
 * device-pointer calls check on the device first, then synchronise). */

/* Stopping rule of Alg. 1: stop after itr_max sweeps or once Res <= tol, where
 * Res = sum_{j < l} || phi_j * (K x_{q != j} phi_q) - u_j ||_1 (the last marginal
 * is exact after its own update) is evaluated in FP64 after every check_every-th
 * sweep (check_every > 0), after the last sweep, and whenever the sweep's own
 * estimate -- the marginal errors its updates removed, sum over j < l-1 of
 * sum_y u_j(y) |phi_j,old(y) / phi_j,new(y) - 1| -- falls below tol * f, where f
 * starts at 1 and halves after each such check that does not reach tol.
 * tol < 0 never stops early (and never uses the estimate).
 * flags: MMOT_FLAG_WARM_START keeps the potentials passed in instead of
 * starting from phi = 1/N (Alg. 1 init); MMOT_FLAG_NO_FAST runs every solve on
 * the extended-range solver (one wavefront per solve) instead of the
 * register-resident one (one workgroup per solve, taken when N fits it);
 * MMOT_FLAG_TILES cuts every instance into tiles (otherwise only long ones:
 * N >= 16384 for l <= 6, N >= 4096 for l >= 7, or, in a batch with fewer than
 * 512 instances off the register-resident path, every such instance from
 * N = 256 up; not with MMOT_FLAG_NO_FAST); MMOT_FLAG_NO_GRAPH launches
 * the tiled sweeps one by one instead of replaying a captured HIP graph of a
 * block of sweeps (same iterates, bit for bit).
 * MMOT_FLAG_JACOBI (mmot_plan only: honoured by mmot_solve and
 * mmot_sinkhorn_iter; mmot_solve_batch rejects it): the all-marginals variant
 * instead of the paper's Gauss-Seidel order (Sec. 4.2).  Every sweep forms the
 * l products from the potentials at the start of the sweep, then moves each
 * a_j by 1/l of its own update, a_j <- a_j + (log u_j - a_j - log J_j) / l: the
 * mean of the l block updates, so the dual never decreases and the iterates
 * reach the same (unique) plan.  Its residual sums the errors of all l
 * marginals and is checked every check_every sweeps (every 10 if 0) and after
 * the last; no estimate. */
typedef struct {
    double tol;
    int64_t itr_max;
    int32_t check_every;
    int32_t flags;
} mmot_opts;

#define MMOT_FLAG_WARM_START 1
#define MMOT_FLAG_NO_FAST 2
#define MMOT_FLAG_TILES 4
#define MMOT_FLAG_NO_GRAPH 8
#define MMOT_FLAG_JACOBI 16

/* Per-solve outcome. */
typedef struct {
    double W;          /* W_eps = <C, T>, transport cost of the plan (Sec. 2 Eq. mmot distance), FP64 */
    double marg_err;   /* last Res (FP64), see mmot_opts */
    int64_t iters;     /* sweeps done */
    int32_t status;    /* MMOT_OK, MMOT_NOT_CONVERGED or MMOT_ERR_NUMERIC */
    int32_t l;
    int64_t N;
} mmot_result;

typedef struct mmot_plan mmot_plan_t;

/*
 * Build an execution plan for one problem shape: validates the problem,
 * derives lambda = exp(-h/eps) and the discount tables of the scans, picks the
 * launch shape and allocates the device workspace (constants, scan
 * checkpoints, result slot).  This is not the transport plan.
 * hip_stream: a hipStream_t or NULL.  *out receives the plan (caller destroys it).
 */
int mmot_plan(const mmot_problem *p, const mmot_opts *o, void *hip_stream, mmot_plan_t **out);

/* Device bytes the plan holds, plus the caller buffers one solve needs
 * (2 * l * N doubles), for admission by HBM footprint. */
int mmot_plan_footprint(const mmot_plan_t *plan, size_t *device_bytes);

int mmot_plan_destroy(mmot_plan_t *plan);

/*
 * One tensor-vector product (Sec. 4.2 Eq. for J^{(l)}; Sec. 3.1 FTVP-1 for l = 3):
 *   log_J[y] = log sum_{i_q, q != j; i_j = y} K(i) prod_{q != j} phi_q(i_q).
 * j: 0-based marginal index.  log_phi: device [l][N] FP64, row j ignored.
 * log_J: device [N] FP64, written.  Runs in the plan's precision.
 */
int mmot_marginal_product(const mmot_plan_t *plan, int32_t j, const double *log_phi, double *log_J);

/*
 * The same product from its definition, for comparison at small sizes: the sum
 * over all N^(l-1) index tuples of the other marginals (Sec. 2, the
 * tensor-vector product with the Gibbs kernel; Alg. 1 as written), O(N^l) work,
 * FP64 log-sum-exp on the device, any plan precision.  Arguments as in
 * mmot_marginal_product; the plan's grid (uniform or coordinates) sets the cost.
 * MMOT_ERR_UNSUPPORTED unless l <= 6, (l + 1) N <= 6144 and N^(l-1) < 2^31.
 */
int mmot_dense_marginal_product(const mmot_plan_t *plan, int32_t j, const double *log_phi, double *log_J);

/*
 * n_sweeps Gauss-Seidel sweeps (Alg. 1 update lines) with the dense product
 * above, FP64, no residual, from the potentials in log_phi (warm start).
 * log_u: device [l][N]; log_phi: device [l][N], in/out.  Asynchronous on the
 * plan's stream.  Same size limits as mmot_dense_marginal_product.
 */
int mmot_dense_sinkhorn_iter(const mmot_plan_t *plan, const double *log_u, double *log_phi, int64_t n_sweeps);

/*
 * n_sweeps Gauss-Seidel sweeps (Alg. 1 loop body, l updates each) starting
 * from the potentials in log_phi, no early stop; warm start = resume.
 * log_u: device [l][N].  log_phi: device [l][N], in/out.
 * marg_err: host, nullable; if given, Res after the last sweep is computed in
 * FP64 and the stream is synchronised.
 */
int mmot_sinkhorn_iter(const mmot_plan_t *plan, const double *log_u, double *log_phi, int64_t n_sweeps,
                       double *marg_err);

/*
 * Whole solve in one launch (Alg. 1 / Alg. FS-3): start from phi = 1/N unless
 * MMOT_FLAG_WARM_START, iterate until Res <= tol or itr_max, then compute W_eps
 * in FP64.  log_u: device [l][N].  log_phi: device [l][N] out (in/out with
 * warm start).  res: host, written after the stream is synchronised.  Returns
 * MMOT_OK, MMOT_NOT_CONVERGED or an error; res->status carries the same.
 */
int mmot_solve(const mmot_plan_t *plan, const double *log_u, double *log_phi, mmot_result *res);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * of mmot_marginal_product for the problem p, without a plan.  Its workspace
 * (the problem descriptor and the scan checkpoints) is a fixed device array of
 * MMOT_NOALLOC_BYTES per GPU, set up on the first call on each device and held
 * until the process ends; no call allocates.  Problems whose workspace would
 * exceed it are rejected with MMOT_ERR_INVALID before any device work.  Every
 * call on one GPU shares that GPU's workspace: calls that overlap on one GPU
 * (other streams or threads) race.  Uniform grids only (p->x must be NULL:
 * MMOT_ERR_UNSUPPORTED otherwise).  Runs the single-pass kernels (no tiles)
 * in p->precision on hip_stream (NULL = default).  j, log_phi, log_J as in
 * mmot_marginal_product.
 */
#define MMOT_NOALLOC_BYTES (16u << 20)
int mmot_marginal_product_noalloc(const mmot_problem *p, int32_t j, const double *log_phi, double *log_J,
                                  void *hip_stream);

/* W_eps = <C, T> of the plan with potentials log_phi (Sec. 2 Eq. mmot distance;
 * Sec. 3.2 FTVP-2 for l = 3), FP64.  W: host, synchronises. */
int mmot_objective(const mmot_plan_t *plan, const double *log_phi, double *W);

/* FP64 L1 errors of all l marginals of the plan with potentials log_phi:
 * err[j] = || phi_j * (K x_{q != j} phi_q) - u_j ||_1.  err: host [l], synchronises. */
int mmot_marginal_errors(const mmot_plan_t *plan, const double *log_u, const double *log_phi, double *err);

/*
 * Three marginals on an N x M grid with separable L1 cost (Sec. 4.1):
 *   c = h1 (|i1 - j1| + |i1 - k1| + |j1 - k1|) + h2 (|i2 - j2| + |i2 - k2| + |j2 - k2|).
 * A marginal (and its potentials, products, errors) is a device array [M][N] of
 * FP64: entry (i1, i2) at i2 N + i1, the paper's column-major flattening; the
 * three of a solve are stacked as [3][M][N].  Everything runs in FP64: each
 * product is a scan along the second axis whose steps are 6 M independent 1-D
 * three-marginal products of length N (Sec. 4.1 recurrences, O(N M) work).
 * Plans take MMOT_FLAG_WARM_START only (MMOT_ERR_UNSUPPORTED otherwise); the
 * stopping rule checks the FP64 residual every check_every sweeps (every 10 if
 * 0) and after the last.
 */
typedef struct {
    int64_t N;   /* points along the first axis (spacing h1) */
    int64_t M;   /* points along the second axis (spacing h2) */
    double h1;
    double h2;
    double eps;
} mmot_problem_2d;

typedef struct mmot_plan_2d mmot_plan_2d_t;

int mmot_plan_2d(const mmot_problem_2d *p, const mmot_opts *o, void *hip_stream, mmot_plan_2d_t **out);
int mmot_plan_2d_destroy(mmot_plan_2d_t *plan);

/* log_J[y][x] = log (K x_{q != j} phi_q)(x, y), j in 0..2 (Sec. 4.1 Eq. for J_{k1 k2}).
 * log_phi: device [3][M][N], row j ignored; log_J: device [M][N]. */
int mmot_marginal_product_2d(const mmot_plan_2d_t *plan, int32_t j, const double *log_phi, double *log_J);

/* Gauss-Seidel sweeps (Sec. 4.1 update formulas) from phi = 1/(N M) unless warm,
 * until Res = err_0 + err_1 <= tol or itr_max, then W_eps = <C, T> in FP64.
 * log_u: device [3][M][N], probability vectors (MMOT_ERR_INVALID otherwise);
 * log_phi: device [3][M][N] out.  res: host; res->N is N M. */
int mmot_solve_2d(const mmot_plan_2d_t *plan, const double *log_u, double *log_phi, mmot_result *res);

/* W_eps = <C, T> of the plan with potentials log_phi (Sec. 4.1 Eq. 2-D distance).  W: host. */
int mmot_objective_2d(const mmot_plan_2d_t *plan, const double *log_phi, double *W);

/* FP64 L1 errors of the three marginals of the plan.  err: host [3]. */
int mmot_marginal_errors_2d(const mmot_plan_2d_t *plan, const double *log_u, const double *log_phi, double *err);

/* One instance of a batch.  log_u / log_phi: device [l][N].  x: NULL (uniform grid of
 * step h) or device [N] coordinates of a non-uniform grid (as mmot_problem.x; checked on
 * the device before any sweep). */
typedef struct {
    int32_t l;
    int64_t N;
    double h;
    double eps;
    const double *log_u;
    double *log_phi;
    const double *x;
} mmot_instance;

/*
 * Solve `count` independent instances of mixed l, N, eps.  Instances whose N
 * fits one workgroup (l <= 4, N <= 1024) run on the register-resident path:
 * rounds of a sweep kernel (one workgroup per instance, until the stopping
 * estimate asks for a check) and an FP64 check kernel.  All others run in one
 * persistent launch of the extended-range solver, one wavefront per instance
 * taking the next unsolved one (largest estimated work first) until none is
 * left.  When one l has more register-resident instances than the device
 * holds at once (768), the first round gives each of them 256 sweeps and
 * pauses (no check); the later rounds take them longest-predicted first (from
 * the estimate's decay over sweeps 128..256), so that the slowest solves
 * start early.  None of this changes an instance's iterates: they are those
 * of solving it alone.  Stopping as in mmot_solve (FP64 residual, estimate-
 * triggered or every o->check_every sweeps, and after the last), then the FP64
 * objective.  precision as in mmot_problem.  res: host [count], written after
 * synchronising hip_stream.  Returns MMOT_OK if every instance converged,
 * MMOT_NOT_CONVERGED if some hit itr_max, MMOT_ERR_NUMERIC if some failed;
 * per-instance status is in res.
 */
int mmot_solve_batch(const mmot_instance *inst, int32_t count, int32_t precision, const mmot_opts *o,
                     void *hip_stream, mmot_result *res);

/* Device time in milliseconds of the last mmot_solve_batch call: from a HIP
 * event recorded on its stream before its first kernel to one after its last
 * (descriptor uploads before, the result copy after are outside; the host
 * round trips between rounds of the register-resident path are inside).
 * *ms: host.  MMOT_ERR_STATE before the first call. */
int mmot_last_batch_kernel_ms(double *ms);

/* Breakdown of the last mmot_solve_batch call, from HIP events around each
 * kernel launch on its stream. */
typedef struct {
    double total_ms;        /* as mmot_last_batch_kernel_ms */
    double sweep_ms;        /* sum over the sweep-kernel launches (register-resident path) */
    double check_ms;        /* sum over the FP64 check-kernel launches */
    double other_ms;        /* extended-range solver launches and the objective kernel */
    double sweep_units;     /* l * N * sweeps done by the sweep-kernel launches */
    int32_t sweep_launches; /* number of sweep-kernel launches */
    int32_t rounds;         /* sweep + check rounds */
} mmot_batch_timing;

int mmot_last_batch_timing(mmot_batch_timing *t);

/* ---------------- serving (continuous batching) ---------------- */

typedef struct mmot_server mmot_server_t;

typedef struct {
    int32_t precision;        /* MMOT_FP64 / MMOT_FP32 */
    mmot_opts opts;           /* per-request stopping rule */
    int32_t max_slots;        /* instances resident on the device at once */
    int64_t block_sweeps;     /* sweeps each resident solve advances per device round */
    size_t hbm_budget_bytes;  /* admission limit on the summed device footprint */
} mmot_serve_cfg;

/* A request: marginals are host memory, copied at admission. */
typedef struct {
    int32_t l;
    int64_t N;
    double h;
    double eps;
    const double *u;          /* host [l][N], probability vectors */
} mmot_request;

/* Per-request record.  Times are seconds on the server's monotonic clock. */
typedef struct {
    mmot_result result;
    double t_submit;
    double t_admit;
    double t_done;
} mmot_request_record;

/*
 * Start a server thread that owns a HIP stream and a device arena.  Requests
 * submitted while others are running are admitted into free slots at the next
 * device-round boundary when their footprint fits the HBM budget; resident
 * solves keep their potentials on the device across rounds.
 */
int mmot_serve_start(const mmot_serve_cfg *cfg, mmot_server_t **out);

/* Queue a request (marginals copied before return).  *ticket identifies it. */
int mmot_serve_submit(mmot_server_t *srv, const mmot_request *req, uint64_t *ticket);

/* Non-blocking: 1 and *rec filled if the request finished, 0 if not yet, <0 error.
 * log_phi_out: host [l][N] or NULL, receives the final potentials. */
int mmot_serve_poll(mmot_server_t *srv, uint64_t ticket, mmot_request_record *rec, double *log_phi_out);

/* Finish queued and running work, stop the thread, free the device arena. */
int mmot_serve_stop(mmot_server_t *srv);

/* Shed the load: requests still queued are finished at once with status
 * MMOT_ERR_STATE (not started), requests on the device end after the current
 * device round with their last residual (status MMOT_NOT_CONVERGED unless it
 * met tol), and no new request is accepted.  Does not wait; mmot_serve_stop
 * then returns after at most that round. */
int mmot_serve_cancel(mmot_server_t *srv);

/* Summary of a blocking serving run. */
typedef struct {
    int64_t completed;
    int64_t rejected;          /* refused at submission: footprint above the whole budget, or a request
                                  mmot_serve_submit rejects (e.g. l > MMOT_MAX_L); the rest are served */
    double wall_seconds;
    double p50_latency;        /* seconds, submit to done */
    double p99_latency;
    double units_per_second;   /* sum over requests of l * N * iters / wall time */
} mmot_serve_stats;

/* Callback for the blocking server: fill *req and *t_arrive (seconds from the
 * start) for request number `index`; return 0 to submit it, 1 when there are no
 * more requests.  The request's u must stay valid until the call returns. */
typedef int (*mmot_request_fn)(void *user, int64_t index, mmot_request *req, double *t_arrive);

/*
 * Blocking serving loop: submits each request at its arrival time (open loop),
 * runs until all are done, fills *stats; records: host array of at least the
 * number of requests, or NULL.
 */
int mmot_serve(const mmot_serve_cfg *cfg, mmot_request_fn next, void *user, mmot_serve_stats *stats,
               mmot_request_record *records, int64_t max_records);

/* Message of the last error on this thread (empty string if none). */
const char *mmot_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MMOT_H */
