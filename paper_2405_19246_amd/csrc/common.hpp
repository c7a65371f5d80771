// Definitions shared by the host runtime and the device kernels of libmmot.
#pragma once
#include <stdint.h>

namespace mmot {

constexpr int MAXL = 10;  // largest number of marginals (MMOT_MAX_L)
constexpr int MAXV = 8;   // largest number of grid positions one lane owns per chunk
constexpr int WAVE = 64;  // CDNA wavefront width

// Exponent that marks zero.  Far below any real value's exponent and far from
// int32 overflow when a few are added.
constexpr int32_t XF_ZERO_E = -(1 << 26);

// Extended-range floating point: value = m * 2^e with m a float or double
// mantissa (normalised to [0.5, 1) after additions, 0 for zero) and an exact
// int32 power-of-two exponent.  It plays the role of a log-sum-exp shift that
// is exact: no value of the transport problem over- or underflows, whatever
// the size of the potentials, and adding two values costs one alignment.
template <typename M>
struct XF {
    M m;
    int32_t e;
};

// A discount factor g^p as an extended-range value whose mantissa is carried
// to twice the working precision (hi + lo): the factors are applied again and
// again along a scan, so a mantissa rounded once would bias every result.
template <typename M>
struct XG {
    M hi;
    M lo;
    int32_t e;
    int32_t pad;
};

// Discount constants of one instance for scans of width V, mantissa M.
// g(k) = lambda^{k (l - k)} is the factor a state with k of the l - 1 summed
// marginals already placed picks up per grid gap (gap form of the L1 cost).
template <typename M>
struct Disc {
    XG<M> g1[MAXL];           // g(k)
    XG<M> gstep[MAXL][6];     // g(k)^(V * 2^s), Kogge-Stone steps across lanes
    XG<M> gfix[MAXL][MAXV];   // g(k)^(t + 1), carry fix-up inside a lane
    double lgV[MAXL];         // V * ln g(k), for the per-lane power g(k)^(V * lane)
    double ck[MAXL + 1];      // k (l - k), gap count weight for the objective
    int32_t V;
    int32_t pad;
};

// Shape and discount constants of one problem (written once, read-only).
struct Inst {
    int64_t N;
    int32_t l;
    int32_t pad;
    double h;
    double hoe;           // h / eps
    Disc<float> d32;      // FP32 update scans
    Disc<double> d64;     // FP64 update and check scans
    Disc<double> dob;     // FP64 objective scans (value, cost-weighted value)
    Disc<double> dck;     // FP64 residual-check scans
    const double *x;      // non-uniform grid: coordinates [N] on the device (team and tile walks
                          // only); null for the uniform grid of step h
    double ieps;          // 1 / eps
};

// Buffers of one solve (caller-owned except scratch).
struct Ptrs {
    const double *log_u;  // [l][N] log marginals
    double *a;            // [l][N] log potentials (in/out)
    double *out;          // [N] product output (log J), product mode only
    void *scratch;        // per-chunk scan checkpoints
    int64_t itr_cap;      // sweeps allowed for this instance in this launch (0: RunOpts.itr_max)
    int64_t it0;          // sweeps already done (resumed solves)
    int32_t flags;        // OR-ed with RunOpts.flags
    int32_t j0;           // resumed solves: sweep it0 goes on at marginal j0 (l: sweep done, check first)
};

// Progress of one fast-path solve across the sweep and check launches.
struct Track {
    double f;         // the estimate asks for a check once it falls below tol * f
    double est;       // marginal-error estimate of the last sweep
    double res;       // last FP64 residual (+inf before the first)
    int64_t it;       // sweeps done
    int32_t state;    // TS_*
    int32_t status;   // final status once state is TS_DONE
    int32_t j0;       // TS_ROBUST: marginal at which the extended-range solver resumes
    int32_t checked;  // a residual has been taken
    double est_mid;   // estimate half-way through a launch with a sweep budget
};
constexpr int32_t TS_SWEEP = 0;   // the sweep kernel goes on with it
constexpr int32_t TS_CHECK = 1;   // a residual check is due
constexpr int32_t TS_ROBUST = 2;  // the extended-range solver takes it over
constexpr int32_t TS_DONE = 3;

// Stopping rule of one launch.
struct RunOpts {
    double tol;           // stop once Res <= tol (tol < 0: never early)
    int64_t itr_max;      // sweeps in this launch
    int32_t check_every;  // Res every this many sweeps (0: only after the last)
    int32_t flags;
    int32_t budget;       // register-resident sweeps: pause after this many sweeps of a launch (0: none)
    int32_t warmup;       // batch host: sweeps of the first round, after which the batch is reordered (0: none)
};

// What a marginal pass does with log J_j (scan.hpp finish_lj, wide.hpp).
enum PassMode { P_PRODUCT = 0, P_UPDATE = 1, P_CHECK = 2, P_OBJECTIVE = 3 };

// Same layout as mmot_result.
struct Result {
    double W;
    double marg_err;
    int64_t iters;
    int32_t status;
    int32_t l;
    int64_t N;
};

// Inst.flags
constexpr int32_t F_WARM = 1;        // keep the given potentials
constexpr int32_t F_NO_CHECK = 2;    // no residual check at all
constexpr int32_t F_NO_OBJ = 4;      // skip the objective
constexpr int32_t F_NO_FAST = 8;     // host only: every instance on the extended-range solver
constexpr int32_t F_TILES = 16;      // host only: every instance is tiled (tests and small shapes)
constexpr int32_t F_VALIDATE = 32;   // host only: check the marginals before solving
constexpr int32_t F_NO_GRAPH = 64;   // host only: tiled sweep blocks launched one by one, not as a graph
constexpr int32_t F_TILE_SMALL = 128; // host only: tile from N = TILE_SMALL_N (a batch too small to fill the GPU)
constexpr int TILE_SMALL_N = 256;     // shortest tiled instance in a small batch
constexpr int SMALL_BATCH = 512;      // fewer instances off the register-resident path than this: small batch
constexpr int TILE_GRAPH_SWEEPS = 8; // sweeps per captured block of a tiled solve

// Lane width V per (l, pass kind) -- trades registers against scan overhead.
// kind 0: FP32 update, 1: FP64 update and product, 2: FP64 objective
// (value, weighted value), 3: FP64 residual check.
constexpr int vsel(int l, int kind)
{
    return kind == 0 ? (l <= 3 ? 8 : l == 4 ? 4 : l == 5 ? 2 : 1)
         : kind == 1 ? (l <= 2 ? 8 : l == 3 ? 4 : l == 4 ? 2 : 1)
         : kind == 2 ? (l <= 2 ? 2 : 1)
                     : (l <= 2 ? 4 : l == 3 ? 2 : 1);
}

// Register-resident fast path (fast.hpp): positions per thread V and threads
// per workgroup by l and precision (1: FP32 sweeps, 0: FP64); an instance fits if
// N <= fast_threads * fast_v.
constexpr int FAST_MAXL = 4;            // largest l the fast path is built for
constexpr bool FAST_PATH_ENABLED = true;  // host routing to the fast path (see fast_eligible)
constexpr int fast_v(int l, int precision)
{
    return precision == 1 ? (l <= 4 ? 4 : l == 5 ? 2 : 1) : (l <= 4 ? 2 : 1);
}
constexpr int fast_threads(int l, int precision) { return precision == 1 || l >= 6 ? 256 : 512; }
constexpr long fast_capacity(int l, int precision) { return (long)fast_threads(l, precision) * fast_v(l, precision); }
// Wavefronts per SIMD the FP32 sweep kernel is compiled for: three blocks of
// four wavefronts per compute unit fit its LDS, and the registers then come to
// 168 per lane (a few values of the outer loops spill).
constexpr int fast_waves_per_eu(int precision) { return precision == 1 ? 3 : 1; }
// Batches larger than the workgroups resident at once (three per compute unit)
// start with a warm-up round of this many sweeps and are then reordered,
// longest predicted solve first.
constexpr int FAST_RESIDENT = 768;
constexpr int FAST_WARMUP_SWEEPS = 256;
// Groups up to this size are reordered after the warm-up on the device (one
// workgroup sorts them in LDS); larger ones by the host.
constexpr int FAST_ORDER_MAX = 4096;
// Pairs of sweep and check launches enqueued back to back after the reordering
// before the host reads the solves' states (a pair with nothing left to do costs
// two near-empty launches).
constexpr int FAST_PAIRS = 4;

// Block floating point holds while the values one thread keeps span at most
// this many bits: rows of l - 1 marginals (row_spread bits each), v positions
// of discount (decay_bits each), and the product of a forward and a backward
// state in the combine must stay normal (FP32: 2^-126, FP64: 2^-1022).
constexpr bool bf_fits_range(int precision, int l, int v, int row_spread, int decay_bits)
{
    return 2 * ((l - 1) * row_spread + v * decay_bits + l + 4) <= (precision == 1 ? 120 : 1000);
}

// Bytes of one scan element of each kind (for checkpoint storage).
constexpr int elem_bytes(int kind) { return kind == 0 ? 8 : kind == 2 ? 32 : 16; }

// Team layout of the subset-state solver (wide.hpp) for l marginals: the
// 2^(l-1) states of a position are spread over TL lanes and RG registers per
// lane.  Element kinds: words = live 32-bit registers of one element (FP32
// extended value 2, FP64 3, FP64 value + cost-weighted value 6), bytes = its
// size in memory.
constexpr int WIDE_MINL = 7;   // l from which batches and plans use the team layout
constexpr int WIDE_MAXL = 10;  // largest l the team layout is built for
constexpr int wide_states(int l) { return 1 << (l - 1); }
// lanes per team: the states of l <= 4 one per lane; beyond, 16 lanes (the
// lane moves stay inside DPP rows) with up to 8 states per lane, growing to 32
// and 64 lanes for l = 9, 10 so that the FP64 states of a lane stay near 8
constexpr int wide_tl(int l)
{
    return l <= 4 ? wide_states(l) : (wide_states(l) / 8 > 16 ? wide_states(l) / 8 : 16);
}
constexpr int wide_rg(int l) { return wide_states(l) / wide_tl(l); }
// positions per recompute block: about 48 registers of forward states per lane
constexpr int wide_ck(int l, int words)
{
    return 48 / (wide_rg(l) * words) < 1 ? 1 : (48 / (wide_rg(l) * words) > 16 ? 16 : 48 / (wide_rg(l) * words));
}
// Where blocks hold at most two positions the forward walk keeps the state after
// every position (at most twice the memory of the block checkpoints) and the
// backward walk reads it instead of recomputing it.
constexpr bool wide_store_all(int l, int words) { return wide_ck(l, words) <= 2; }
// checkpoint bytes of one pass over len positions
constexpr long wide_ck_bytes(int l, int words, int bytes, long len)
{
    return (wide_store_all(l, words) ? len : (len + wide_ck(l, words) - 1) / wide_ck(l, words)) *
           (long)wide_states(l) * (long)bytes;
}
// checkpoint bytes of one instance: the largest over the FP32, FP64 and objective passes
constexpr long wide_scratch_bytes(int l, long N)
{
    return wide_ck_bytes(l, 2, 8, N) > wide_ck_bytes(l, 3, 16, N)
               ? (wide_ck_bytes(l, 2, 8, N) > wide_ck_bytes(l, 6, 32, N) ? wide_ck_bytes(l, 2, 8, N)
                                                                         : wide_ck_bytes(l, 6, 32, N))
               : (wide_ck_bytes(l, 3, 16, N) > wide_ck_bytes(l, 6, 32, N) ? wide_ck_bytes(l, 3, 16, N)
                                                                          : wide_ck_bytes(l, 6, 32, N));
}

// Per-instance buffers and shape of a tiled solve.
struct TileInst {
    int32_t ntile;   // tiles
    int32_t B;       // positions per tile (the last may be shorter)
    char *agg;       // [ntile][2][l][2^(l-1)] elements: Q_m, m = 0..l-1 (index space of the team)
    char *carry;     // [ntile][2][2^(l-1)] elements: state entering each tile (index space)
    char *ck;        // [ntile][ck_stride] checkpoint scratch of the final passes
    double *part;    // [l][ntile] per-tile sums of the update / check passes
    long ck_stride;  // bytes of checkpoint scratch per tile
};

// State of one instance across the launches of a tiled solve.
struct TileTrack {
    double f;        // the estimate asks for a check once it falls below tol * f
    double est;      // marginal-error estimate of the last sweep
    double res;      // last FP64 residual (+inf before the first)
    int64_t it;      // sweeps done
    int32_t state;   // TS_SWEEP, TS_CHECK or TS_DONE
    int32_t status;  // final status once TS_DONE
    int32_t checked; // a residual has been taken
    int32_t pad;
};

constexpr int32_t TS_OBJ = 4;  // tiled solves: objective pending

}  // namespace mmot
