// Host-side tables of libmmot: discount factors, device descriptors and
// checkpoint sizes.  Plain C++ (no HIP calls), shared by the runtime and the
// serving loop.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstring>
#include <cmath>

namespace mmot {
namespace rt {

namespace {
constexpr double H_LN2_HI = 6.93147180369123816490e-01;
constexpr double H_LN2_LO = 1.90821492927058770002e-10;
constexpr double H_LOG2E = 1.44269504088896338700e+00;

// exp(lognat) as a discount factor with a hi + lo mantissa.
template <typename M>
XG<M> host_xg(double lognat)
{
    if (!(lognat > -1.0e15)) return {M(0), M(0), XF_ZERO_E, 0};
    const double k = std::nearbyint(lognat * H_LOG2E);
    double r = std::fma(-k, H_LN2_HI, lognat);
    r = std::fma(-k, H_LN2_LO, r);
    int ex = 0;
    const double vm = std::frexp(std::exp(r), &ex);
    const M hi = (M)vm;
    const M lo = (M)(vm - (double)hi);
    return {hi, lo, (int32_t)k + ex, 0};
}
}  // namespace

// Discount tables for scans of lane width V: g(k) = lambda^{k (l - k)},
// ln g(k) = -k (l - k) h / eps, for k = 0..l-1 (k summed marginals placed).
template <typename M>
void fill_disc(Disc<M> &d, int l, double hoe, int V)
{
    std::memset(&d, 0, sizeof d);
    d.V = V;
    for (int k = 0; k < MAXL; ++k) {
        const double lg = (k < l) ? -(double)(k * (l - k)) * hoe : 0.0;
        d.g1[k] = host_xg<M>(lg);
        for (int s = 0; s < 6; ++s) d.gstep[k][s] = host_xg<M>(lg * (double)(V << s));
        for (int t = 0; t < MAXV; ++t) d.gfix[k][t] = host_xg<M>(lg * (double)(t + 1));
        d.lgV[k] = lg * (double)V;
    }
    for (int k = 0; k <= MAXL; ++k) d.ck[k] = (k <= l) ? (double)(k * (l - k)) : 0.0;
}

Inst make_inst(int l, int64_t N, double h, double eps)
{
    Inst I;
    std::memset(&I, 0, sizeof I);
    I.N = N;
    I.l = l;
    I.h = h;
    I.hoe = h / eps;
    I.ieps = 1.0 / eps;
    I.x = nullptr;
    fill_disc<float>(I.d32, l, I.hoe, vsel(l, 0));
    fill_disc<double>(I.d64, l, I.hoe, vsel(l, 1));
    fill_disc<double>(I.dob, l, I.hoe, vsel(l, 2));
    fill_disc<double>(I.dck, l, I.hoe, vsel(l, 3));
    return I;
}

// Checkpoint bytes for one instance: the largest over the passes it runs.
int64_t tile_min_n(int l)
{
    // below this length a sweep on one team (l >= 7) or one wavefront (l <= 6)
    // is about as fast as the tiled launches and cheaper in total work
    return l >= WIDE_MINL ? 4096 : 16384;
}

size_t scratch_bytes(int l, int64_t N, int precision, int flags)
{
    // room for the untiled passes and, from N = TILE_SMALL_N up, for every tiled layout the batch
    // host or the autotuner may pick
    int nt = 0, B = 0;
    size_t b = pass_scratch_bytes(l, N, precision);
    if (tile_shape(l, N, flags | F_TILE_SMALL, &nt, &B)) b = std::max(b, tile_scratch_bytes(l, N, nt, B));
    return b;
}

size_t pass_scratch_bytes(int l, int64_t N, int precision)
{
    if (l >= WIDE_MINL) return ((size_t)wide_scratch_bytes(l, (long)N) + 255) & ~(size_t)255;
    const int D1 = (1 << (l - 1)) - 1;
    size_t best = 0;
    const int kinds[3] = {precision == MMOT_FP32 ? 0 : 1, 2, 3};
    for (int kind : kinds) {
        const int64_t CH = (int64_t)WAVE * vsel(l, kind);
        const int64_t C = (N + CH - 1) / CH;
        best = std::max(best, (size_t)C * (size_t)D1 * (size_t)elem_bytes(kind));
    }
    return (best + 255) & ~(size_t)255;
}

int scan_precision(const Inst &I, int precision, bool team_layout)
{
    if (precision != MMOT_FP32) return MMOT_FP64;
    // the slowest-decaying state takes g = lambda^(l-1) per position; a scan then
    // sums about 1 / (1 - g) positions of comparable terms, and FP32 rounding of
    // that many steps stays below ~1e-7 relative only for short windows
    const double window = 1.0 / -std::expm1(-(double)(I.l - 1) * I.hoe);
    return window <= (team_layout ? FP32_MAX_WINDOW_TEAM : FP32_MAX_WINDOW) ? MMOT_FP32 : MMOT_FP64;
}

bool fast_eligible(const Inst &I, int precision)
{
    if (!FAST_PATH_ENABLED) return false;
    const int l = I.l;
    if (l < 2 || l > FAST_MAXL) return false;
    if (I.N > std::min(fast_capacity(l, precision), fast_capacity(l, 0))) return false;
    int dec = 0;
    for (int k = 0; k < l; ++k) dec = std::max(dec, 1 - host_xg<double>(-(double)(k * (l - k)) * I.hoe).e);
    return bf_fits_range(precision, l, fast_v(l, precision), 0, dec) && bf_fits_range(0, l, fast_v(l, 0), 0, dec);
}

int fast_waves(int l, int64_t N, int kind, int precision)
{
    const int p = kind == 1 ? 0 : precision;
    const int64_t per = (int64_t)WAVE * fast_v(l, p);
    return (int)std::max<int64_t>(1, (N + per - 1) / per);
}

namespace {

size_t tr256(size_t n) { return (n + 255) & ~(size_t)255; }

int pow2_ceil(double x)
{
    int p = 1;
    while ((double)p < x && p < (1 << 30)) p <<= 1;
    return p;
}

struct Carve {
    size_t agg, carry, ck_stride, ck, part, total;
};

Carve carve(int l, int ntile, int B)
{
    const size_t D = (size_t)wide_states(l);
    Carve c;
    c.agg = tr256((size_t)ntile * 2 * (size_t)l * D * 32);  // elements up to the objective's 32 B
    c.carry = tr256((size_t)ntile * 2 * D * 32);
    c.ck_stride = tr256((size_t)wide_scratch_bytes(l, B));
    c.ck = (size_t)ntile * c.ck_stride;
    c.part = tr256((size_t)l * (size_t)ntile * sizeof(double));
    c.total = c.agg + c.carry + c.ck + c.part;
    return c;
}

std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tune;  // (l, ceil(log2 N)) -> tile length picked by the autotuner

int size_class(int64_t N)
{
    int c = 0;
    while (((int64_t)1 << c) < N) ++c;
    return c;
}

int rule_length(int64_t N, bool force)
{
    const int b = force ? pow2_ceil(std::sqrt((double)N)) : pow2_ceil(std::sqrt(8.0 * (double)N));
    return std::max(force ? 8 : 64, std::min(b, 4096));
}

}  // namespace

bool tile_shape(int l, int64_t N, int flags, int *ntile, int *B)
{
    const bool force = (flags & F_TILES) != 0;
    if (!force && N < ((flags & F_TILE_SMALL) ? (int64_t)TILE_SMALL_N : tile_min_n(l))) return false;
    int b = rule_length(N, force);
    if (!force) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find({l, size_class(N)});
        if (it != g_tune.end()) b = it->second;
    }
    *B = b;
    *ntile = (int)((N + b - 1) / b);
    return true;
}

int tile_candidates(int l, int64_t N, int flags, int *cand)
{
    const bool force = (flags & F_TILES) != 0;
    if (!force && N < ((flags & F_TILE_SMALL) ? (int64_t)TILE_SMALL_N : tile_min_n(l))) return 0;
    const int b = rule_length(N, force);
    if (force) {
        cand[0] = b;
        return 1;
    }
    int k = 0;
    for (int c : {b / 8, b / 4, b / 2, b, 2 * b})
        if (c >= 64 && c <= 8192) cand[k++] = c;
    return k;
}

bool tile_tuned(int l, int64_t N)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune.count({l, size_class(N)}) != 0;
}

void tile_set_tuned(int l, int64_t N, int B)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{l, size_class(N)}] = B;
}

size_t tile_scratch_bytes(int l, int64_t N, int ntile, int B)
{
    // room for every length the autotuner may pick for this N
    (void)ntile;
    (void)B;
    int cand[5];
    const int k = tile_candidates(l, N, F_TILE_SMALL, cand);
    size_t best = 0;
    for (int i = 0; i < k; ++i) best = std::max(best, carve(l, (int)((N + cand[i] - 1) / cand[i]), cand[i]).total);
    const int b = rule_length(N, true);
    best = std::max(best, carve(l, (int)((N + b - 1) / b), b).total);
    return best;
}

TileInst tile_inst(int l, int ntile, int B, char *scratch)
{
    const Carve c = carve(l, ntile, B);
    TileInst T;
    std::memset(&T, 0, sizeof T);
    T.ntile = ntile;
    T.B = B;
    T.agg = scratch;
    T.carry = scratch + c.agg;
    T.ck = scratch + c.agg + c.carry;
    T.part = reinterpret_cast<double *>(scratch + c.agg + c.carry + c.ck);
    T.ck_stride = (long)c.ck_stride;
    return T;
}

}  // namespace rt
}  // namespace mmot
