// Host-side tables of libmmot (see tables.cpp).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"
#include "mmot.h"

namespace mmot {
namespace rt {

// Descriptor of one problem: shape and the discount tables of every pass kind.
Inst make_inst(int l, int64_t N, double h, double eps);

// Scratch bytes one instance needs in the given precision (checkpoints of the
// one-wavefront and one-team solvers, or every buffer of a tiled solve).
// flags: F_TILES forces tiles.
size_t scratch_bytes(int l, int64_t N, int precision, int flags);

// Checkpoint bytes of one untiled product / check / objective pass.
size_t pass_scratch_bytes(int l, int64_t N, int precision);

// Shortest N that is tiled without F_TILES.
int64_t tile_min_n(int l);

// Whether an instance is tiled, and its tile count and tile length B (positions).
bool tile_shape(int l, int64_t N, int flags, int *ntile, int *B);

// Autotuner of the tile length: candidate lengths for an instance (0 if it is
// not tiled), whether its (l, ceil(log2 N)) class has been measured, and the
// measured choice (process-wide cache, read by tile_shape).
int tile_candidates(int l, int64_t N, int flags, int *cand);
bool tile_tuned(int l, int64_t N);
void tile_set_tuned(int l, int64_t N, int B);

// Scratch bytes of a tiled solve (room for every candidate length) and its
// layout inside a scratch block.
size_t tile_scratch_bytes(int l, int64_t N, int ntile, int B);
TileInst tile_inst(int l, int ntile, int B, char *scratch);

// Mantissa precision of the scans of an instance solved in `precision`: FP32
// mode keeps FP32 mantissas on the one-wavefront solver (block floating point)
// where the scan window 1 / (1 - lambda^(l-1)) is at most FP32_MAX_WINDOW
// positions, and FP64 mantissas beyond.  The team and tiled layouts take FP64
// mantissas in FP32 mode (FP32_MAX_WINDOW_TEAM = 0): their FP32 iterations
// settled about 1e-6 relative away from the FP64 fixed point (l = 5, N = 1000,
// eps = 0.02, window 5.5: Res never below 1e-6).  On this GPU without packed
// FP32 both run at the same VALU rate; only registers and memory double.
constexpr double FP32_MAX_WINDOW = 64.0;
constexpr double FP32_MAX_WINDOW_TEAM = 0.0;
int scan_precision(const Inst &I, int precision, bool team_layout);

// Whether the register-resident path (fast.hpp) takes an instance: its N fits
// one workgroup of the sweep and of the FP64 check kernel, and the discount
// decay over a thread's positions leaves room for block floating point.
bool fast_eligible(const Inst &I, int precision);

// Wavefronts per workgroup for an instance of length N: kind 0 sweeps in the
// given precision, kind 1 FP64 checks.
int fast_waves(int l, int64_t N, int kind, int precision);

}  // namespace rt
}  // namespace mmot
