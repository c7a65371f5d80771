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

// Checkpoint bytes one instance needs in the given precision.
size_t scratch_bytes(int l, int64_t N, int precision);

// Whether the register-resident path (fast.hpp) takes an instance: its N fits
// one workgroup of the sweep and of the FP64 check kernel, and the discount
// decay over a thread's positions leaves room for block floating point.
bool fast_eligible(const Inst &I, int precision);

// Wavefronts per workgroup for an instance of length N: kind 0 sweeps in the
// given precision, kind 1 FP64 checks.
int fast_waves(int l, int64_t N, int kind, int precision);

}  // namespace rt
}  // namespace mmot
