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

}  // namespace rt
}  // namespace mmot
