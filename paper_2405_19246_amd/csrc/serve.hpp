// Internal interface between the batch launcher and the serving loop.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "common.hpp"
#include "mmot.h"
#include "tables.hpp"

namespace mmot {

// Device buffers of batch_launch, each for up to `capacity` instances
// (dorder: 2 * capacity).
struct BatchBuffers {
    Inst *dI;
    Ptrs *dP;
    int *dorder;
    Result *dR;
    int *dticket;
    Track *dT;
};

// Allocates / frees a BatchBuffers set (hipMalloc; returns the HIP error).
hipError_t batch_buffers_alloc(BatchBuffers *bb, size_t capacity);
void batch_buffers_free(BatchBuffers *bb);

namespace rt {
extern thread_local std::string g_err;
int fail(int code, const std::string &msg);
int check_shape(int l, int64_t N, double h, double eps);
int check_opts(const mmot_opts *o);
}  // namespace rt

// Solves `count` instances: those the register-resident path takes run in
// rounds of its sweep and check kernels, the rest in one persistent launch of
// the extended-range solver; copies results to hR and synchronises the stream.
// timed: record the device time of the whole batch for mmot_last_batch_kernel_ms.
// Returns an MMOT_* code.
int batch_launch(const Inst *hI, const Ptrs *hP, int count, int precision, const RunOpts &o, hipStream_t s,
                 Result *hR, BatchBuffers *bb, bool timed = false);

}  // namespace mmot
