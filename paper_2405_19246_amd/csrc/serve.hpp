// Internal interface between the batch launcher and the serving loop.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
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
    TileInst *dTI;    // tiled solves: per-instance buffers
    TileTrack *dTT;   // tiled solves: per-instance state
    char *djobs;      // tiled solves: job lists (grow-only)
    size_t jobs_cap;
    int *dflags;      // marginal checks: per-instance flags
};

// Job lists of the tiled launches of instances g (all with l marginals) in bb's
// job buffer; host keeps the uploaded bytes until the stream has copied them.
hipError_t upload_jobs(const std::vector<int> &g, const std::vector<TileInst> &hTI, int l, BatchBuffers *bb,
                       hipStream_t s, std::vector<char> &host, TileJobs *J);

// Grows bb's job-list buffer to at least jobs_bytes.
hipError_t tile_buffers_reserve(BatchBuffers *bb, size_t jobs_bytes);

// Tiled solves of the instances g (all with l marginals) of a batch of count:
// sweeps in blocks of launches until each stops, then the FP64 objective; fills
// hR[i] for i in g.  dI/dP of bb hold the batch's descriptors already.  The
// tiled launches start after `start` (an event recorded on s) if given, else
// after everything enqueued on s so far; later work on s waits for them.
int tiled_group_solve(int l, const std::vector<int> &g, int count, const Inst *hI, const Ptrs *hP, int precision,
                      const RunOpts &o, int flags, hipStream_t s, BatchBuffers *bb, Result *hR,
                      hipEvent_t start = nullptr);

// Allocates / frees a BatchBuffers set (hipMalloc; returns the HIP error).
hipError_t batch_buffers_alloc(BatchBuffers *bb, size_t capacity);
void batch_buffers_free(BatchBuffers *bb);

namespace rt {
extern thread_local std::string g_err;
int fail(int code, const std::string &msg);
// Maps the exception being handled to an MMOT_* code (inside a catch block).
int guard_fail();
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
