// Internal interface between the batch launcher and the serving loop.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "common.hpp"
#include "mmot.h"
#include "tables.hpp"

namespace mmot {

struct BatchBuffers {
    Inst *dI;
    Ptrs *dP;
    int *dorder;
    Result *dR;
    int *dticket;
};

namespace rt {
extern thread_local std::string g_err;
int fail(int code, const std::string &msg);
int check_shape(int l, int64_t N, double h, double eps);
int check_opts(const mmot_opts *o);
}  // namespace rt

// One persistent launch over `count` instances; copies results to hR and
// synchronises the stream.  Returns an MMOT_* code.
int batch_launch(const Inst *hI, const Ptrs *hP, int count, int precision, const RunOpts &o, hipStream_t s,
                 Result *hR, BatchBuffers *bb);

}  // namespace mmot
