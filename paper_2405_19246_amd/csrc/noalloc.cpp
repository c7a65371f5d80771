// mmot_marginal_product_noalloc: the product of mmot_marginal_product without a
// plan and without any allocation.  Its workspace -- the problem descriptor
// followed by the scan checkpoints -- lives in the file-scope device array
// `scratch` below, one copy per GPU, held until the process ends.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "launch.hpp"
#include "mmot.h"
#include "serve.hpp"
#include "tables.hpp"

using namespace mmot;
using namespace mmot::rt;

namespace {

static __device__ __align__(256) char scratch[MMOT_NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};    // device address of `scratch` on each GPU (its name is a host stand-in)
Inst g_inst[MAX_DEVICES];         // host copy of the descriptor last sent to each GPU

size_t desc_bytes() { return (sizeof(Inst) + 255) & ~(size_t)255; }

// Address of this GPU's copy of `scratch`, looked up once per device with the
// device current.
int workspace(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MMOT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = reinterpret_cast<char *>(g_ptr[dev]);
    return MMOT_OK;
}

}  // namespace

extern "C" int mmot_marginal_product_noalloc(const mmot_problem *p, int32_t j, const double *log_phi, double *log_J,
                                             void *hip_stream)
{
    try {
        if (!p || !log_phi || !log_J) return fail(MMOT_ERR_INVALID, "NULL argument");
        if (p->x) return fail(MMOT_ERR_UNSUPPORTED, "the workspace-free product takes uniform grids only");
        int rc = check_shape(p->l, p->N, p->h, p->eps);
        if (rc) return rc;
        if (p->precision != MMOT_FP64 && p->precision != MMOT_FP32)
            return fail(MMOT_ERR_INVALID, "precision must be MMOT_FP64 or MMOT_FP32");
        if (j < 0 || j >= p->l) return fail(MMOT_ERR_INVALID, "j out of range");
        const size_t need = desc_bytes() + pass_scratch_bytes(p->l, p->N, p->precision);
        if (need > (size_t)MMOT_NOALLOC_BYTES)
            return fail(MMOT_ERR_INVALID, "problem needs " + std::to_string(need) +
                                              " bytes of workspace, more than the fixed " +
                                              std::to_string((size_t)MMOT_NOALLOC_BYTES));
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
            return fail(MMOT_ERR_HIP, "no current HIP device");
        char *base = nullptr;
        rc = workspace(dev, &base);
        if (rc) return rc;
        const hipStream_t s = (hipStream_t)hip_stream;
        g_inst[dev] = make_inst(p->l, p->N, p->h, p->eps);
        hipError_t e = hipMemcpyAsync(base, &g_inst[dev], sizeof(Inst), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail(MMOT_ERR_HIP, std::string("descriptor copy: ") + hipGetErrorString(e));
        const Ptrs P = {nullptr, const_cast<double *>(log_phi), log_J, base + desc_bytes(), 0, 0, 0, 0};
        e = launch_pass(p->l, p->precision, P_PRODUCT, reinterpret_cast<const Inst *>(base), P, j, nullptr, s);
        if (e != hipSuccess) return fail(MMOT_ERR_HIP, std::string("product launch: ") + hipGetErrorString(e));
        return MMOT_OK;
    } catch (...) {
        return fail(MMOT_ERR_HIP, "unexpected exception");
    }
}
