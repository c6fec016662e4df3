// hisq_dslash_multi_rhs for callers that cannot allocate device memory.
//
// The only device memory the epilogue form needs beyond the caller's buffers
// is the per-RHS coefficient array.  Here it lives in a fixed array of the
// library's code object, one copy per GPU, so a call allocates nothing.  Host
// code never uses the array's name as an address (in host code it is only a
// stand-in symbol): the address of each device's copy is looked up once, with
// that device current, on the entry point's first call there.

#include <mutex>

#include "solver_internal.h"

namespace hisq {

static __device__ __align__(256) double scratch[HISQ_NOALLOC_MAX_RHS];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current.
static int scratch_for(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("hisq_dslash_multi_rhs_noalloc: device index out of range");
        return HISQ_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return HISQ_ERR_HIP;
        }
        g_scratch_dev[device] = (double *)ptr;
    }
    *out = g_scratch_dev[device];
    return HISQ_OK;
}

}  // namespace hisq

using namespace hisq;

extern "C" int hisq_dslash_multi_rhs_noalloc(hisq_gauge_t g, int out_parity, int prec, int nrhs, const void *in,
                                             void *out, const double *diag, const void *y, void *stream) {
    int rc = check_multi_rhs(g, out_parity, prec, nrhs, in, out, diag, y);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!diag) return gauge_dslash(g, out_parity, prec, prec, prec, nrhs, in, out, nullptr, nullptr, nullptr, nullptr, s);
    if (nrhs > HISQ_NOALLOC_MAX_RHS) {
        set_error("hisq_dslash_multi_rhs_noalloc: with diag, nrhs must not exceed HISQ_NOALLOC_MAX_RHS (" +
                  std::to_string(HISQ_NOALLOC_MAX_RHS) + ")");
        return HISQ_ERR_INVALID;
    }
    int dev = -1;
    HISQ_HIP_CHECK(hipGetDevice(&dev));
    if (dev != g->device) {
        set_error("hisq_dslash_multi_rhs_noalloc: the handle's device must be current");
        return HISQ_ERR_INVALID;
    }
    double *coef = nullptr;
    if ((rc = scratch_for(dev, &coef))) return rc;
    // stream-ordered: the kernel below reads what this copy writes
    HISQ_HIP_CHECK(hipMemcpyAsync(coef, diag, sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
    return gauge_dslash(g, out_parity, prec, prec, prec, nrhs, in, out, y, coef, nullptr, nullptr, s);
}
