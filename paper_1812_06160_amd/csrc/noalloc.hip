// ilu_apply_noalloc: the apply with its published intermediates (the forward
// result y and the backward result z, [n][nrhs] each) in a static device array
// instead of handle buffers that ilu_apply allocates on first use.  For callers
// that cannot allocate device memory during the call (graph capture, serving
// loops).  Everything else the apply touches -- factor, tiles, claim counters,
// status word -- was allocated by ilu_analyze / ilu_factor.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "handle.h"
#include "javelin.h"

using namespace jv;

namespace {

// y and z of one call: 2 * n * nrhs elements of the accumulate type (8 bytes
// for FP64 factors, 4 for FP32/BF16).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` on each device

// The device address of this device's copy of `scratch` (looked up once per
// device, with that device current).
hipError_t scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" ilu_status ilu_apply_noalloc(ilu_handle h, const void *b, void *x, int32_t nrhs, int64_t ld,
                                        int32_t fac_prec, int32_t vec_prec, int32_t flags, hipStream_t s) {
    if (!h) return fail(ILU_ERR_STATE, "ilu_apply_noalloc: NULL handle");
    if (h->host_only) return fail(ILU_ERR_STATE, "ilu_apply_noalloc: host-only analysis");
    if (!h->factored) return fail(ILU_ERR_STATE, "ilu_apply_noalloc: no factor");
    if (!b || !x || nrhs < 1 || ld < nrhs) return fail(ILU_ERR_ARG, "ilu_apply_noalloc: bad vectors or sizes");
    if (vec_prec != ILU_PREC_F64 && vec_prec != ILU_PREC_F32) return fail(ILU_ERR_ARG, "ilu_apply_noalloc: vec_prec");
    if (flags & ~ILU_PERMUTED_SPACE) return fail(ILU_ERR_ARG, "ilu_apply_noalloc: unknown flags");
    const void *val;
    switch (fac_prec) {
        case ILU_PREC_F64: val = h->d_lu; break;
        case ILU_PREC_F32:
            if (!h->has32) return fail(ILU_ERR_STATE, "ilu_apply_noalloc: factor has no FP32 copy");
            val = h->d_lu32;
            break;
        case ILU_PREC_BF16:
            if (!h->has16) return fail(ILU_ERR_STATE, "ilu_apply_noalloc: factor has no BF16 copy");
            val = h->d_lu16;
            break;
        default: return fail(ILU_ERR_ARG, "ilu_apply_noalloc: fac_prec");
    }
    const size_t elt = fac_prec == ILU_PREC_F64 ? 8 : 4;
    const size_t count = (size_t)h->H.n * (size_t)nrhs;
    if (count > kScratchBytes / (2 * elt))
        return fail(ILU_ERR_ARG, "ilu_apply_noalloc: n * nrhs = " + std::to_string(count) + " exceeds the " +
                                     std::to_string(kScratchBytes / (2 * elt)) +
                                     " elements of the static workspace (64 MiB for y and z)");
    void *base = nullptr;
    hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess) return hip_fail(e, "ilu_apply_noalloc: workspace address");
    SolveWork ws{base, static_cast<unsigned char *>(base) + count * elt, nrhs, true};
    return run_solves(h, 0, val, fac_prec, vec_prec == ILU_PREC_F64 ? 0 : 1, b, x, nullptr, nullptr, nrhs, ld, flags,
                      s, &ws);
}
