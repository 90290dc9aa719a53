// Calibration micro-benchmarks (ilu_calibrate): the floors the hot path is
// measured against -- achievable HBM stream bandwidth, the latency of one
// published-value hop between two workgroups (the unit of every dependency wait
// in the sync-free kernels), and the cost of a kernel launch (the unit of the
// level-launch scheme).  Every spin is bounded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "handle.h"
#include "javelin.h"

namespace {

constexpr int kCalBlock = 256;

__device__ __forceinline__ unsigned cal_xcc() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xf;
}

__global__ __launch_bounds__(kCalBlock) void k_cal_read(const double4 *__restrict__ a, size_t n4, double *out) {
    double s = 0;
    const size_t stride = (size_t)gridDim.x * kCalBlock;
    for (size_t i = (size_t)blockIdx.x * kCalBlock + threadIdx.x; i < n4; i += stride) {
        const double4 v = a[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == -1.0) out[0] = s;   // keeps the loads; the buffer holds zeros
}

__global__ __launch_bounds__(kCalBlock) void k_cal_copy(const double4 *__restrict__ a, double4 *__restrict__ b,
                                                        size_t n4) {
    const size_t stride = (size_t)gridDim.x * kCalBlock;
    for (size_t i = (size_t)blockIdx.x * kCalBlock + threadIdx.x; i < n4; i += stride) b[i] = a[i];
}

__global__ void k_cal_empty() {}

// Blocks a and b bounce a counter `iters` times with agent-scope relaxed atomics;
// the elapsed realtime ticks of block a land in out[0], the XCC ids in xcc[0..1].
__global__ void k_cal_pingpong(int *flag, int *abort_flag, int a, int b, int iters, unsigned long long *out,
                               unsigned *xcc) {
    if (threadIdx.x != 0) return;
    const int me = blockIdx.x;
    if (me != a && me != b) return;
    xcc[me == a ? 0 : 1] = cal_xcc();
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (int i = 0; i < iters; ++i) {
        const int want = me == a ? 2 * i + 2 : 2 * i + 1;
        if (me == a) __hip_atomic_store(flag, 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        long long s = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
            if (++s > (1ll << 24) ||
                __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        }
        if (me == b) __hip_atomic_store(flag, 2 * i + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (me == a) out[0] = __builtin_amdgcn_s_memrealtime() - t0;
}

}  // namespace

extern "C" ilu_status ilu_calibrate(int64_t bytes, double *results, int32_t cap) {
    using jv::fail;
    using jv::hip_fail;
    if (!results || cap < 1) return fail(ILU_ERR_ARG, "ilu_calibrate: results");
    if (bytes <= 0) bytes = (int64_t)2 << 30;
    bytes = std::max<int64_t>(bytes & ~(int64_t)255, 1 << 20);
    std::vector<double> r(5, 0.0);
    void *A = nullptr, *B = nullptr, *small = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&A, (size_t)bytes);
    if (e == hipSuccess) e = hipMalloc(&B, (size_t)bytes);
    if (e == hipSuccess) e = hipMalloc(&small, 4096);
    if (e == hipSuccess) e = hipMemset(A, 0, (size_t)bytes);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const size_t n4 = (size_t)bytes / sizeof(double4);
    auto best_ms = [&](auto &&launch, float *out_ms) -> hipError_t {
        float best = 1e30f;
        for (int rep = 0; rep < 5; ++rep) {
            hipError_t x = hipEventRecord(e0, 0);
            if (x != hipSuccess) return x;
            launch();
            if ((x = hipGetLastError()) != hipSuccess) return x;
            if ((x = hipEventRecord(e1, 0)) != hipSuccess) return x;
            if ((x = hipEventSynchronize(e1)) != hipSuccess) return x;
            float ms = 0.f;
            if ((x = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return x;
            best = std::min(best, ms);
        }
        *out_ms = best;
        return hipSuccess;
    };
    float ms = 0.f;
    if (e == hipSuccess) {
        e = best_ms([&]() { hipLaunchKernelGGL(k_cal_read, dim3(16384), dim3(kCalBlock), 0, 0, (const double4 *)A, n4,
                                               (double *)small); }, &ms);
        r[0] = (double)bytes / (ms * 1e-3) / 1e9;
    }
    if (e == hipSuccess) {
        e = best_ms([&]() { hipLaunchKernelGGL(k_cal_copy, dim3(16384), dim3(kCalBlock), 0, 0, (const double4 *)A,
                                               (double4 *)B, n4 / 2); }, &ms);
        r[1] = 2.0 * (double)(n4 / 2) * sizeof(double4) / (ms * 1e-3) / 1e9;
    }
    // flag hop: blocks 0 and 8 (one XCD under round-robin dispatch) and 0 and 1
    int *flag = (int *)small, *abortf = flag + 64;
    unsigned long long *ticks = (unsigned long long *)(flag + 128);
    unsigned *xcc = (unsigned *)(flag + 256);
    const int iters = 2000;
    const int pairs[2][2] = {{0, 8}, {0, 1}};
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        if ((e = hipMemset(small, 0, 4096)) != hipSuccess) break;
        hipLaunchKernelGGL(k_cal_pingpong, dim3(16), dim3(64), 0, 0, flag, abortf, pairs[k][0], pairs[k][1], iters, ticks,
                           xcc);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = hipDeviceSynchronize()) != hipSuccess) break;
        unsigned long long t = 0;
        int ab = 0;
        if ((e = hipMemcpy(&t, ticks, 8, hipMemcpyDeviceToHost)) != hipSuccess) break;
        if ((e = hipMemcpy(&ab, abortf, 4, hipMemcpyDeviceToHost)) != hipSuccess) break;
        // realtime counter at 100 MHz: 10 ns per tick; one hop is half a round trip
        r[2 + k] = ab ? -1.0 : (double)t * 10.0 / iters / 2.0;
    }
    if (e == hipSuccess) {
        const int nl = 1000;
        e = best_ms([&]() {
            for (int i = 0; i < nl; ++i) hipLaunchKernelGGL(k_cal_empty, dim3(1), dim3(64), 0, 0);
        }, &ms);
        r[4] = 1e3 * ms / nl;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    if (small) (void)hipFree(small);
    if (e != hipSuccess) return hip_fail(e, "ilu_calibrate");
    for (int i = 0; i < cap && i < 5; ++i) results[i] = r[i];
    return ILU_OK;
}
