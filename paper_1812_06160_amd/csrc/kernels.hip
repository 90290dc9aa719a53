// HIP kernels for gfx950: up-looking ILU factor, triangular solves, spmv, casts.
//
// Every kernel works on groups of G lanes (G in {4, 8, 16, 32, 64}) inside a
// 64-wide wavefront; a group owns one row.  Two launch schemes share the same
// per-row code:
//
//  * level launch: one kernel per level (the kernel boundary is the barrier
//    between levels, the classic level-set scheme the paper compares against,
//    Sec. VI "CSR-LS");
//  * sync-free launch: one kernel for all levels.  Each wave runs one
//    level-homogeneous task (up to 64/G consecutive rows of one level); blocks
//    take their tasks in start order from per-XCD task streams (claim_task).  A
//    row reads each value it depends on with an agent-scope atomic load until it
//    is no longer the "pending" bit pattern.  This is the GPU form of the paper's
//    point-to-point synchronisation (Sec. III, "Level Scheduling, Upper Stage"): a
//    row waits only for the rows it needs, never for a whole level.  Values are
//    published with agent-scope relaxed atomic stores, so no cache-flushing
//    release fence is needed (coherence of atomics to one address is enough:
//    each consumed value is its own flag).
//
// Deadlock freedom of the sync-free scheme: a task only waits on rows of earlier
// levels, i.e. on tasks of earlier-claimed block slots, whose blocks already run
// or have finished; blocks claim slots when they start, so the smallest
// unfinished task is always held by a running wave or claimed by the next block
// that starts on its XCD, whatever the number of resident blocks.  Every wait
// is bounded in time (kWaitTicks) and raises a device abort flag that stops all waits.
//
// Floating point: the library is compiled with -ffp-contract=off, so a - l*u is
// a rounded multiply then a rounded subtract, and FP64 division is IEEE
// correctly rounded; with the columns of a row taken in ascending order the
// factor reproduces a serial up-looking ILU bit for bit.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <climits>
#include <cstdint>

#include "device.h"

namespace jv {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint64_t ld_acq_u64(const uint64_t *p) {
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_acq_u32(const uint32_t *p) {
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_pub_u64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_pub_u32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int aborted(int32_t *info) {
    return __hip_atomic_load(&info[kInfoAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wall-clock bound of one wait: kWaitTicks of the 100 MHz realtime counter; the
// first call starts the clock.
__device__ __forceinline__ bool expired(uint64_t &t0) {
    const uint64_t now = __builtin_amdgcn_s_memrealtime();
    if (t0 == 0) {
        t0 = now;
        return false;
    }
    return now - t0 > kWaitTicks;
}

// Bounded wait until *p differs from the pending pattern.  On expiry (or when
// another wave has expired) returns a quiet NaN; the host reports ILU_ERR_TIMEOUT.
__device__ uint64_t wait_u64(const uint64_t *p, int32_t *info, int sleep) {
    uint64_t v = ld_acq_u64(p);
    if (v != kPending64) return v;
    int spins = 0;
    uint64_t t0 = 0;
    for (;;) {
        for (int k = 0; k < sleep; ++k) __builtin_amdgcn_s_sleep(1);
        v = ld_acq_u64(p);
        if (v != kPending64) return v;
        if ((++spins & 63) == 0) {
            if (aborted(info)) return kQNaN64;
            if (expired(t0)) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return kQNaN64;
            }
        }
    }
}

__device__ uint32_t wait_u32(const uint32_t *p, int32_t *info, int sleep) {
    uint32_t v = ld_acq_u32(p);
    if (v != kPending32) return v;
    int spins = 0;
    uint64_t t0 = 0;
    for (;;) {
        for (int k = 0; k < sleep; ++k) __builtin_amdgcn_s_sleep(1);
        v = ld_acq_u32(p);
        if (v != kPending32) return v;
        if ((++spins & 63) == 0) {
            if (aborted(info)) return kQNaN32;
            if (expired(t0)) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return kQNaN32;
            }
        }
    }
}

template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int gi) {
    if constexpr (G == 64) return ballot;
    else return (ballot >> (gi * G)) & ((1ull << G) - 1ull);
}

// Cross-lane moves inside rows of 16 lanes (DPP): quad permutations and mirrors
// execute in the vector pipeline, where a general shuffle would be an LDS-unit
// permute with LDS latency.
enum : int {
    kDppQuadXor1 = 0xB1,     // quad_perm [1, 0, 3, 2]
    kDppQuadXor2 = 0x4E,     // quad_perm [2, 3, 0, 1]
    kDppHalfMirror = 0x141,  // lane i <- lane 7 - i within each 8 lanes
    kDppMirror = 0x140       // lane i <- lane 15 - i within each 16 lanes
};
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the G lanes of an aligned lane group, returned in every lane of the
// group.  Lanes pair in the same order at every width, and each pairwise sum is
// commutative, so all lanes of a group hold identical bits.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
    if constexpr (G >= 2) {
        if constexpr (G >= 4) v += dpp_mov<kDppQuadXor2>(v);
        v += dpp_mov<kDppQuadXor1>(v);
    }
    if constexpr (G >= 8) v += dpp_mov<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += dpp_mov<kDppMirror>(v);
#pragma unroll
    for (int off = 16; off < G; off <<= 1) v += __shfl_xor(v, off, G);
    return v;
}

// ---------------------------------------------------------------------------------
// Typed access to published intermediates
// ---------------------------------------------------------------------------------
template <typename TA> struct Pub;
template <> struct Pub<double> {
    using U = uint64_t;
    static constexpr uint64_t kPend = kPending64;
    __device__ static U load(const double *p) { return ld_acq_u64(reinterpret_cast<const uint64_t *>(p)); }
    __device__ static double from(U b) { return __longlong_as_double((long long)b); }
    __device__ static double wait(const double *p, int32_t *info, int sleep) {
        return __longlong_as_double((long long)wait_u64(reinterpret_cast<const uint64_t *>(p), info, sleep));
    }
    __device__ static void publish(double *p, double v) {
        uint64_t b = (uint64_t)__double_as_longlong(v);
        if (v != v) b = kQNaN64;
        st_pub_u64(reinterpret_cast<uint64_t *>(p), b);
    }
    __device__ static double pending() { return __longlong_as_double((long long)kPending64); }
};
template <> struct Pub<float> {
    using U = uint32_t;
    static constexpr uint32_t kPend = kPending32;
    __device__ static U load(const float *p) { return ld_acq_u32(reinterpret_cast<const uint32_t *>(p)); }
    __device__ static float from(U b) { return __uint_as_float(b); }
    __device__ static float wait(const float *p, int32_t *info, int sleep) {
        return __uint_as_float(wait_u32(reinterpret_cast<const uint32_t *>(p), info, sleep));
    }
    __device__ static void publish(float *p, float v) {
        uint32_t b = __float_as_uint(v);
        if (v != v) b = kQNaN32;
        st_pub_u32(reinterpret_cast<uint32_t *>(p), b);
    }
    __device__ static float pending() { return __uint_as_float(kPending32); }
};

__device__ __forceinline__ double load_val(const double *v, int64_t p) { return v[p]; }
__device__ __forceinline__ float load_val(const float *v, int64_t p) { return v[p]; }
__device__ __forceinline__ float load_val(const uint16_t *v, int64_t p) {
    return __uint_as_float(((uint32_t)v[p]) << 16);
}

// ---------------------------------------------------------------------------------
// Utility kernels
// ---------------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t *p, uint64_t value, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}
__global__ void k_zero_counters(int32_t *c) {
    if (threadIdx.x < kStreams) c[threadIdx.x * kCounterStride] = 0;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t value, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

// Re-arms the solve intermediates when the abort flag is up; the last block to
// finish clears the flag and counts the timeout.  Nothing else writes the flag
// while this kernel runs (stream order), so every block reads the same value and
// either all blocks take part or none does.
__global__ void k_solve_guard(int32_t *info, uint64_t *y64, uint64_t *z64, int64_t n64, uint32_t *y32,
                              uint32_t *z32, int64_t n32) {
    if (!aborted(info)) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n64; i += stride) {
        y64[i] = kPending64;
        z64[i] = kPending64;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n32; i += stride) {
        y32[i] = kPending32;
        z32[i] = kPending32;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&info[kInfoGuardDone], 1) == (int)gridDim.x - 1) {
            info[kInfoGuardDone] = 0;
            atomicAdd(&info[kInfoTimeouts], 1);
            __hip_atomic_store(&info[kInfoAbort], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void k_factor_prologue(int32_t *info, uint64_t *y64, uint64_t *z64, int64_t n64, uint32_t *y32,
                                  uint32_t *z32, int64_t n32, int32_t *counters) {
    if (blockIdx.x == 0) {
        if (counters && threadIdx.x < kStreams) counters[threadIdx.x * kCounterStride] = 0;
        if (threadIdx.x == 0) {
            info[kInfoBadKey] = INT_MAX;
            info[kInfoDropLo] = 0;
            info[kInfoDropLo + 1] = 0;
        }
    }
    if (!aborted(info)) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n64; i += stride) {
        y64[i] = kPending64;
        z64[i] = kPending64;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n32; i += stride) {
        y32[i] = kPending32;
        z32[i] = kPending32;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&info[kInfoGuardDone], 1) == (int)gridDim.x - 1) {
            info[kInfoGuardDone] = 0;
            atomicAdd(&info[kInfoTimeouts], 1);
            __hip_atomic_store(&info[kInfoAbort], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// one thread per range; ranges are a few entries long (the U part of one row)
__global__ void k_arm_ranges(uint64_t *lu, const int2 *__restrict__ ranges, int32_t count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int2 r = ranges[i];
    for (int j = 0; j < r.y; ++j) lu[r.x + j] = kPending64;
}

__global__ void k_raise_abort(int32_t *info) {
    if (threadIdx.x == 0) __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// tau_r = tau * ||A(perm[r], :)||_2, squares summed in the input order of the row
__global__ void k_row_tau(int32_t n, const int32_t *__restrict__ in_rp, const double *__restrict__ a,
                          const int32_t *__restrict__ perm, double tau, double *__restrict__ row_tau) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int i = perm[r];
    double s = 0.0;
    for (int p = in_rp[i]; p < in_rp[i + 1]; ++p) {
        double sq = a[p] * a[p];
        s = s + sq;
    }
    row_tau[r] = tau * sqrt(s);
}

__global__ void k_gather(int64_t m, const int32_t *__restrict__ src, const double *__restrict__ a,
                         double *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) {
        int s = src[i];
        out[i] = s >= 0 ? a[s] : 0.0;
    }
}

__global__ void k_cast_f32(int64_t m, const double *__restrict__ x, float *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) y[i] = (float)x[i];
}

// FP64 -> FP32 (round to nearest even), then FP32 -> BF16 keeping the upper half
// of the pattern with round-to-nearest-even on the dropped half; NaN stays NaN.
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t bias = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + bias) >> 16);
}
__global__ void k_cast_bf16(int64_t m, const double *__restrict__ x, uint16_t *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) y[i] = to_bf16((float)x[i]);
}

// After a factor with tau > 0 or k < k_max: dropped entries become 0.0 with state
// 1, absent entries state 2, kept entries state 0; counts the drops.
__global__ void k_factor_fixup(int64_t nnz, double *__restrict__ lu, const int8_t *__restrict__ flev, int32_t k,
                               int32_t use_flev, int8_t *__restrict__ stat, int32_t *info) {
    __shared__ unsigned long long cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    unsigned long long mine = 0;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < nnz; i += stride) {
        uint64_t b = (uint64_t)__double_as_longlong(lu[i]);
        int8_t st = 0;
        if (b == kDropped64) {
            lu[i] = 0.0;
            st = 1;
            ++mine;
        } else if (use_flev && flev[i] > k) {
            st = 2;
        }
        stat[i] = st;
    }
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0 && cnt)
        atomicAdd(reinterpret_cast<unsigned long long *>(&info[kInfoDropLo]), cnt);
}

// ---------------------------------------------------------------------------------
// Task claiming of the sync-free kernels
// ---------------------------------------------------------------------------------
__device__ __forceinline__ unsigned xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xf;   // HW_REG_XCC_ID[3:0]
}

// Claims the next block slot of this XCD's stream (start order) -- or, when that
// stream is exhausted, of the next stream that is not -- and runs task
// slot * waves_per_block + wave of that stream on each wave.  Block 0 also clears
// the counters of the pass that runs next.
template <typename F>
__device__ __forceinline__ void claim_task(const Claims &C, int nstreams, F &&task_fn) {
    __shared__ int s_slot, s_stream;
    if (C.zero_counters && blockIdx.x == 0 && threadIdx.x < kStreams)
        C.zero_counters[threadIdx.x * kCounterStride] = 0;
    if (threadIdx.x == 0) {
        const int x0 = C.xcc_stream[xcc_id()];
        s_stream = -1;
        for (int k = 0; k < nstreams; ++k) {
            const int x = (x0 + k) % nstreams;
            const int slots = (C.stream_ptr[x + 1] - C.stream_ptr[x] + kBlock / 64 - 1) / (kBlock / 64);
            const int v = __hip_atomic_fetch_add(C.counters + x * kCounterStride, 1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (v < slots) {
                s_slot = v;
                s_stream = x;
                break;
            }
        }
    }
    __syncthreads();
    const int x = s_stream;
    if (x < 0) return;
    const int lo = C.stream_ptr[x];
    const int len = C.stream_ptr[x + 1] - lo;
    const int i = s_slot * (kBlock / 64) + (int)(threadIdx.x >> 6);
    if (i < len) task_fn(C.stream_tasks[lo + i]);
}

__global__ void k_probe_xcc(int32_t *out) {
    if (threadIdx.x == 0) out[blockIdx.x] = (int32_t)xcc_id();
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------------
// Up-looking ILU on the fixed pattern (paper Sec. III, Fig. 1), one row per group
// ---------------------------------------------------------------------------------
// Lane t of the group holds entry rs+t of row r (the host guarantees row length <= G).
// For each earlier column c of the row, in ascending order: lane e divides its
// entry by the pivot u_cc, the multiplier is broadcast, and every lane whose
// column matches a later column j of row c subtracts l * u_cj.
//
// Staged form (STAGE): the upper parts (diagonal first) of all dependency rows c
// are gathered into the group's LDS slice in one parallel pass -- in the
// persistent kernel this is the single point where the row waits for its
// dependencies -- and the ascending elimination then reads them from LDS.
// Unstaged form: each dependency row is loaded when its turn comes.

template <int G, bool SF>
__device__ __forceinline__ void factor_finish(const FactorArgs &A, int r, int t, int gi, int p, bool act, int col,
                                              int absent, int dropped, double v, double tr, int diag_lane) {
    if (A.use_tau && act && !absent && col > r && fabs(v) < tr) dropped = 1;
    if (A.milu && A.use_tau) {
        // modified ILU: dropped U entries go back to the diagonal, ascending column
        for (int j = diag_lane + 1; j < G; ++j) {
            const double dv = __shfl(v, j, G);
            if (__shfl(dropped, j, G) && t == diag_lane) v = v + dv;
        }
    }
    const double pv = __shfl(v, diag_lane, G);
    const bool nonfinite = act && !absent && !dropped && !isfinite(v);
    const uint64_t nfm = group_bits<G>(__ballot(nonfinite), gi);
    if (t == 0) {
        if (pv == 0.0) atomicMin(&A.info[kInfoBadKey], 2 * r);
        else if (nfm) atomicMin(&A.info[kInfoBadKey], 2 * r + 1);
    }
    if (act) {
        uint64_t bits;
        if (absent) bits = 0;
        else if (dropped) bits = kDropped64;
        else bits = (v != v) ? kQNaN64 : (uint64_t)__double_as_longlong(v);
        if constexpr (SF) st_pub_u64(reinterpret_cast<uint64_t *>(&A.lu[p]), bits);
        else A.lu[p] = __longlong_as_double((long long)bits);
    }
}

template <int G, bool SF>
__device__ __forceinline__ void factor_row(const FactorArgs &A, int r, int t, int gi) {
    const int rs = A.rp[r], re = A.rp[r + 1], d = A.diag[r];
    const int nL = d - rs, dl = d - rs;
    const int p = rs + t;
    const bool act = p < re;
    const int col = act ? A.ci[p] : INT_MAX;
    const int absent = (act && A.use_flev && A.flev[p] > A.k) ? 1 : 0;
    const int s = act ? A.src[p] : -1;
    double v = (s >= 0 && !absent) ? A.a[s] : 0.0;
    int dropped = 0;
    const double tr = A.use_tau ? A.row_tau[r] : 0.0;
    int dcl = 0, ecl = 0;
    if (t < nL) {
        dcl = A.diag[col];
        ecl = A.rp[col + 1];
    }
    for (int e = 0; e < nL; ++e) {
        if (__shfl(absent, e, G)) continue;
        const int dc = __shfl(dcl, e, G);
        const int lenU = __shfl(ecl, e, G) - dc;
        const bool inU = t < lenU;
        int ucol = -1, uabs = 0;
        double uv = 0.0;
        if (inU) {
            const int q = dc + t;
            ucol = A.ci[q];
            uabs = (A.use_flev && A.flev[q] > A.k) ? 1 : 0;
            if constexpr (SF) uv = Pub<double>::wait(&A.lu[q], A.info, A.poll_sleep);
            else uv = A.lu[q];
        }
        const double piv = __shfl(uv, 0, G);
        double before = 0.0;
        if (t == e) {
            before = v;
            v = v / piv;
            if (A.use_tau && fabs(v) < tr) dropped = 1;
        }
        if (__shfl(dropped, e, G)) {
            if (A.milu) {
                // modified ILU: a dropped multiplier gives back its value before the division
                const double bv = __shfl(before, e, G);
                if (t == dl) v = v + bv;
            }
            continue;
        }
        const double l = __shfl(v, e, G);
        for (int j = 1; j < lenU; ++j) {
            const int uc = __shfl(ucol, j, G);
            const double uu = __shfl(uv, j, G);
            const int ua = __shfl(uabs, j, G);
            const bool kept = !ua && (uint64_t)__double_as_longlong(uu) != kDropped64;
            const bool mine = kept && col == uc && !absent;
            // modified ILU: an update whose target is not a kept entry of row r is
            // subtracted from the diagonal instead, in U(c)'s column order
            const bool taken = A.milu && group_bits<G>(__ballot(mine && t != dl), gi) != 0;
            if (A.milu && t == dl) {
                if (kept && !taken) {
                    const double lost = l * uu;
                    v = v - lost;
                }
            } else if (mine) {
                const double prod = l * uu;
                v = v - prod;
            }
        }
    }
    factor_finish<G, SF>(A, r, t, gi, p, act, col, absent, dropped, v, tr, d - rs);
}

// Staged row with the elimination split in three phases:
//  gather  all dependency rows' upper parts (diagonal first) into LDS, with the
//          loads of every lane issued together and re-polled together while pending;
//  match   (no chain) lane t looks up, for every dependency e, the upper entry of
//          row c_e in its own column and keeps it in a register (MAXL of them);
//  chain   for e ascending: lane e divides by its pivot, the multiplier is
//          broadcast, every lane with a match subtracts l * u -- the same
//          operations in the same order as the unstaged form.
template <int G, int MAXL, bool SF>
__device__ __forceinline__ void factor_row_staged(const FactorArgs &A, int r, int t, int gi, double *sv, int *sc,
                                                  int *soff, int *sdc) {
    constexpr int kTaken = -2;   // column slot of a U(c) entry that a lane of the row took
    const int rs = A.rp[r], re = A.rp[r + 1], d = A.diag[r];
    const int nL = d - rs, dl = d - rs;
    const int p = rs + t;
    const bool act = p < re;
    const int col = act ? A.ci[p] : INT_MAX;
    const int absent = (act && A.use_flev && A.flev[p] > A.k) ? 1 : 0;
    const int s = act ? A.src[p] : -1;
    double v = (s >= 0 && !absent) ? A.a[s] : 0.0;
    int dropped = 0;
    const double tr = A.use_tau ? A.row_tau[r] : 0.0;
    // length of U(c) (diagonal included) for each kept dependency; 0 when absent
    int dc = 0, len = 0;
    if (t < nL && !absent) {
        dc = A.diag[col];
        len = A.rp[col + 1] - dc;
    }
    int inc = len;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const int y = __shfl_up(inc, o, G);
        if (t >= o) inc += y;
    }
    const int total = __shfl(inc, G - 1, G);
    const int off = inc - len;
    if (t < nL) {
        soff[t] = off;
        sdc[t] = dc;
    }
    wave_sync_lds();
    // ---- gather: JM values per lane in one polling round, the rest one by one ----
    constexpr int JM = 4;
    uint64_t raw[JM];
    int qs[JM];
#pragma unroll
    for (int m = 0; m < JM; ++m) {
        const int j = t + m * G;
        qs[m] = -1;
        raw[m] = 0;
        if (j < total) {
            int e = 0;
            while (e + 1 < nL && soff[e + 1] <= j) ++e;
            const int q = sdc[e] + (j - soff[e]);
            qs[m] = q;
            sc[j] = (A.use_flev && A.flev[q] > A.k) ? -1 : A.ci[q];
            if constexpr (SF) raw[m] = ld_acq_u64(reinterpret_cast<const uint64_t *>(&A.lu[q]));
            else raw[m] = (uint64_t)__double_as_longlong(A.lu[q]);
        }
    }
    if constexpr (SF) {
        int spins = 0;
        uint64_t t0 = 0;
        for (;;) {
            bool pending = false;
#pragma unroll
            for (int m = 0; m < JM; ++m) pending |= (qs[m] >= 0 && raw[m] == kPending64);
            if (!pending) break;
            for (int k = 0; k < A.poll_sleep; ++k) __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int m = 0; m < JM; ++m)
                if (qs[m] >= 0 && raw[m] == kPending64)
                    raw[m] = ld_acq_u64(reinterpret_cast<const uint64_t *>(&A.lu[qs[m]]));
            if ((++spins & 63) == 0) {
                if (aborted(A.info)) break;
                if (expired(t0)) {
                    __hip_atomic_store(&A.info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < JM; ++m)
        if (qs[m] >= 0) sv[t + m * G] = __longlong_as_double((long long)raw[m]);
    for (int j = t + JM * G; j < total; j += G) {
        int e = 0;
        while (e + 1 < nL && soff[e + 1] <= j) ++e;
        const int q = sdc[e] + (j - soff[e]);
        sc[j] = (A.use_flev && A.flev[q] > A.k) ? -1 : A.ci[q];
        double uv;
        if constexpr (SF) uv = Pub<double>::wait(&A.lu[q], A.info, A.poll_sleep);
        else uv = A.lu[q];
        sv[j] = uv;
    }
    wave_sync_lds();
    // ---- match: off the elimination chain ----
    const double mypiv = (t < nL && len > 0) ? sv[off] : 1.0;
    double wv[MAXL];
    uint64_t mmask = 0;
#pragma unroll
    for (int e = 0; e < MAXL; ++e) {
        wv[e] = 0.0;
        if (e < nL && act && !absent) {
            const int oe = soff[e];
            const int le = (e + 1 < nL ? soff[e + 1] : total) - oe;
            // columns of U(c_e) ascend: binary search for this lane's column in [oe + 1, oe + le)
            int lo = oe + 1, hi = oe + le;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sc[mid] < col && sc[mid] >= 0) lo = mid + 1;
                else if (sc[mid] < 0) {
                    // absent entries keep their column order; read the true column
                    const int q = sdc[e] + (mid - oe);
                    if (A.ci[q] < col) lo = mid + 1;
                    else hi = mid;
                } else hi = mid;
            }
            if (lo < oe + le && sc[lo] == col) {
                const double u = sv[lo];
                if ((uint64_t)__double_as_longlong(u) != kDropped64) {
                    wv[e] = u;
                    mmask |= 1ull << e;
                    // modified ILU: positions another lane takes are marked for the
                    // diagonal lane, which gives back the rest (the search of this
                    // region has ended for every lane of the group)
                    if (A.milu && t != dl) sc[lo] = kTaken;
                }
            }
        }
    }
    wave_sync_lds();   // the slice is reused by the group's next row (or, in the
                       // modified form, read by the diagonal lane in the chain)
    // ---- chain ----
#pragma unroll
    for (int e = 0; e < MAXL; ++e) {
        if (e < nL) {                                   // uniform across the group
            if (__shfl(len, e, G) != 0) {               // kept dependency
                double before = 0.0;
                if (t == e) {
                    before = v;
                    v = v / mypiv;
                    if (A.use_tau && fabs(v) < tr) dropped = 1;
                }
                const int de = __shfl(dropped, e, G);
                const double l = __shfl(v, e, G);
                const double bv = A.milu ? __shfl(before, e, G) : 0.0;
                if (A.milu && t == dl) {
                    if (de) {
                        v = v + bv;
                    } else {
                        // U(c_e) in column order: kept entries no other lane took
                        const int oe = soff[e];
                        const int le = (e + 1 < nL ? soff[e + 1] : total) - oe;
                        for (int j = oe + 1; j < oe + le; ++j) {
                            const int cj = sc[j];
                            const double u = sv[j];
                            if (cj >= 0 && (uint64_t)__double_as_longlong(u) != kDropped64) {
                                const double lost = l * u;
                                v = v - lost;
                            }
                        }
                    }
                } else if (!de && ((mmask >> e) & 1ull)) {
                    const double prod = l * wv[e];
                    v = v - prod;
                }
            }
        }
    }
    if (A.milu) wave_sync_lds();   // the diagonal lane's reads end before the next row's gather
    factor_finish<G, SF>(A, r, t, gi, p, act, col, absent, dropped, v, tr, d - rs);
}

// Long rows (more than 64 entries): one wave per row, the row's values in an LDS
// buffer.  For each kept L entry c in ascending column order every lane computes
// l = a_rc / u_cc (the same operation, the same result); lane 0 keeps it.  The
// U(c) entries are then taken 64 at a time, lane j finding its column in row r
// by binary search and updating that entry -- each target is hit at most once per
// c, so every entry sees the serial algorithm's updates in its order (Sec. III,
// Fig. 1).  Updates that land on the diagonal (its own, and in the modified form
// the ones whose target row r does not hold) are applied by lane 0 in U(c)'s
// column order.
template <bool SF>
__device__ void factor_row_long(const FactorArgs &A, int r, int lane, double *rv) {
    const int rs = A.rp[r], re = A.rp[r + 1], d = A.diag[r];
    const int len = re - rs, dl = d - rs;
    const double tr = A.use_tau ? A.row_tau[r] : 0.0;
    for (int k = lane; k < len; k += 64) {
        const int p = rs + k;
        const bool absent = A.use_flev && A.flev[p] > A.k;
        const int s = A.src[p];
        rv[k] = (s >= 0 && !absent) ? A.a[s] : 0.0;
    }
    wave_sync_lds();
    for (int e = 0; e < dl; ++e) {
        const int p = rs + e;
        if (A.use_flev && A.flev[p] > A.k) continue;   // absent L entry
        const int c = A.ci[p];
        const int dc = A.diag[c], ec = A.rp[c + 1];
        double piv;
        if constexpr (SF) piv = Pub<double>::wait(&A.lu[dc], A.info, A.poll_sleep);
        else piv = A.lu[dc];
        const double before = rv[e];
        const double l = before / piv;
        if (A.use_tau && fabs(l) < tr) {
            if (lane == 0) {
                rv[e] = __longlong_as_double((long long)kDropped64);
                if (A.milu) rv[dl] = rv[dl] + before;
            }
            wave_sync_lds();
            continue;
        }
        if (lane == 0) rv[e] = l;
        for (int j0 = dc + 1; j0 < ec; j0 += 64) {
            const int j = j0 + lane;
            const bool act = j < ec;
            int pos = -1;
            bool kept = false;
            double u = 0.0;
            if (act) {
                const bool uabs = A.use_flev && A.flev[j] > A.k;
                if (!uabs) {
                    if constexpr (SF) u = Pub<double>::wait(&A.lu[j], A.info, A.poll_sleep);
                    else u = A.lu[j];
                    kept = (uint64_t)__double_as_longlong(u) != kDropped64;
                }
                if (kept) {
                    const int col = A.ci[j];
                    int lo = rs, hi = re;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (A.ci[mid] < col) lo = mid + 1;
                        else hi = mid;
                    }
                    if (lo < re && A.ci[lo] == col && !(A.use_flev && A.flev[lo] > A.k)) pos = lo - rs;
                }
            }
            const double prod = l * u;
            if (pos >= 0 && pos != dl) rv[pos] = rv[pos] - prod;
            // diagonal updates in column order
            uint64_t dm = __ballot(kept && (pos == dl || (A.milu && pos < 0)));
            while (dm) {
                const int b = __builtin_ctzll(dm);
                dm &= dm - 1;
                const double q = __shfl(prod, b, 64);
                if (lane == 0) rv[dl] = rv[dl] - q;
            }
        }
        wave_sync_lds();
    }
    // U entries below the drop threshold at the end of the row, in column order
    if (A.use_tau && lane == 0) {
        for (int k = dl + 1; k < len; ++k) {
            if (A.use_flev && A.flev[rs + k] > A.k) continue;
            const double v = rv[k];
            if (fabs(v) < tr) {
                if (A.milu) rv[dl] = rv[dl] + v;
                rv[k] = __longlong_as_double((long long)kDropped64);
            }
        }
    }
    wave_sync_lds();
    const double pv = rv[dl];
    bool bad = false;
    for (int k = lane; k < len; k += 64) {
        const int p = rs + k;
        const bool absent = A.use_flev && A.flev[p] > A.k;
        const double v = rv[k];
        const uint64_t raw = (uint64_t)__double_as_longlong(v);
        uint64_t bits;
        if (absent) bits = 0;
        else if (raw == kDropped64) bits = kDropped64;
        else {
            if (!isfinite(v)) bad = true;
            bits = (v != v) ? kQNaN64 : raw;
        }
        if constexpr (SF) st_pub_u64(reinterpret_cast<uint64_t *>(&A.lu[p]), bits);
        else A.lu[p] = __longlong_as_double((long long)bits);
    }
    const bool any_bad = __ballot(bad) != 0;
    if (lane == 0) {
        if (pv == 0.0) atomicMin(&A.info[kInfoBadKey], 2 * r);
        else if (any_bad) atomicMin(&A.info[kInfoBadKey], 2 * r + 1);
    }
    wave_sync_lds();   // the buffer is reused by the wave's next row
}

template <bool SF>
__global__ __launch_bounds__(kBlock) void k_factor_long(FactorArgs A) {
    extern __shared__ double lds_f[];
    const int lane = threadIdx.x & 63;
    double *rv = lds_f + (size_t)(threadIdx.x >> 6) * A.lcap;
    if constexpr (SF) {
        claim_task(A.claims, A.nstreams, [&](int task) {
            const int r = A.claims.task_ptr[task];
            if (r < A.claims.task_ptr[task + 1]) factor_row_long<true>(A, r, lane, rv);
        });
    } else {
        const int r = A.row_begin + (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
        if (r < A.row_end) factor_row_long<false>(A, r, lane, rv);
    }
}

// per-group LDS slices: [ngroups][tcap] doubles, then per group tcap + 2G ints
template <int G>
__device__ __forceinline__ void group_slices(int tcap, double *&sv, int *&sc, int *&soff, int *&sdc) {
    extern __shared__ double lds_f[];
    constexpr int ngroups = kBlock / G;
    const int g = threadIdx.x / G;
    sv = lds_f + g * tcap;
    int *ib = reinterpret_cast<int *>(lds_f + ngroups * tcap);
    sc = ib + g * (tcap + 2 * G);
    soff = sc + tcap;
    sdc = soff + G;
}

// MAXL > 0: staged rows with at most MAXL strictly lower entries; MAXL == 0: unstaged
template <int G, int MAXL>
__global__ __launch_bounds__(kBlock) void k_factor_level(FactorArgs A) {
    const int gid = (blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int t = threadIdx.x % G;
    const int gi = (threadIdx.x & 63) / G;
    const int r = A.row_begin + gid;
    if constexpr (MAXL > 0) {
        double *sv;
        int *sc, *soff, *sdc;
        group_slices<G>(A.tcap, sv, sc, soff, sdc);
        if (r < A.row_end) factor_row_staged<G, MAXL, false>(A, r, t, gi, sv, sc, soff, sdc);
    } else {
        if (r < A.row_end) factor_row<G, false>(A, r, t, gi);
    }
}

template <int G, int MAXL>
__global__ __launch_bounds__(kBlock) void k_factor_syncfree(FactorArgs A) {
    const int t = threadIdx.x % G;
    const int gi = (threadIdx.x & 63) / G;
    double *sv = nullptr;
    int *sc = nullptr, *soff = nullptr, *sdc = nullptr;
    if constexpr (MAXL > 0) group_slices<G>(A.tcap, sv, sc, soff, sdc);
    claim_task(A.claims, A.nstreams, [&](int task) {
        const int r = A.claims.task_ptr[task] + gi;
        if (r < A.claims.task_ptr[task + 1]) {
            if constexpr (MAXL > 0) factor_row_staged<G, MAXL, true>(A, r, t, gi, sv, sc, soff, sdc);
            else factor_row<G, true>(A, r, t, gi);
        }
    });
}

// ---------------------------------------------------------------------------------
// Triangular solves (paper Sec. VI), one row per group, lanes over the row's entries
// ---------------------------------------------------------------------------------
// Forward: y_r = (b'_r - sum_{c<r} a_rc y_c) [/ a_rr unless unit]; b' = P b.
// Backward: z_r = (y_r - sum_{c>r} a_rc z_c) [/ a_rr unless unit]; x = P^T z.
// The y and z buffers keep the invariant "all pending" between applies: the
// forward pass re-arms z[r], the backward pass re-arms y[r] after reading it.
template <typename TA>
__device__ __forceinline__ TA load_vec(const void *v, int f32, int64_t i) {
    return f32 ? (TA) static_cast<const float *>(v)[i] : (TA) static_cast<const double *>(v)[i];
}
template <typename TA>
__device__ __forceinline__ void store_vec(void *v, int f32, int64_t i, TA x) {
    if (f32) static_cast<float *>(v)[i] = (float)x;
    else static_cast<double *>(v)[i] = (double)x;
}

// NR right-hand sides per pass: every lane accumulates all NR sums over its
// entries (the NR values of one dependency row are adjacent in the [n][cap]
// buffers), then lane t finishes right-hand sides t, t + G, ... of the batch.
template <int G, int NR, typename TV, typename TA, bool SF, bool FWD>
__device__ __forceinline__ void solve_row(const SolveArgs &A, int r, int t) {
    constexpr int RPL = (NR + G - 1) / G;   // right-hand sides finished per lane
    const TV *val = static_cast<const TV *>(A.val);
    TA *y = static_cast<TA *>(A.y);
    TA *z = static_cast<TA *>(A.z);
    const int rs = A.rp[r], re = A.rp[r + 1], d = A.diag[r];
    const int lo = FWD ? rs : d + 1;
    const int hi = FWD ? d : re;
    TA *dep = FWD ? y : z;
    const int64_t cap = A.cap;
    const int out_row = A.perm ? A.perm[r] : r;
    // everything that does not depend on other rows is loaded before the waits
    const TA inv_piv = A.unit_diag ? (TA)1 : (TA)load_val(val, A.vmap ? A.vmap[d] : d);
    for (int s0 = 0; s0 < A.nrhs; s0 += NR) {
        const int nr = A.nrhs - s0 < NR ? A.nrhs - s0 : NR;
        TA rhs[RPL];
#pragma unroll
        for (int m = 0; m < RPL; ++m) {
            const int k = t + m * G;
            rhs[m] = 0;
            if (k < nr) {
                if constexpr (FWD) rhs[m] = load_vec<TA>(A.b, A.vec_f32, (int64_t)out_row * A.ld + s0 + k);
                else rhs[m] = y[(int64_t)r * cap + s0 + k];
            }
        }
        TA acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = 0;
        for (int p = lo + t; p < hi; p += G) {
            const int c = A.ci[p];
            const TA a = (TA)load_val(val, A.vmap ? A.vmap[p] : p);
            const TA *dc = dep + (int64_t)c * cap + s0;
            if constexpr (SF) {
                // all loads of the batch first, then wait only on values still pending
                typename Pub<TA>::U raw[NR];
#pragma unroll
                for (int k = 0; k < NR; ++k) raw[k] = k < nr ? Pub<TA>::load(dc + k) : 0;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    if (k < nr) {
                        TA xc = Pub<TA>::from(raw[k]);
                        if (raw[k] == Pub<TA>::kPend) xc = Pub<TA>::wait(dc + k, A.info, A.poll_sleep);
                        const TA prod = a * xc;
                        acc[k] = acc[k] + prod;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    if (k < nr) {
                        const TA prod = a * dc[k];
                        acc[k] = acc[k] + prod;
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const TA sum = group_sum<G>(acc[k]);
            if (k < nr && (k % G) == t) {
                TA v = rhs[k / G] - sum;
                if (!A.unit_diag) v = v / inv_piv;
                const int64_t o = (int64_t)r * cap + s0 + k;
                if constexpr (FWD) {
                    if constexpr (SF) Pub<TA>::publish(&y[o], v);
                    else y[o] = v;
                    z[o] = Pub<TA>::pending();
                    if (A.y_out) static_cast<TA *>(A.y_out)[(int64_t)r * A.ld + s0 + k] = v;
                } else {
                    if constexpr (SF) Pub<TA>::publish(&z[o], v);
                    else z[o] = v;
                    y[o] = Pub<TA>::pending();
                    store_vec<TA>(A.x, A.vec_f32, (int64_t)out_row * A.ld + s0 + k, v);
                    if (A.z_out) static_cast<TA *>(A.z_out)[(int64_t)r * A.ld + s0 + k] = v;
                }
            }
        }
    }
}

template <int G, int NR, typename TV, typename TA, bool FWD>
__global__ __launch_bounds__(kBlock) void k_solve_level(SolveArgs A) {
    const int pos = A.row_begin + (blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (pos >= A.row_end) return;
    const int r = A.rows ? A.rows[pos] : pos;
    solve_row<G, NR, TV, TA, false, FWD>(A, r, threadIdx.x % G);
}

template <int G, int NR, typename TV, typename TA, bool FWD>
__global__ __launch_bounds__(kBlock) void k_solve_syncfree(SolveArgs A) {
    const int t = threadIdx.x % G;
    const int gi = (threadIdx.x & 63) / G;
    claim_task(A.claims, A.nstreams, [&](int task) {
        const int pos = A.claims.task_ptr[task] + gi;
        if (pos < A.claims.task_ptr[task + 1]) {
            const int r = A.rows ? A.rows[pos] : pos;
            solve_row<G, NR, TV, TA, true, FWD>(A, r, t);
        }
    });
}

// ---------------------------------------------------------------------------------
// Tiled sync-free solve: one workgroup per tile, everything the tile reads in LDS
// ---------------------------------------------------------------------------------
// LDS of a block: the value slots (tile rows, then imports, then one slot that
// holds 0 for padded entries), the staged rows (dependency slots and factor
// values packed kmax per row, pivot, right-hand side, row id) and the position ->
// slot map.  Every value slot starts as the pending pattern, so the value is its
// own flag.  The poller wave copies imports from the published y/z buffers as
// they appear.  Compute wave w takes the chunks w, w + 4, ... of kTileUnit
// positions; a chunk holds rows of one local level and every dependency inside
// the tile sits in an earlier chunk, so the lowest unfinished chunk can always
// proceed, and imports only come from earlier tiles.

template <typename TA>
__device__ __forceinline__ typename Pub<TA>::U lds_ld(typename Pub<TA>::U *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename TA>
__device__ __forceinline__ void lds_st(typename Pub<TA>::U *p, typename Pub<TA>::U v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename TA>
__device__ __forceinline__ typename Pub<TA>::U bits_of(TA v);
template <>
__device__ __forceinline__ uint64_t bits_of<double>(double v) {
    return v != v ? kQNaN64 : (uint64_t)__double_as_longlong(v);
}
template <>
__device__ __forceinline__ uint32_t bits_of<float>(float v) {
    return v != v ? kQNaN32 : __float_as_uint(v);
}
template <typename TA>
__device__ __forceinline__ TA qnan_of() {
    return Pub<TA>::from(sizeof(TA) == 8 ? (typename Pub<TA>::U)kQNaN64 : (typename Pub<TA>::U)kQNaN32);
}

// Bounded wait of a compute wave on an LDS word.  It never touches global memory
// except to raise the device abort flag: a global load here would make the wave
// wait for its own outstanding global stores before the load's result is used
// (stores and loads share one counter), which would put a store round trip on
// every step.  The poller mirrors the device abort flag into *lds_abort.
template <typename TA>
__device__ TA lds_wait(typename Pub<TA>::U *p, int *lds_abort, int32_t *info) {
    using U = typename Pub<TA>::U;
    int spins = 0;
    uint64_t t0 = 0;
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        const U v = lds_ld<TA>(p);
        if (v != Pub<TA>::kPend) return Pub<TA>::from(v);
        if ((++spins & 63) == 0) {
            if (__hip_atomic_load(lds_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return qnan_of<TA>();
            if (expired(t0)) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(lds_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return qnan_of<TA>();
            }
        }
    }
}

// Poller: copies the tile's imports (right-hand sides s0 .. s0 + nr - 1) from
// the published buffer into LDS slots `first` .. as they appear.  The imported
// rows are staged in LDS with the tile, so a round costs one global load per
// pending import.  Imports are numbered in order of first use; the poller works
// on a window of kPollBatch rows of 64 imports starting at the first unresolved
// row, which moves on once that row is resolved, and rounds that find nothing new
// back off up to kPollMaxSleep pause steps.  Bounded like every wait.
constexpr int kPollBatch = 2;
constexpr int kPollMaxSleep = 8;
constexpr int kStageRows = 4;   // rows per lane group per staging step
constexpr int kStageCopy = 8;   // elements per thread per staging copy step

template <int NR, typename TA>
__device__ void tile_poll(const int32_t *imp, int nimp, const TA *dep, int64_t cap, int s0, int nr,
                          typename Pub<TA>::U *vals, int first, int32_t *info, int sleep0,
                          int *lds_abort) {
    using U = typename Pub<TA>::U;
    const int lane = threadIdx.x & 63;
    const int total = nimp * nr;
    int head = 0, sleep = 0, spins = 0;
    uint64_t t0 = 0;
    while (head < total) {
        U raw[kPollBatch];
        int sl[kPollBatch];
#pragma unroll
        for (int b = 0; b < kPollBatch; ++b) {
            const int i = head + 64 * b + lane;
            sl[b] = -1;
            raw[b] = Pub<TA>::kPend;
            if (i < total) {
                const int m = i / nr, k = i - m * nr;
                const int q = (first + m) * NR + k;
                if (lds_ld<TA>(vals + q) == Pub<TA>::kPend) {
                    sl[b] = q;
                    raw[b] = Pub<TA>::load(dep + (int64_t)imp[m] * cap + s0 + k);
                }
            }
        }
        bool got = false, pend0 = false;
#pragma unroll
        for (int b = 0; b < kPollBatch; ++b) {
            if (sl[b] < 0) continue;
            if (raw[b] != Pub<TA>::kPend) {
                lds_st<TA>(vals + sl[b], raw[b]);
                got = true;
            } else if (b == 0) {
                pend0 = true;
            }
        }
        if (!__any(pend0)) {   // the first window row is resolved: move on
            head += 64;
            continue;
        }
        sleep = __any(got) ? sleep0 : (sleep * 2 + 1 < kPollMaxSleep ? sleep * 2 + 1 : kPollMaxSleep);
        for (int k = 0; k < sleep; ++k) __builtin_amdgcn_s_sleep(1);
        if ((++spins & 15) == 0) {
            if (aborted(info)) break;
            if (expired(t0)) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    if (head >= total) return;
    // aborted: release every waiter of this block with a quiet NaN
    if (lane == 0) __hip_atomic_store(lds_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (int i = lane; i < total; i += 64) {
        const int m = i / nr, k = i - m * nr;
        U *p = vals + (first + m) * NR + k;
        if (lds_ld<TA>(p) == Pub<TA>::kPend) lds_st<TA>(p, bits_of<TA>(qnan_of<TA>()));
    }
}

// Global stores of one solved value: publish it, re-arm the other buffer, write
// the outputs.
template <typename TA, bool FWD>
__device__ __forceinline__ void tile_store(const SolveArgs &A, int r, int orow, int col, TA v) {
    TA *y = static_cast<TA *>(A.y);
    TA *z = static_cast<TA *>(A.z);
    const int64_t o = (int64_t)r * A.cap + col;
    if constexpr (FWD) {
        Pub<TA>::publish(&y[o], v);
        z[o] = Pub<TA>::pending();
        if (A.y_out) static_cast<TA *>(A.y_out)[(int64_t)r * A.ld + col] = v;
    } else {
        Pub<TA>::publish(&z[o], v);
        y[o] = Pub<TA>::pending();
        store_vec<TA>(A.x, A.vec_f32, (int64_t)orow * A.ld + col, v);
        if (A.z_out) static_cast<TA *>(A.z_out)[(int64_t)r * A.ld + col] = v;
    }
}

// Copies n elements from global memory into LDS, every thread issuing U loads
// before storing any.
template <int U, int B = kTileBlock, typename T>
__device__ __forceinline__ void lds_copy(T *dst, const T *__restrict__ src, int n) {
    for (int i0 = threadIdx.x; i0 < n; i0 += B * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * B;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * B;
            if (i < n) dst[i] = v[u];
        }
    }
}

// The staged data of one row of a chunk, loaded one chunk ahead: with G = 1 a lane
// holds all (at most J) dependencies of its row, with G > 1 lane t of the row's
// group holds entries t, t + G, ... (at most J of them).
template <int J, int NR, typename TA>
struct TileRow {
    int sl;              // LDS slot of the row (-1: padding)
    int dsl[J];
    TA a[J];
    int r;
    TA pv;
    TA rhs[NR];
};

template <int G, int J, int NR, typename TA>
__device__ __forceinline__ void tile_row_load(TileRow<J, NR, TA> &R, const int16_t *ps, const TA *ev,
                                              const uint16_t *es, const int32_t *rowid, const TA *piv, const TA *rhs,
                                              int K, int pos, int t, int nr) {
    R.sl = ps[pos];
    if (R.sl < 0) return;
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
        const int j = t + jj * G;
        R.dsl[jj] = j < K ? es[R.sl * K + j] : -1;
        R.a[jj] = j < K ? ev[R.sl * K + j] : (TA)0;
    }
    R.r = rowid[R.sl];
    R.pv = piv[R.sl];
#pragma unroll
    for (int k = 0; k < NR; ++k) R.rhs[k] = k < nr ? rhs[R.sl * NR + k] : (TA)0;
}

// Compute waves: wave w solves the chunks w, w + solve_waves<TA>(), ... of the
// tile (a chunk is 64 / G positions of one local level), writing each value only
// to its LDS slot and publishing it.  The next chunk's staged row data is loaded
// while the current one waits and computes, and all dependency values of a row
// are read at once, so one LDS round trip plus the arithmetic separates one local
// level from the next.  The wave issues no global load: the bounded waits only
// look at LDS (a global load would make the wave wait for its outstanding
// stores before using the result).  Every row of the tile has
// at most J * G dependencies (the launcher checks).  With G = 1 a lane sums its
// row's products in column order; with G > 1 the lanes of a group sum their
// entries and the group adds them up.
template <int G, int J, int NR, typename TA, bool FWD>
__device__ __forceinline__ void tile_compute(const SolveArgs &A, typename Pub<TA>::U *vals, const TA *ev,
                                             const uint16_t *es, const int16_t *ps, const int32_t *rowid,
                                             const int32_t *orows, const TA *piv, const TA *rhs, int K, int npos,
                                             int wave, int gi, int t, int s0, int nr, int *lds_abort) {
    using U = typename Pub<TA>::U;
    constexpr int UNIT = 64 / G;
    constexpr int STEP = solve_waves<TA>() * UNIT;
    TileRow<J, NR, TA> cur;
    int c0 = wave * UNIT;
    cur.sl = -1;
    if (c0 < npos) tile_row_load<G, J, NR, TA>(cur, ps, ev, es, rowid, piv, rhs, K, c0 + gi, t, nr);
    for (; c0 < npos; c0 += STEP) {
        TileRow<J, NR, TA> nxt;
        nxt.sl = -1;
        if (c0 + STEP < npos) tile_row_load<G, J, NR, TA>(nxt, ps, ev, es, rowid, piv, rhs, K, c0 + STEP + gi, t, nr);
        if (cur.sl >= 0) {
            U raw[J][NR];
#pragma unroll
            for (int jj = 0; jj < J; ++jj)
#pragma unroll
                for (int k = 0; k < NR; ++k)
                    raw[jj][k] = (cur.dsl[jj] >= 0 && k < nr) ? lds_ld<TA>(vals + cur.dsl[jj] * NR + k) : 0;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                TA acc = 0;
#pragma unroll
                for (int jj = 0; jj < J; ++jj) {
                    if (cur.dsl[jj] >= 0 && k < nr) {
                        TA xc = Pub<TA>::from(raw[jj][k]);
                        if (raw[jj][k] == Pub<TA>::kPend)
                            xc = lds_wait<TA>(vals + cur.dsl[jj] * NR + k, lds_abort, A.info);
                        const TA prod = cur.a[jj] * xc;
                        acc = acc + prod;
                    }
                }
                const TA sum = group_sum<G>(acc);
                if (k < nr && (k % G) == t) {
                    TA v = cur.rhs[k] - sum;
                    // a unit diagonal (L, or L^T of the adjoint) needs nothing; else
                    // multiply by the reciprocal of the pivot taken at staging, off
                    // the dependency chain
                    if (!A.unit_diag) v = v * cur.pv;
                    lds_st<TA>(vals + cur.sl * NR + k, bits_of<TA>(v));
                    tile_store<TA, FWD>(A, cur.r, orows[cur.sl], s0 + k, v);
                }
            }
        }
        cur = nxt;
    }
}

template <int G, int J, int NR, typename TV, typename TA, bool FWD>
__global__ __launch_bounds__(solve_block<TA>()) void k_solve_tiled(SolveArgs A, TileArgs T) {
    constexpr int B = solve_block<TA>();
    using U = typename Pub<TA>::U;
    extern __shared__ __align__(16) unsigned char tile_smem[];
    U *vals = reinterpret_cast<U *>(tile_smem);
    TA *rhs = reinterpret_cast<TA *>(tile_smem + T.off_rhs);
    TA *piv = reinterpret_cast<TA *>(tile_smem + T.off_piv);
    TA *ev = reinterpret_cast<TA *>(tile_smem + T.off_eval);
    uint16_t *es = reinterpret_cast<uint16_t *>(tile_smem + T.off_eslot);
    int32_t *rowid = reinterpret_cast<int32_t *>(tile_smem + T.off_rowid);
    int16_t *ps = reinterpret_cast<int16_t *>(tile_smem + T.off_pslot);
    int32_t *impl = reinterpret_cast<int32_t *>(tile_smem + T.off_imp);
    int32_t *orows = reinterpret_cast<int32_t *>(tile_smem + T.off_orow);
    __shared__ int s_tile;
    __shared__ int s_abort;
    if (threadIdx.x == 0) {
        if (T.zero_counter && blockIdx.x == 0) T.zero_counter[0] = 0;
        s_tile = __hip_atomic_fetch_add(T.counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_abort = 0;
    }
    __syncthreads();
    const int tile = s_tile;
    if (tile >= T.ntiles) return;
    const int pbase = T.tile_ptr[tile], npos = T.tile_ptr[tile + 1] - pbase;
    const int rbase = T.rows_ptr[tile], nrows = T.rows_ptr[tile + 1] - rbase;
    const int ibase = T.imp_ptr[tile], nimp = T.imp_ptr[tile + 1] - ibase;
    const int K = T.kmax;
    const int zero = T.max_slots;   // the slot that always holds 0
    const TV *val = static_cast<const TV *>(A.val);
    TA *y = static_cast<TA *>(A.y);
    TA *z = static_cast<TA *>(A.z);
    const int64_t cap = A.cap;
    const int t = threadIdx.x % G;

    // stage the tile (every thread issues all loads of a step before it uses any):
    // position -> slot, imports, then per row its id, pivot, dependency slots and
    // values.  When the position and import tables each fit one step of the block,
    // their loads are issued here and stored after the row loop has issued its
    // own, so the three chains share one memory latency.
    constexpr int PC = 2;   // elements per thread of each table in that case
    const bool one_step = npos <= B * PC && nimp <= B * PC;
    int16_t pv_pos[PC];
    int32_t pv_imp[PC];
    if (one_step) {
#pragma unroll
        for (int u = 0; u < PC; ++u) {
            const int i = threadIdx.x + u * B;
            pv_pos[u] = i < npos ? T.pslot[pbase + i] : (int16_t)0;
            pv_imp[u] = i < nimp ? T.imp[ibase + i] : 0;
        }
    } else {
        lds_copy<kStageCopy, B>(ps, T.pslot + pbase, npos);
        lds_copy<kStageCopy, B>(impl, T.imp + ibase, nimp);
    }
    constexpr int SR = kStageRows;
    constexpr int SJ = G == 1 ? 4 : 2;   // entries per lane fetched with the batched loads
    constexpr int GROUPS = B / G;
    for (int s0r = threadIdx.x / G; s0r < nrows; s0r += GROUPS * SR) {
        int4 mt[SR];
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            const int sl = s0r + u * GROUPS;
            mt[u] = sl < nrows ? T.meta[rbase + sl] : make_int4(-1, 0, 0, 0);
        }
        TA pv[SR];
        int es_r[SR][SJ];
        TA ev_r[SR][SJ];
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            // values through the view's gather map (transposed views) when there is one
            pv[u] = (mt[u].x >= 0 && !A.unit_diag) ? (TA)load_val(val, A.vmap ? A.vmap[mt[u].w] : mt[u].w) : (TA)1;
#pragma unroll
            for (int jj = 0; jj < SJ; ++jj) {
                const int p = mt[u].y + t + jj * G;
                const bool on = mt[u].x >= 0 && p < mt[u].z;
                es_r[u][jj] = on ? T.sci[p] : zero;
                ev_r[u][jj] = on ? (TA)load_val(val, A.vmap ? A.vmap[p] : p) : (TA)0;
            }
        }
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            const int sl = s0r + u * GROUPS;
            if (sl >= nrows) continue;
            if (t == 0) {
                rowid[sl] = mt[u].x;
                piv[sl] = A.unit_diag ? (TA)1 : (TA)1 / pv[u];
                if constexpr (!FWD) orows[sl] = mt[u].x;
            }
#pragma unroll
            for (int jj = 0; jj < SJ; ++jj) {
                const int j = t + jj * G;
                if (j < K) {
                    es[sl * K + j] = (uint16_t)es_r[u][jj];
                    ev[sl * K + j] = ev_r[u][jj];
                }
            }
            // longer rows: the rest one by one
            for (int j = t + SJ * G; j < K; j += G) {
                const int p = mt[u].y + j;
                const bool on = p < mt[u].z;
                es[sl * K + j] = (uint16_t)(on ? T.sci[p] : zero);
                ev[sl * K + j] = on ? (TA)load_val(val, A.vmap ? A.vmap[p] : p) : (TA)0;
            }
        }
    }
    if (one_step) {
#pragma unroll
        for (int u = 0; u < PC; ++u) {
            const int i = threadIdx.x + u * B;
            if (i < npos) ps[i] = pv_pos[u];
            if (i < nimp) impl[i] = pv_imp[u];
        }
    }
    if constexpr (!FWD) {
        if (A.perm) {
            __syncthreads();
            for (int i0 = threadIdx.x; i0 < nrows; i0 += B * kStageCopy) {
                int o[kStageCopy];
#pragma unroll
                for (int u = 0; u < kStageCopy; ++u) {
                    const int i = i0 + u * B;
                    if (i < nrows) o[u] = A.perm[rowid[i]];
                }
#pragma unroll
                for (int u = 0; u < kStageCopy; ++u) {
                    const int i = i0 + u * B;
                    if (i < nrows) orows[i] = o[u];
                }
            }
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int gi = (threadIdx.x & 63) / G;
    for (int s0 = 0; s0 < A.nrhs; s0 += NR) {
        const int nr = A.nrhs - s0 < NR ? A.nrhs - s0 : NR;
        for (int i = threadIdx.x; i < (nrows + nimp) * NR; i += B) vals[i] = Pub<TA>::kPend;
        if (threadIdx.x < NR) vals[zero * NR + threadIdx.x] = bits_of<TA>((TA)0);
        for (int i0 = threadIdx.x; i0 < nrows * nr; i0 += B * kStageCopy) {
            int64_t at[kStageCopy];
#pragma unroll
            for (int u = 0; u < kStageCopy; ++u) {
                const int i = i0 + u * B;
                at[u] = -1;
                if (i < nrows * nr) {
                    const int sl = i / nr, k = i - sl * nr;
                    const int r = rowid[sl];
                    if constexpr (FWD) at[u] = (int64_t)r * A.ld + s0 + k;   // permuted below if needed
                    else at[u] = (int64_t)r * cap + s0 + k;
                }
            }
            if constexpr (FWD) {
                if (A.perm) {
#pragma unroll
                    for (int u = 0; u < kStageCopy; ++u) {
                        const int i = i0 + u * B;
                        if (at[u] >= 0) {
                            const int sl = i / nr, k = i - sl * nr;
                            at[u] = (int64_t)A.perm[rowid[sl]] * A.ld + s0 + k;
                        }
                    }
                }
            }
            TA bv[kStageCopy];
#pragma unroll
            for (int u = 0; u < kStageCopy; ++u) {
                if (at[u] < 0) continue;
                if constexpr (FWD) bv[u] = load_vec<TA>(A.b, A.vec_f32, at[u]);
                else bv[u] = y[at[u]];
            }
#pragma unroll
            for (int u = 0; u < kStageCopy; ++u) {
                const int i = i0 + u * B;
                if (at[u] < 0) continue;
                const int sl = i / nr, k = i - sl * nr;
                rhs[sl * NR + k] = bv[u];
            }
        }
        __syncthreads();
        if (wave == solve_waves<TA>()) {
            tile_poll<NR, TA>(impl, nimp, FWD ? y : z, cap, s0, nr, vals, nrows, A.info, A.poll_sleep, &s_abort);
        } else {
            // One wait per pass for all this wave has outstanding (the staging
            // loads have landed; at most the previous pass's stores remain).  It
            // clears the compiler's bookkeeping, which otherwise carries the
            // poller's loads around the pass loop and waits on the wave's own
            // stores inside the compute loop, once per chunk.
            __builtin_amdgcn_s_waitcnt(0);
            tile_compute<G, J, NR, TA, FWD>(A, vals, ev, es, ps, rowid, orows, piv, rhs, K, npos, wave, gi, t, s0, nr,
                                            &s_abort);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// Lower stage (tail) of a triangular solve: one workgroup streams the narrow
// levels at the end of the level order (Sec. III-B, Fig. 7)
// ---------------------------------------------------------------------------------
// Wave 0 computes the steps in order.  For each step it reads the staged
// coefficients and dependency values (a dependency computed a few steps earlier
// is read from the ring of recent results, any other one was fetched by a stager
// from the published buffer), sums each row's products over its lane group,
// writes the result to the ring and publishes it.  Waves 1..kStreamStagers take
// steps round-robin and stage step s into buffer s % kTailQ once wave 0 has
// finished step s - kTailQ.  The lowest unstaged step only waits for steps at
// least kTailQ earlier, which wave 0 can always finish, so the block cannot
// deadlock; every wait is bounded and a raised abort flag releases all of them.
constexpr int kStreamBlock = 64 * (1 + kStreamStagers);
constexpr int kStreamEnt = 64 * kTailJ;   // entries of one step

// Sum over each lane's aligned group of 2^gl lanes (gl differs between groups of a
// wave; gmax is the largest); every lane of a group ends with the group's sum.
template <typename T>
__device__ __forceinline__ T seg_sum(T v, int gl, int gmax) {
    if (gmax >= 1) {
        const T w = dpp_mov<kDppQuadXor1>(v);
        if (gl >= 1) v = v + w;
    }
    if (gmax >= 2) {
        const T w = dpp_mov<kDppQuadXor2>(v);
        if (gl >= 2) v = v + w;
    }
    if (gmax >= 3) {
        const T w = dpp_mov<kDppHalfMirror>(v);
        if (gl >= 3) v = v + w;
    }
    if (gmax >= 4) {
        const T w = dpp_mov<kDppMirror>(v);
        if (gl >= 4) v = v + w;
    }
    if (gmax >= 5) {
        const T w = __shfl_xor(v, 16);
        if (gl >= 5) v = v + w;
    }
    if (gmax >= 6) {
        const T w = __shfl_xor(v, 32);
        if (gl >= 6) v = v + w;
    }
    return v;
}

// Bounded wait until the LDS counter *p reaches v; false when the block gives up
// (its abort word, the device abort flag when `global` allows a global load, or
// the wall-clock bound).  With `backoff` the pause between polls doubles up to 8
// steps (waves far ahead of the one they wait for poll LDS less).
__device__ bool lds_wait_ge(int *p, int v, int *labort, int32_t *info, bool global, bool backoff = false) {
    int spins = 0, pause = 1;
    uint64_t t0 = 0;
    for (;;) {
        if (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= v) return true;
        for (int k = 0; k < pause; ++k) __builtin_amdgcn_s_sleep(1);
        if (backoff && pause < 8) pause *= 2;
        if ((++spins & 63) == 0) {
            if (__hip_atomic_load(labort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
            if (global && aborted(info)) {
                __hip_atomic_store(labort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return false;
            }
            if (expired(t0)) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(labort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return false;
            }
        }
    }
}

// A step's record as a stager lane holds it, for the compute lane of the same
// number (lane < nlanes): its lane word, the row of its lane group (4 words), and
// its kTailJ entries (entry j * nlanes + lane of the record).  The row is read
// only by a group's leader lane.
template <int J>
struct StreamRec {
    int h, nent, nrows, nlanes;
    int li;
    int4 lr;
    int p[J], code[J];
};

template <int J>
__device__ __forceinline__ void stream_rec_load(StreamRec<J> &R, const StreamArgs &T, int4 hd, int lane) {
    R.h = hd.y;
    R.nent = hd.z;
    R.nrows = hd.y & 255;
    R.nlanes = (hd.y >> 8) & 255;
    const int off = hd.x;
    R.li = lane < R.nlanes ? T.rec[off + 4 * R.nrows + lane] : 0;
    R.lr = (lane < R.nlanes && ((R.li >> 16) & 1))
               ? *reinterpret_cast<const int4 *>(T.rec + off + 4 * (R.li & 255))
               : make_int4(0, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int e = j * R.nlanes + lane;
        R.p[j] = lane < R.nlanes ? T.rec[off + 4 * R.nrows + R.nlanes + e] : -1;
        R.code[j] = lane < R.nlanes ? T.rec[off + 4 * R.nrows + R.nlanes + R.nent + e] : -1;
    }
}

template <typename TV, typename TA, bool FWD>
__global__ __launch_bounds__(kStreamBlock) void k_solve_stream(SolveArgs A, StreamArgs T) {
    using U = typename Pub<TA>::U;
    constexpr int Q = kTailQ, E = kStreamEnt, W = kTailW, J = kTailJ, S = kStreamStagers;
    extern __shared__ __align__(16) unsigned char st_smem[];
    U *vals = reinterpret_cast<U *>(st_smem + T.off_vals);          // ring [W], staged old values [Q][E], zero
    TA *sa = reinterpret_cast<TA *>(st_smem + T.off_a);             // [Q][J][64] coefficients
    uint16_t *sc = reinterpret_cast<uint16_t *>(st_smem + T.off_c); // [Q][J][64] value slot of each entry
    // [Q][64] per compute lane: log2 group | leader << 8, and for a leader its
    // row's ring slot, row, output row; right-hand side and reciprocal pivot
    int4 *slane = reinterpret_cast<int4 *>(st_smem + T.off_lane);
    TA *srhs = reinterpret_cast<TA *>(st_smem + T.off_rhs);         // [Q][64]
    TA *spiv = reinterpret_cast<TA *>(st_smem + T.off_piv);         // [Q][64]
    int32_t *shdr = reinterpret_cast<int32_t *>(st_smem + T.off_hdr);     // [Q]
    int32_t *ready = reinterpret_cast<int32_t *>(st_smem + T.off_sync);   // [Q]
    int32_t *done = ready + Q;
    int32_t *labort = ready + Q + 1;
    const int zero = W + Q * E;
    const int col = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < Q; i += kStreamBlock) ready[i] = -1;
    if (threadIdx.x == 0) {
        *done = -1;
        *labort = 0;
        vals[zero] = bits_of<TA>((TA)0);
    }
    __syncthreads();
    const TV *val = static_cast<const TV *>(A.val);
    TA *y = static_cast<TA *>(A.y);
    TA *z = static_cast<TA *>(A.z);
    const int64_t cap = A.cap;
    if (wave == 0) {
        // Everything a step needs is staged per compute lane, so the first LDS
        // round trip of a step depends on nothing and is issued speculatively at
        // the end of the previous step together with the read of the step's ready
        // word (LDS serves one wave's reads in order, so data read after a ready
        // word that shows the step is the staged data); only when the word shows
        // an older step does the wave wait and read again.  The second round trip
        // reads the dependency values; then the group sum, one ring write and the
        // published stores.
        TA carry = (TA)0;
        int rdy, h, c[J];
        int4 ln;
        TA a[J], rhs, piv;
        auto first_batch = [&](int slot) {
            rdy = __hip_atomic_load(&ready[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            h = shdr[slot];
            ln = slane[slot * 64 + lane];
            rhs = srhs[slot * 64 + lane];
            piv = spiv[slot * 64 + lane];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                c[j] = sc[(slot * J + j) * 64 + lane];
                a[j] = sa[(slot * J + j) * 64 + lane];
            }
        };
        if (T.nsteps > 0) first_batch(0);
        for (int s = 0; s < T.nsteps; ++s) {
            if (rdy < s) {
                if (!lds_wait_ge(&ready[s % Q], s, labort, A.info, false)) break;
                first_batch(s % Q);
            }
            TA acc = (TA)0;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const TA x = Pub<TA>::from(lds_ld<TA>(vals + c[j]));
                const TA prod = a[j] * x;
                acc = acc + prod;
            }
            acc = seg_sum(acc, ln.x & 255, (h >> 16) & 255);
            const int flags = h >> 24;
            if (flags & kTailCarryIn) acc = acc + carry;
            if (!(flags & kTailEmit)) {
                carry = acc;
            } else if (ln.x >> 8) {
                TA v = rhs - acc;
                if (!A.unit_diag) v = v * piv;
                lds_st<TA>(vals + ln.y, bits_of<TA>(v));
                tile_store<TA, FWD>(A, ln.z, ln.w, col, v);
            }
            // the step's buffer is free: every read of it has returned (its values
            // were used above), and LDS takes this write after them
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (lane == 0) __hip_atomic_store(done, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (s + 1 < T.nsteps) first_batch((s + 1) % Q);
        }
        return;
    }
    // Stagers: wave w stages steps w - 1, w - 1 + S, ...  Software pipeline over
    // the wave's steps: the header two steps ahead, the record one ahead, the
    // values it points at for the current step, issued before the wait for the
    // step's buffer
    const TA *dep = FWD ? y : z;
    const int s0 = wave - 1;
    if (s0 >= T.nsteps) return;
    StreamRec<J> cur;
    stream_rec_load<J>(cur, T, T.hdr[s0], lane);
    int4 hd1 = s0 + S < T.nsteps ? T.hdr[s0 + S] : make_int4(0, 0, 0, 0);
    for (int s = s0; s < T.nsteps; s += S) {
        const int slot = s % Q;
        // the values of step s; this lane stages compute lane `lane`, whose row
        // is row k of the step (its lane word), for which it also reads the
        // right-hand side and the pivot
        TA a[J];
        U xo[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            a[j] = cur.p[j] >= 0 ? (TA)load_val(val, cur.p[j]) : (TA)0;
            xo[j] = cur.code[j] >= W ? Pub<TA>::load(dep + (int64_t)(cur.code[j] - W) * cap + col) : (U)0;
        }
        const bool lead = lane < cur.nlanes && ((cur.li >> 16) & 1);
        TA rhs = (TA)0, pv = (TA)1;
        int outr = 0;
        if (lead) {
            if constexpr (FWD) {
                rhs = load_vec<TA>(A.b, A.vec_f32, (int64_t)(A.perm ? cur.lr.z : cur.lr.x) * A.ld + col);
            } else {
                rhs = y[(int64_t)cur.lr.x * cap + col];
                if (!A.unit_diag) pv = (TA)load_val(val, cur.lr.w);
            }
            outr = A.perm ? cur.lr.z : cur.lr.x;
        }
        // the record of step s + S and the header of step s + 2S
        StreamRec<J> nxt;
        nxt.nrows = nxt.nlanes = nxt.nent = 0;
        if (s + S < T.nsteps) stream_rec_load<J>(nxt, T, hd1, lane);
        const int4 hd2 = s + 2 * S < T.nsteps ? T.hdr[s + 2 * S] : make_int4(0, 0, 0, 0);
        // the buffer is free once step s - Q is done
        if (s >= Q && !lds_wait_ge(done, s - Q, labort, A.info, true, true)) break;
        // a dependency published but not yet visible is waited for (it was
        // computed kTailQ or more steps ago)
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (cur.code[j] >= W && xo[j] == Pub<TA>::kPend)
                xo[j] = bits_of<TA>(Pub<TA>::wait(dep + (int64_t)(cur.code[j] - W) * cap + col, A.info, A.poll_sleep));
        // entry j of compute lane `lane` to [slot][j][lane]; padding and lanes
        // beyond the step's lanes read the zero slot with coefficient 0
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int q = slot * E + j * 64 + lane;
            int idx = zero;
            if (cur.code[j] >= W) {
                idx = W + q;
                lds_st<TA>(vals + idx, xo[j]);
            } else if (cur.code[j] >= 0) {
                idx = cur.code[j];
            }
            sc[q] = (uint16_t)idx;
            sa[q] = a[j];
        }
        const int gl = lane < cur.nlanes ? (cur.li >> 8) & 255 : 0;
        slane[slot * 64 + lane] = make_int4(gl | (lead ? 256 : 0), cur.lr.y, cur.lr.x, outr);
        srhs[slot * 64 + lane] = rhs;
        spiv[slot * 64 + lane] = (TA)1 / pv;
        if (lane == 0) {
            shdr[slot] = cur.h;
            __hip_atomic_store(&ready[slot], s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        cur = nxt;
        hd1 = hd2;
    }
}

// ---------------------------------------------------------------------------------
// Lower stage of the numeric factor (Sec. III-B, Even-Rows, Fig. 7): one workgroup
// factors the tail rows in level order, a step (rows of one level) at a time
// ---------------------------------------------------------------------------------
// Wave 0 computes.  Lane t of a row's group holds entry t; for the row's L
// entries e ascending, lane e divides by u_(c_e c_e), the multiplier goes to the
// group, and each later entry whose column lies in U(c_e) subtracts l * u --
// the serial up-looking order, hence the serial bits.  The U values a step needs
// come from the ring of recent rows' U parts in LDS (written by wave 0 itself in
// an earlier step) or, for older rows and rows before the tail, from the factor
// buffer, fetched by a stager into the step's buffer.  Waves 1..15 take steps
// round-robin and stage step s into buffer s % q once step s - q is done.
constexpr int kFStreamStagers = 15;
constexpr int kFStreamBlock = 64 * (1 + kFStreamStagers);
constexpr int kFStreamNone = 0xFFFF;

struct FStreamLds {
    double *vals;        // ring [kFTailRing], then staged values [q][kFTailK][64]
    uint16_t *sidx;      // [q][kFTailK][64] LDS index of each (L entry, lane) U value
    int4 *smeta;         // [q][64]: g | t << 8 | K << 16 | len << 24, factor entry, ring slot, row
    double *sa;          // [q][64] input value
    int32_t *skmax;      // [q]
    int32_t *ready;      // [q]
    int32_t *done;
    int32_t *labort;
};

__device__ __forceinline__ FStreamLds fstream_lds(unsigned char *m, int q) {
    FStreamLds L;
    size_t o = 0;
    L.vals = reinterpret_cast<double *>(m + o);
    o += (size_t)(kFTailRing + q * kFTailK * 64) * 8;
    L.sa = reinterpret_cast<double *>(m + o);
    o += (size_t)q * 64 * 8;
    L.smeta = reinterpret_cast<int4 *>(m + o);
    o += (size_t)q * 64 * 16;
    L.sidx = reinterpret_cast<uint16_t *>(m + o);
    o += (size_t)q * kFTailK * 64 * 2;
    L.skmax = reinterpret_cast<int32_t *>(m + o);
    L.ready = L.skmax + q;
    L.done = L.ready + q;
    L.labort = L.done + 1;
    return L;
}

__host__ __device__ inline size_t fstream_lds_bytes(int q) {
    return (size_t)(kFTailRing + q * kFTailK * 64) * 8 + (size_t)q * 64 * (8 + 16) + (size_t)q * kFTailK * 64 * 2 +
           (size_t)(2 * q + 2) * 4;
}

__global__ __launch_bounds__(kFStreamBlock) void k_factor_stream(FactorArgs A, FactorStreamArgs T) {
    extern __shared__ __align__(16) unsigned char fs_smem[];
    const int q = T.q;
    const FStreamLds L = fstream_lds(fs_smem, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < q; i += kFStreamBlock) L.ready[i] = -1;
    if (threadIdx.x == 0) {
        *L.done = -1;
        *L.labort = 0;
    }
    __syncthreads();
    if (wave == 0) {
        for (int s = 0; s < T.nsteps; ++s) {
            const int slot = s % q;
            if (!lds_wait_ge(&L.ready[slot], s, L.labort, A.info, false)) break;
            const int kmax = L.skmax[slot];
            const int4 m = L.smeta[slot * 64 + lane];
            const int g = m.x & 255, t = (m.x >> 8) & 255, K = (m.x >> 16) & 255, len = (m.x >> 24) & 255;
            const bool act = t < len;
            const int gbase = lane & ~((1 << g) - 1);
            const double a = L.sa[slot * 64 + lane];
            double u[kFTailK];
            uint32_t hasu = 0;   // bit e: entry e of the row meets U(c_e)
#pragma unroll
            for (int e = 0; e < kFTailK; ++e) {
                const int ix = e < kmax ? (int)L.sidx[(slot * kFTailK + e) * 64 + lane] : kFStreamNone;
                u[e] = L.vals[ix != kFStreamNone ? ix : 0];
                if (ix != kFStreamNone) hasu |= 1u << e;
            }
            double v = a;
#pragma unroll
            for (int e = 0; e < kFTailK; ++e) {
                if (e < kmax) {   // uniform: the step's longest L part
                    if (t == e && e < K && act) v = v / u[e];   // (a row with fewer L entries is done)
                    const double l = __shfl(v, gbase + e);
                    if (t > e && hasu >> e & 1) {
                        const double prod = l * u[e];
                        v = v - prod;
                    }
                }
            }
            // the U part to the ring (read by later steps), then the published row
            if (act && t >= K) L.vals[m.z] = v;
            if (act) {
                const uint64_t bits = (v != v) ? kQNaN64 : (uint64_t)__double_as_longlong(v);
                st_pub_u64(reinterpret_cast<uint64_t *>(&A.lu[m.y]), bits);
                const float f = (float)__longlong_as_double((long long)bits);
                if (A.lu32) A.lu32[m.y] = f;
                if (A.lu16) A.lu16[m.y] = to_bf16(f);
                if (A.bval) A.bval[m.y] = a;
            }
            // a zero pivot or a non-finite entry (the checks of the other schedules)
            const uint64_t zp = __ballot(act && t == K && v == 0.0);
            const uint64_t nf = __ballot(act && !isfinite(v));
            if (act && t == 0) {
                const uint64_t gm = (g == 6) ? ~0ull : (((1ull << (1 << g)) - 1ull) << gbase);
                if (zp & gm) atomicMin(&A.info[kInfoBadKey], 2 * m.w);
                else if (nf & gm) atomicMin(&A.info[kInfoBadKey], 2 * m.w + 1);
            }
            // the step's buffer is free: its reads have returned (their values were
            // used above) and LDS takes this write after them
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (lane == 0) __hip_atomic_store(L.done, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        return;
    }
    // stagers
    for (int s = wave - 1; s < T.nsteps; s += kFStreamStagers) {
        const int slot = s % q;
        const int4 hd = T.hdr[s];
        const int k = T.lmap[(size_t)hd.w + lane];
        int4 ra = make_int4(0, 0, 0, 0), rb = make_int4(0, 0, 0, 0);
        if (k != 255) {
            ra = T.rows[2 * (size_t)(hd.x + k)];
            rb = T.rows[2 * (size_t)(hd.x + k) + 1];
        }
        const int len = k != 255 ? (ra.z & 255) : 0, K = (ra.z >> 8) & 255, g = (ra.z >> 16) & 255;
        const int t = k != 255 ? lane - ((ra.z >> 24) & 255) : 64;
        const bool act = t < len;
        const int p = act ? ra.y + t : 0;
        const int pin = act ? A.src[p] : -1;
        const double a = pin >= 0 ? A.a[pin] : 0.0;
        // the sources of this lane's U values, one per L entry e of its row
        int ix[kFTailK];
        double xo[kFTailK];
        int64_t gsrc[kFTailK];
#pragma unroll
        for (int e = 0; e < kFTailK; ++e) {
            ix[e] = kFStreamNone;
            gsrc[e] = -1;
            xo[e] = 0.0;
            if (e < K && act && t >= e) {
                const int j = T.match[(size_t)rb.y + (size_t)e * len + t];
                if (j != 255) {
                    const int src = T.lsrc[rb.x + e];
                    if (src >= 0) ix[e] = src + j;
                    else gsrc[e] = (int64_t)(-src - 1) + j;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < kFTailK; ++e)
            if (gsrc[e] >= 0) xo[e] = __longlong_as_double((long long)ld_acq_u64(reinterpret_cast<const uint64_t *>(A.lu + gsrc[e])));
        // the buffer is free once step s - q is done
        if (s >= q && !lds_wait_ge(L.done, s - q, L.labort, A.info, true, true)) break;
        // a value not yet visible was computed at least q steps ago: wait for it
#pragma unroll
        for (int e = 0; e < kFTailK; ++e)
            if (gsrc[e] >= 0 && (uint64_t)__double_as_longlong(xo[e]) == kPending64)
                xo[e] = __longlong_as_double((long long)wait_u64(reinterpret_cast<const uint64_t *>(A.lu + gsrc[e]),
                                                                 A.info, A.poll_sleep));
#pragma unroll
        for (int e = 0; e < kFTailK; ++e) {
            const int qi = (slot * kFTailK + e) * 64 + lane;
            int idx = ix[e];
            if (gsrc[e] >= 0) {
                idx = kFTailRing + qi;
                L.vals[idx] = xo[e];
            }
            L.sidx[qi] = (uint16_t)idx;
        }
        L.smeta[slot * 64 + lane] = make_int4(g | (act ? t : 255) << 8 | K << 16 | len << 24, p,
                                              act && t >= K ? ra.w + (t - K) : 0, ra.x);
        L.sa[slot * 64 + lane] = a;
        if (lane == 0) {
            L.skmax[slot] = hd.z;
            __hip_atomic_store(&L.ready[slot], s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

}  // namespace

hipError_t launch_factor_stream(const FactorArgs &A, const FactorStreamArgs &T, hipStream_t s) {
    if (T.nsteps <= 0) return hipSuccess;
    if (T.q < 2 || T.q > kFTailQ) return hipErrorInvalidValue;
    const size_t lds = fstream_lds_bytes(T.q);
    if (lds > 163840) return hipErrorInvalidValue;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void *)k_factor_stream, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_factor_stream, dim3(1), dim3(kFStreamBlock), lds, s, A, T);
    return hipGetLastError();
}

namespace {

// ---------------------------------------------------------------------------------
// Tiled factor (ILU(k, tau) at k = k_max on the forward tiles): rows and imported
// U rows in LDS
// ---------------------------------------------------------------------------------
// The block of a tile stages, into LDS, the tile's rows (their input values), the
// per-L-entry data (where U(c) sits in LDS, its ready flag, and each lane's index
// into U(c)), and reserves room for the U parts of its imports, which the poller
// wave copies from the factor buffer as they are published.  A compute wave
// factors one chunk (64/G rows of one local level) at a time, G lanes per row,
// lane t holding entry t: for the L entries in ascending column order, the lane of
// the entry divides by u_cc, the multiplier is broadcast, and every lane whose
// column is in U(c) subtracts l * u_cj -- the serial up-looking algorithm's
// operations in its order (Sec. III, Fig. 1), so the result is bit for bit the
// serial one.  A row then writes its values to LDS, raises its ready flag and
// publishes its values to the factor buffer for other tiles.

// A tiled-factor row (or import) is ready when its ready word holds its pivot
// u_cc instead of the pending pattern; the word is written last, with release
// semantics, so that the U part it guards is in LDS.  Returns the pivot, or a NaN
// after an abort or an expired wait.
__device__ __forceinline__ double lds_wait_pivot(const uint64_t *f, int *lds_abort, int32_t *info) {
    int spins = 0;
    uint64_t t0 = 0;
    for (;;) {
        const uint64_t b = __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (b != kPending64) return __longlong_as_double((long long)b);
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 63) == 0) {
            if (__hip_atomic_load(lds_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                return __longlong_as_double((long long)kQNaN64);
            if (expired(t0)) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(lds_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return __longlong_as_double((long long)kQNaN64);
            }
        }
    }
}

// Poller of the tiled factor: lane l holds imports l, l + 64 of the window (in
// order of first use); each round loads every still-missing U value of a held
// import, copies the published ones into LDS and sets the import's ready word
// to its pivot once its whole U part is there.  The window moves by 64 when its first 64
// imports are complete.  Bounded like every wait.
template <int G>
__device__ void factor_poll(const int4 *imp, int nimp, const double *lu, double *vals, uint64_t *rdy, int nrows,
                            int32_t *info, int sleep0, int *lds_abort) {
    const int lane = threadIdx.x & 63;
    int head = 0, sleep = 0, spins = 0;
    uint64_t t0 = 0;
    uint32_t have[2] = {0u, 0u};   // U values already copied, per held import
    while (head < nimp) {
        bool got = false, left0 = false;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int i = head + 64 * b + lane;
            if (i >= nimp) continue;
            const int4 m = imp[i];
            const uint32_t all = m.y >= 32 ? 0xFFFFFFFFu : ((1u << m.y) - 1u);
            if (have[b] == all) continue;
            // a U part has at most G entries, fetched up to 8 at a time
            constexpr int PJ = G < 8 ? G : 8;
            for (int j0 = 0; j0 < m.y; j0 += PJ) {
                uint64_t raw[PJ];
#pragma unroll
                for (int q = 0; q < PJ; ++q) {
                    const int j = j0 + q;
                    raw[q] = (j < m.y && !(have[b] >> j & 1u))
                                 ? ld_acq_u64(reinterpret_cast<const uint64_t *>(lu + m.x + j))
                                 : kPending64;
                }
#pragma unroll
                for (int q = 0; q < PJ; ++q) {
                    const int j = j0 + q;
                    if (j < m.y && !(have[b] >> j & 1u) && raw[q] != kPending64) {
                        reinterpret_cast<uint64_t *>(vals)[m.z + j] = raw[q];
                        have[b] |= 1u << j;
                        got = true;
                    }
                }
            }
            if (have[b] == all) {
                const uint64_t pv = reinterpret_cast<const uint64_t *>(vals)[m.z];   // u_cc, copied above
                __hip_atomic_store(&rdy[nrows + i], pv, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            else if (b == 0) left0 = true;
        }
        if (!__any(left0)) {
            head += 64;
            have[0] = have[1];
            have[1] = 0u;
            continue;
        }
        sleep = __any(got) ? sleep0 : (sleep * 2 + 1 < kPollMaxSleep ? sleep * 2 + 1 : kPollMaxSleep);
        for (int k = 0; k < sleep; ++k) __builtin_amdgcn_s_sleep(1);
        if ((++spins & 15) == 0) {
            if (aborted(info)) break;
            if (expired(t0)) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    if (head >= nimp) return;
    // aborted: release every waiter of this block
    if (lane == 0) __hip_atomic_store(lds_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int G>
__device__ __forceinline__ void factor_tile(const FactorArgs &A, const FactorTileArgs &T, int tile, unsigned char *fsmem,
                                            int &s_abort) {
    // The tile's header (uniform: scalar loads) and its LDS image: values, ready
    // words, the tables (one blob, copied as is), thresholds, modified-ILU masks.
    const int32_t *th = T.hdr + (size_t)kFactorHdr * tile;
    const int boff = th[kFhBlob], bsz = th[kFhBlobSize], nrows = th[kFhRows], nimp = th[kFhImps];
    const int nl = th[kFhLents], npos = th[kFhPos], vbase = th[kFhVsrc], nvr = th[kFhRowVals];
    const int nvals = th[kFhVals], l0 = th[kFhL0];
    double *vals = reinterpret_cast<double *>(fsmem);
    uint64_t *rdy = reinterpret_cast<uint64_t *>(fsmem + ((nvals * 8 + 15) & ~15));
    unsigned char *blob = reinterpret_cast<unsigned char *>(rdy) + (((nrows + nimp) * 8 + 15) & ~15);
    const int4 *rmeta = reinterpret_cast<const int4 *>(blob);
    const uint32_t *lent = reinterpret_cast<const uint32_t *>(blob + th[kFhLent]);
    int8_t *match = reinterpret_cast<int8_t *>(blob + th[kFhMatch]);
    int4 *imp = reinterpret_cast<int4 *>(blob + th[kFhImp]);
    int16_t *ps = reinterpret_cast<int16_t *>(blob + th[kFhPs]);
    double *tau = reinterpret_cast<double *>(blob + (size_t)bsz * 16);
    uint32_t *cmask = reinterpret_cast<uint32_t *>(tau + (A.use_tau ? nrows : 0));
    const int t = threadIdx.x % G;

    // Staging in two memory round trips: the blob and the rows' value sources are
    // loaded together, then the input values; the tables reach LDS meanwhile.
    constexpr int UB = 4, UV = G <= 16 ? 8 : 4, B = kTileBlock;
    const int4 *gblob = T.blob + boff;
    int4 *lblob = reinterpret_cast<int4 *>(blob);
    // (loads are unconditional, at clamped indices, so that they issue together;
    // a tile has at least one row and one blob unit)
    int vs[UV];
    for (int b0 = 0;; b0 += B * UB) {
        int4 v[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) v[u] = gblob[min(b0 + (int)threadIdx.x + u * B, bsz - 1)];
        if (b0 == 0) {
#pragma unroll
            for (int u = 0; u < UV; ++u) vs[u] = T.vsrc[vbase + min((int)threadIdx.x + u * B, nvr - 1)];
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int i = b0 + threadIdx.x + u * B;
            if (i < bsz) lblob[i] = v[u];
        }
        if (b0 + B * UB >= bsz) break;
    }
    for (int k0 = 0; k0 < nvr; k0 += B * UV) {
        if (k0 > 0) {
#pragma unroll
            for (int u = 0; u < UV; ++u) vs[u] = T.vsrc[vbase + min(k0 + (int)threadIdx.x + u * B, nvr - 1)];
        }
        double a[UV];
#pragma unroll
        for (int u = 0; u < UV; ++u) a[u] = A.a[max(vs[u], 0)];
#pragma unroll
        for (int u = 0; u < UV; ++u) {
            const int k = k0 + threadIdx.x + u * B;
            if (k < nvr) vals[k] = vs[u] >= 0 ? a[u] : 0.0;   // fill entries start at 0
        }
    }
    for (int i = threadIdx.x; i < nrows + nimp; i += B) rdy[i] = kPending64;
    if (A.use_tau || A.milu) {
        __syncthreads();
        // the rows' drop thresholds and the modified form's masks, so that the
        // compute waves issue no global load
        if (A.use_tau) {
            for (int i = threadIdx.x; i < nrows; i += B) {
                const int mx = rmeta[i].x;
                tau[i] = A.row_tau[mx < 0 ? ~mx : mx];
            }
        }
        if (A.milu) lds_copy<kStageCopy>(cmask, T.cmask + l0, nl);
    }
    // (imported U parts are read only after their ready word: the poller sets it
    // once it has copied the whole part)
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int gi = (threadIdx.x & 63) / G;
    if (wave == kTileComputeWaves) {
        factor_poll<G>(imp, nimp, A.lu, vals, rdy, nrows, A.info, A.poll_sleep, &s_abort);
        return;
    }
    // Every staging load has landed.  Saying so keeps the compiler from waiting
    // on the stores of earlier rows inside the loop, which has no global load.
    __builtin_amdgcn_s_waitcnt(0);
    constexpr int UNIT = 64 / G;
    for (int c0 = wave * UNIT; c0 < npos; c0 += kTileComputeWaves * UNIT) {
        const int sl = ps[c0 + gi];
        if (sl < 0) continue;
        const int4 m = rmeta[sl];
        const int2 o = make_int2(m.z & 0xFFFF, m.w);
        const int len = (m.z >> 16) & 0xFF, K = (m.z >> 24) & 0xFF;
        const bool flat = m.x < 0;             // L entries independent of one another
        const int row = flat ? ~m.x : m.x;
        const bool act = t < len;
        const double tr = A.use_tau ? tau[sl] : 0.0;
        double v = act ? vals[o.x + t] : 0.0;
        const double vin = v;                  // the input value (the spmv operand, stored below)
        double before = 0.0;                   // an L entry's value before its division
        int dropped = 0;
        if (flat && !A.milu && K > 0) {
            // Independent L entries: lane t < K waits for its own dependency and
            // divides; the multipliers then go to the U lanes four at a time, the
            // U(c_e) values they meet read in one LDS round (positions read before
            // the wait, every load unconditional so that none waits on another)
            // and subtracted in ascending e as the serial loop does.
            int uix[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int li = o.y + (q < K ? q : K - 1);
                const int j = match[li * G + t], dl = (int)(lent[li] & 0xFFFFu);
                uix[q] = (q < K && j > 0) ? dl + j : -1;
            }
            const int myrdy = (int)(lent[o.y + (t < K ? t : K - 1)] >> 16);
            if (t < K) {
                const double piv = lds_wait_pivot(&rdy[myrdy], &s_abort, A.info);
                v = v / piv;
                if (A.use_tau && fabs(v) < tr) dropped = 1;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const uint64_t dm = A.use_tau ? group_bits<G>(__ballot(dropped != 0), gi) : 0ull;
            for (int e0 = 0;;) {
                double u[4], l[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = vals[uix[q] >= 0 ? uix[q] : 0];
#pragma unroll
                for (int q = 0; q < 4; ++q) l[q] = __shfl(v, (e0 + q) & (G - 1), G);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool use = uix[q] >= 0 && !(dm >> (e0 + q) & 1ull) &&
                                     (uint64_t)__double_as_longlong(u[q]) != kDropped64;
                    const double prod = l[q] * u[q];
                    const double nv = v - prod;
                    v = use ? nv : v;
                }
                e0 += 4;
                if (!__any(e0 < K)) break;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = e0 + q;
                    const int li = o.y + (e < K ? e : K - 1);
                    const int j = match[li * G + t], dl = (int)(lent[li] & 0xFFFFu);
                    uix[q] = (e < K && j > 0) ? dl + j : -1;
                }
            }
        } else {
        if (flat) {
            // every multiplier at once: lane t < K waits for its own dependency and
            // divides; the updates below then only reach U entries
            if (t < K) {
                const double piv = lds_wait_pivot(&rdy[lent[o.y + t] >> 16], &s_abort, A.info);
                before = v;
                v = v / piv;
                if (A.use_tau && fabs(v) < tr) dropped = 1;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        for (int e = 0; e < K; ++e) {
            const int li = o.y + e;
            const int loc = (int)(lent[li] & 0xFFFFu);
            if (!flat) {
                const double piv = lds_wait_pivot(&rdy[lent[li] >> 16], &s_abort, A.info);
                if (t == e) {
                    before = v;
                    v = v / piv;
                    if (A.use_tau && fabs(v) < tr) dropped = 1;
                }
            }
            const double l = __shfl(v, e, G);
            if (A.use_tau && __shfl(dropped, e, G)) {
                // a dropped multiplier updates nothing; the modified form gives its
                // value before the division back to the diagonal
                const double bv = __shfl(before, e, G);
                if (A.milu && t == K) v = v + bv;
                continue;
            }
            if (A.milu && t == K) {
                // modified ILU: the diagonal takes its own update and every update
                // whose target row r does not hold, in U(c)'s column order
                uint32_t mk = cmask[li];
                while (mk) {
                    const int jj = __builtin_ctz(mk);
                    mk &= mk - 1;
                    const double u = vals[loc + jj];
                    if ((uint64_t)__double_as_longlong(u) == kDropped64) continue;
                    const double lost = l * u;
                    v = v - lost;
                }
            } else {
                const int j = match[li * G + t];
                if (j > 0) {
                    const double u = vals[loc + j];
                    if ((uint64_t)__double_as_longlong(u) != kDropped64) {
                        const double prod = l * u;
                        v = v - prod;
                    }
                }
            }
        }
        }
        // U entries below the threshold at the end of the row (the modified form adds
        // them to the diagonal in column order), then the checks of the sync-free factor
        if (A.use_tau) {
            if (act && t > K && fabs(v) < tr) dropped = 1;
            if (A.milu) {
                for (int j = K + 1; j < G; ++j) {
                    const double dv = __shfl(v, j, G);
                    if (__shfl(dropped, j, G) && t == K) v = v + dv;
                }
            }
        }
        // The row in LDS, then its ready word (its pivot) for the rows of this tile;
        // the global copies and the checks of the sync-free factor come after, off
        // the path from one level to the next.
        const uint64_t bits = dropped ? kDropped64 : (v != v) ? kQNaN64 : (uint64_t)__double_as_longlong(v);
        if (act) reinterpret_cast<uint64_t *>(vals)[o.x + t] = bits;
        if (t == K) __hip_atomic_store(&rdy[sl], bits, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (act) {
            st_pub_u64(reinterpret_cast<uint64_t *>(&A.lu[m.y + t]), bits);
            // the storage copies of the final value (a dropped entry is 0): the same
            // roundings as the cast kernels, written while the row is at hand
            const float f = dropped ? 0.0f : (float)__longlong_as_double((long long)bits);
            if (A.lu32) A.lu32[m.y + t] = f;
            if (A.lu16) A.lu16[m.y + t] = to_bf16(f);
            // the spmv operand (same pattern as the factor): A's value in the
            // permuted copy
            if (A.bval) A.bval[m.y + t] = vin;
        }
        // a zero pivot (lane K) or a non-finite kept entry, by ballot
        const uint64_t zpm = group_bits<G>(__ballot(t == K && v == 0.0), gi);
        const bool nonfinite = act && !dropped && !isfinite(v);
        const uint64_t nfm = group_bits<G>(__ballot(nonfinite), gi);
        if (t == 0) {
            if (zpm) atomicMin(&A.info[kInfoBadKey], 2 * row);
            else if (nfm) atomicMin(&A.info[kInfoBadKey], 2 * row + 1);
        }
    }
}

// Persistent blocks: each claims tiles in start order until none is left, so that
// a finished tile's slot goes to the next tile without a new workgroup dispatch.
// A tile waits only on tiles claimed before it, which are held by running blocks.
template <int G>
__global__ __launch_bounds__(kTileBlock, 5) void k_factor_tiled(FactorArgs A, FactorTileArgs T) {
    extern __shared__ __align__(16) unsigned char fsmem[];
    __shared__ int s_tile, s_abort;
    if (threadIdx.x == 0) s_abort = 0;
    for (;;) {
        if (threadIdx.x == 0) s_tile = __hip_atomic_fetch_add(T.counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int tile = s_tile;
        if (tile >= T.ntiles || s_abort) return;
        factor_tile<G>(A, T, tile, fsmem, s_abort);
        // every wave is done with the tile's LDS image before the next one is staged
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// spmv y = alpha A x + beta y (paper Sec. I-II), one row per group
// ---------------------------------------------------------------------------------
template <int G, bool PERM>
__global__ __launch_bounds__(kBlock) void k_spmv(SpmvArgs A) {
    const int r = (blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int t = threadIdx.x % G;
    if (r >= A.n) return;
    const int rs = A.rp[r], re = A.rp[r + 1];
    if (re - rs > A.heavy_min) return;   // a long row: the one-wave pass takes it
    const int yr = PERM ? A.perm[r] : r;
    for (int s = 0; s < A.nrhs; ++s) {
        double acc = 0.0;
        for (int p = rs + t; p < re; p += G) {
            const int c = PERM ? A.perm[A.ci[p]] : A.ci[p];
            const double prod = A.val[p] * A.x[(int64_t)c * A.ld + s];
            acc = acc + prod;
        }
        acc = group_sum<G>(acc);
        if (t == 0) {
            double out = A.alpha * acc;
            if (A.beta != 0.0) {
                const double by = A.beta * A.y[(int64_t)yr * A.ld + s];
                out = out + by;
            }
            A.y[(int64_t)yr * A.ld + s] = out;
        }
    }
}

// One row per lane, for short rows: the lane loads its row's column indices and
// values eight at a time, all at once, then the x entries they name, so every load
// of a row is in flight together and a wave covers 64 rows; entries are added in
// column-position order.
template <bool PERM>
__global__ __launch_bounds__(kBlock) void k_spmv_lane(SpmvArgs A) {
    constexpr int K = 8;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= A.n) return;
    const int rs = A.rp[r], re = A.rp[r + 1];
    if (re - rs > A.heavy_min) return;   // a long row: the one-wave pass takes it
    const int yr = PERM ? A.perm[r] : r;
    for (int s = 0; s < A.nrhs; ++s) {
        double acc = 0.0;
        for (int b = rs; b < re; b += K) {
            int c[K];
            double v[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (b + j < re) {
                    c[j] = A.ci[b + j];
                    v[j] = A.val[b + j];
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (b + j < re) {
                    const int cc = PERM ? A.perm[c[j]] : c[j];
                    const double prod = v[j] * A.x[(int64_t)cc * A.ld + s];
                    acc = acc + prod;
                }
            }
        }
        double out = A.alpha * acc;
        if (A.beta != 0.0) {
            const double by = A.beta * A.y[(int64_t)yr * A.ld + s];
            out = out + by;
        }
        A.y[(int64_t)yr * A.ld + s] = out;
    }
}

// ---------------------------------------------------------------------------------
// Adjoint outer products restricted to the factor pattern, one row per 8 lanes
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_outer(int32_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ W, const double *__restrict__ Bp,
                                                  const double *__restrict__ x, const double *__restrict__ y,
                                                  double *__restrict__ glu, int32_t nrhs, int64_t ld) {
    constexpr int G = 8;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int t = threadIdx.x % G;
    if (i >= n) return;
    for (int p = rp[i] + t; p < rp[i + 1]; p += G) {
        const int j = ci[p];
        double acc = 0.0;
        for (int s = 0; s < nrhs; ++s) {
            double prod;
            if (j >= i) prod = W[(int64_t)i * ld + s] * x[(int64_t)perm[j] * ld + s];
            else prod = Bp[(int64_t)i * ld + s] * y[(int64_t)j * ld + s];
            acc = acc + prod;
        }
        glu[p] = -acc;
    }
}

int grid_for(int64_t work_items, int per_block) {
    int64_t g = (work_items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 30)) g = 1 << 30;
    return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------
hipError_t launch_fill_u64(uint64_t *p, uint64_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int g = grid_for(count, kBlock);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(kBlock), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_zero_counters(int32_t *counters, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, counters);
    return hipGetLastError();
}

hipError_t launch_solve_guard(int32_t *info, uint64_t *y64, uint64_t *z64, int64_t n64, uint32_t *y32, uint32_t *z32,
                              int64_t n32, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_guard, dim3(256), dim3(kBlock), 0, s, info, y64, z64, y64 ? n64 : 0, y32, z32,
                       y32 ? n32 : 0);
    return hipGetLastError();
}

hipError_t launch_factor_prologue(int32_t *info, uint64_t *y64, uint64_t *z64, int64_t n64, uint32_t *y32,
                                  uint32_t *z32, int64_t n32, int32_t *counters, hipStream_t s) {
    hipLaunchKernelGGL(k_factor_prologue, dim3(256), dim3(kBlock), 0, s, info, y64, z64, y64 ? n64 : 0, y32, z32,
                       y32 ? n32 : 0, counters);
    return hipGetLastError();
}

hipError_t launch_arm_ranges(uint64_t *lu, const int2 *ranges, int32_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_arm_ranges, dim3(grid_for(count, kBlock)), dim3(kBlock), 0, s, lu, ranges, count);
    return hipGetLastError();
}

hipError_t launch_raise_abort(int32_t *info, hipStream_t s) {
    hipLaunchKernelGGL(k_raise_abort, dim3(1), dim3(64), 0, s, info);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int g = grid_for(count, kBlock);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(kBlock), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_row_tau(int32_t n, const int32_t *in_rp, const double *a, const int32_t *perm, double tau,
                          double *row_tau, hipStream_t s) {
    hipLaunchKernelGGL(k_row_tau, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, in_rp, a, perm, tau, row_tau);
    return hipGetLastError();
}

hipError_t launch_gather(int64_t m, const int32_t *src, const double *a, double *out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    int g = grid_for(m, kBlock);
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(kBlock), 0, s, m, src, a, out);
    return hipGetLastError();
}

hipError_t launch_cast_f32(int64_t m, const double *x, float *y, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    int g = grid_for(m, kBlock);
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_cast_f32, dim3(g), dim3(kBlock), 0, s, m, x, y);
    return hipGetLastError();
}

hipError_t launch_cast_bf16(int64_t m, const double *x, uint16_t *y, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    int g = grid_for(m, kBlock);
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_cast_bf16, dim3(g), dim3(kBlock), 0, s, m, x, y);
    return hipGetLastError();
}

hipError_t launch_factor_fixup(int64_t nnz, double *lu, const int8_t *flev, int32_t k, int32_t use_flev,
                               int8_t *stat, int32_t *info, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    int g = grid_for(nnz, kBlock);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_factor_fixup, dim3(g), dim3(kBlock), 0, s, nnz, lu, flev, k, use_flev, stat, info);
    return hipGetLastError();
}

hipError_t launch_outer(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *perm, const double *W,
                        const double *Bp, const double *x, const double *y, double *glu, int32_t nrhs, int64_t ld,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_outer, dim3(grid_for((int64_t)n * 8, kBlock)), dim3(kBlock), 0, s, n, rp, ci, perm, W, Bp, x,
                       y, glu, nrhs, ld);
    return hipGetLastError();
}

template <int G>
static size_t lds_bytes_g(int tcap) {
    if (tcap <= 0) return 0;
    constexpr int ngroups = kBlock / G;
    return (size_t)ngroups * tcap * 8 + (size_t)ngroups * (tcap + 2 * G) * 4;
}

size_t factor_lds_bytes(int lanes, int tcap) {
    size_t b = 0;
    switch (lanes) {
        case 4: b = lds_bytes_g<4>(tcap); break;
        case 8: b = lds_bytes_g<8>(tcap); break;
        case 16: b = lds_bytes_g<16>(tcap); break;
        case 32: b = lds_bytes_g<32>(tcap); break;
        default: b = lds_bytes_g<64>(tcap); break;
    }
    return b <= 48 * 1024 ? b : 0;
}

template <int G, int MAXL>
static hipError_t factor_launch(const FactorArgs &A, bool syncfree, int grid, size_t lds, hipStream_t s) {
    if (syncfree) {
        hipLaunchKernelGGL((k_factor_syncfree<G, MAXL>), dim3(grid), dim3(kBlock), lds, s, A);
    } else {
        int64_t rows = A.row_end - A.row_begin;
        if (rows <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_factor_level<G, MAXL>), dim3(grid_for(rows * G, kBlock)), dim3(kBlock), lds, s, A);
    }
    return hipGetLastError();
}

template <int G>
static hipError_t factor_dispatch(const FactorArgs &A, bool syncfree, int grid, hipStream_t s) {
    const size_t lds = A.tcap > 0 ? lds_bytes_g<G>(A.tcap) : 0;
    const int ml = A.max_lower;
    if (!lds || ml > 32) return factor_launch<G, 0>(A, syncfree, grid, 0, s);
    if (ml <= 4) return factor_launch<G, 4>(A, syncfree, grid, lds, s);
    if constexpr (G >= 8) if (ml <= 8) return factor_launch<G, 8>(A, syncfree, grid, lds, s);
    if constexpr (G >= 16) if (ml <= 16) return factor_launch<G, 16>(A, syncfree, grid, lds, s);
    if constexpr (G >= 32) return factor_launch<G, 32>(A, syncfree, grid, lds, s);
    return factor_launch<G, 0>(A, syncfree, grid, 0, s);
}

hipError_t launch_factor(const FactorArgs &A, int lanes, bool syncfree, int grid, hipStream_t s) {
    switch (lanes) {
        case 4: return factor_dispatch<4>(A, syncfree, grid, s);
        case 8: return factor_dispatch<8>(A, syncfree, grid, s);
        case 16: return factor_dispatch<16>(A, syncfree, grid, s);
        case 32: return factor_dispatch<32>(A, syncfree, grid, s);
        case 64: return factor_dispatch<64>(A, syncfree, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_factor_long(const FactorArgs &A, bool syncfree, int grid, hipStream_t s) {
    const size_t lds = (size_t)(kBlock / 64) * A.lcap * 8;
    if (A.lcap <= 0 || lds > (size_t)kFactorTileLdsMax) return hipErrorInvalidValue;
    const void *fn = syncfree ? (const void *)k_factor_long<true> : (const void *)k_factor_long<false>;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (syncfree) {
        hipLaunchKernelGGL((k_factor_long<true>), dim3(grid), dim3(kBlock), lds, s, A);
    } else {
        const int64_t rows = A.row_end - A.row_begin;
        if (rows <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_factor_long<false>), dim3(grid_for(rows * 64, kBlock)), dim3(kBlock), lds, s, A);
    }
    return hipGetLastError();
}

hipError_t probe_xcc_ids(int blocks, int32_t *host_ids) {
    int32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(int32_t) * blocks);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_probe_xcc, dim3(blocks), dim3(64), 0, 0, d);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(host_ids, d, sizeof(int32_t) * blocks, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e;
}

template <int G, int NR, typename TV, typename TA>
static hipError_t solve_dispatch3(const SolveArgs &A, bool fwd, bool syncfree, int grid, hipStream_t s) {
    if (syncfree) {
        if (fwd) hipLaunchKernelGGL((k_solve_syncfree<G, NR, TV, TA, true>), dim3(grid), dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_solve_syncfree<G, NR, TV, TA, false>), dim3(grid), dim3(kBlock), 0, s, A);
    } else {
        int64_t rows = A.row_end - A.row_begin;
        if (rows <= 0) return hipSuccess;
        dim3 g(grid_for(rows * G, kBlock));
        if (fwd) hipLaunchKernelGGL((k_solve_level<G, NR, TV, TA, true>), g, dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_solve_level<G, NR, TV, TA, false>), g, dim3(kBlock), 0, s, A);
    }
    return hipGetLastError();
}

template <int G, typename TV, typename TA>
static hipError_t solve_dispatch2(const SolveArgs &A, bool fwd, bool syncfree, int grid, hipStream_t s) {
    if (A.nrhs == 1) return solve_dispatch3<G, 1, TV, TA>(A, fwd, syncfree, grid, s);
    if (A.nrhs <= 4) return solve_dispatch3<G, 4, TV, TA>(A, fwd, syncfree, grid, s);
    return solve_dispatch3<G, 16, TV, TA>(A, fwd, syncfree, grid, s);
}

template <int G>
static hipError_t solve_dispatch1(const SolveArgs &A, bool fwd, int prec, bool syncfree, int grid, hipStream_t s) {
    switch (prec) {
        case 0: return solve_dispatch2<G, double, double>(A, fwd, syncfree, grid, s);
        case 1: return solve_dispatch2<G, float, float>(A, fwd, syncfree, grid, s);
        case 2: return solve_dispatch2<G, uint16_t, float>(A, fwd, syncfree, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve(const SolveArgs &A, bool forward, int prec, int vec, int lanes, bool syncfree, int grid,
                        hipStream_t s) {
    SolveArgs B = A;
    B.vec_f32 = vec;
    switch (lanes) {
        case 4: return solve_dispatch1<4>(B, forward, prec, syncfree, grid, s);
        case 8: return solve_dispatch1<8>(B, forward, prec, syncfree, grid, s);
        case 16: return solve_dispatch1<16>(B, forward, prec, syncfree, grid, s);
        case 32: return solve_dispatch1<32>(B, forward, prec, syncfree, grid, s);
        case 64: return solve_dispatch1<64>(B, forward, prec, syncfree, grid, s);
        default: return hipErrorInvalidValue;
    }
}

static size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

// LDS carve-up of a tiled launch: value slots (+1 zero slot), right-hand sides,
// pivots, packed entry values, packed entry slots, row ids, position -> slot map
static size_t tile_layout(const TileArgs &T, int nr, int acc, TileArgs *out) {
    size_t o = align8((size_t)(T.max_slots + 1) * nr * acc);
    const size_t rhs = o;
    o = align8(o + (size_t)T.max_rows * nr * acc);
    const size_t pv = o;
    o = align8(o + (size_t)T.max_rows * acc);
    const size_t evl = o;
    o = align8(o + (size_t)T.max_rows * T.kmax * acc);
    const size_t esl = o;
    o = align8(o + (size_t)T.max_rows * T.kmax * 2);
    const size_t rid = o;
    o = align8(o + (size_t)T.max_rows * 4);
    const size_t psl = o;
    o = align8(o + (size_t)T.max_pos * 2);
    const size_t imp = o;
    o = align8(o + (size_t)T.max_imps * 4);   // the import list of the tile with the most imports
    const size_t orw = o;
    o = align8(o + (size_t)T.max_rows * 4);
    if (out) {
        out->off_imp = (int32_t)imp;
        out->off_orow = (int32_t)orw;
        out->off_rhs = (int32_t)rhs;
        out->off_piv = (int32_t)pv;
        out->off_eval = (int32_t)evl;
        out->off_eslot = (int32_t)esl;
        out->off_rowid = (int32_t)rid;
        out->off_pslot = (int32_t)psl;
        out->lds_bytes = (int32_t)o;
    }
    return o;
}

size_t tile_lds_bytes(int max_rows, int max_slots, int max_pos, int max_imps, int kmax, int nr, int acc_bytes) {
    TileArgs T{};
    T.max_rows = max_rows;
    T.max_slots = max_slots;
    T.max_pos = max_pos;
    T.max_imps = max_imps;
    T.kmax = kmax;
    return tile_layout(T, nr, acc_bytes, nullptr);
}

template <int G, int J, int NR, typename TV, typename TA>
static hipError_t tiled_launch(const SolveArgs &A, const TileArgs &T0, bool fwd, hipStream_t s) {
    TileArgs T = T0;
    size_t lds = tile_layout(T, NR, sizeof(TA), &T);
    // a cap on resident tiles per CU is an LDS request that leaves room for no more
    if (T.blocks_per_cu > 0 && lds <= (size_t)kTileLdsMax) {
        const size_t floor_bytes = (size_t)kTileLdsMax / (size_t)(T.blocks_per_cu + 1) + 1024;
        if (lds < floor_bytes) lds = std::min(floor_bytes, (size_t)kTileLdsMax / (size_t)T.blocks_per_cu);
    }
    // a tile may take the whole LDS of a CU (opt-in above 64 KB): grid tiles stay
    // far below (three blocks per CU), import-heavy tiles trade blocks for fewer
    // crossings
    const size_t cap = (size_t)kTileLdsMax;
    if (lds > cap || T.max_slots + 1 > 65535 || T.max_pos > 32767) return hipErrorInvalidValue;
    if (T.ntiles <= 0) return hipSuccess;
    if (lds > 65536) {
        const void *fn = fwd ? (const void *)k_solve_tiled<G, J, NR, TV, TA, true>
                             : (const void *)k_solve_tiled<G, J, NR, TV, TA, false>;
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (fwd)
        hipLaunchKernelGGL((k_solve_tiled<G, J, NR, TV, TA, true>), dim3(T.ntiles), dim3(solve_block<TA>()), lds, s, A, T);
    else
        hipLaunchKernelGGL((k_solve_tiled<G, J, NR, TV, TA, false>), dim3(T.ntiles), dim3(solve_block<TA>()), lds, s, A, T);
    return hipGetLastError();
}

// lanes per row from the tiling's chunk size; right-hand sides per pass: 4 when
// that blocking fits LDS, else 1
template <int NR, typename TV, typename TA>
static hipError_t tiled_lanes(const SolveArgs &A, const TileArgs &T, bool fwd, hipStream_t s) {
    if (T.unit == 64) {
        if (T.kmax > kTileShortRow) return hipErrorInvalidValue;
        return tiled_launch<1, kTileShortRow, NR, TV, TA>(A, T, fwd, s);
    }
    if (T.unit == 16) {
        // entries per lane: as few as the tiling's longest row needs
        if (T.kmax <= 4) return tiled_launch<4, 1, NR, TV, TA>(A, T, fwd, s);
        if (T.kmax <= 8) return tiled_launch<4, 2, NR, TV, TA>(A, T, fwd, s);
        if (T.kmax > 4 * kTileLongJ) return hipErrorInvalidValue;
        return tiled_launch<4, kTileLongJ, NR, TV, TA>(A, T, fwd, s);
    }
    return hipErrorInvalidValue;
}

template <typename TV, typename TA>
static hipError_t tiled_dispatch(const SolveArgs &A, const TileArgs &T, bool fwd, hipStream_t s) {
    // several right-hand sides per pass (up to the whole LDS of a CU) only for tiles
    // with few imports: the one poller wave walks every import's right-hand sides
    // in turn, so import-heavy tiles do better with single-right-hand-side passes
    const size_t l4 = tile_layout(T, 4, sizeof(TA), nullptr);
    const bool few_imports = T.max_slots <= 2 * T.max_rows;
    if (A.nrhs > 1 && few_imports && l4 <= (size_t)kTileLdsMax) return tiled_lanes<4, TV, TA>(A, T, fwd, s);
    return tiled_lanes<1, TV, TA>(A, T, fwd, s);
}

// LDS carve-up of a stream launch
static size_t stream_layout(StreamArgs *T, int acc_bytes) {
    constexpr int Q = kTailQ, E = kStreamEnt;
    size_t o = 0;
    T->off_vals = 0;
    o = align8((size_t)(kTailW + Q * E + 1) * acc_bytes);
    T->off_a = (int32_t)o;
    o = align8(o + (size_t)Q * E * acc_bytes);
    T->off_c = (int32_t)o;
    o = align8(o + (size_t)Q * E * 2);
    o = (o + 15) & ~(size_t)15;
    T->off_lane = (int32_t)o;
    o = align8(o + (size_t)Q * 64 * 16);
    T->off_rhs = (int32_t)o;
    o = align8(o + (size_t)Q * 64 * acc_bytes);
    T->off_piv = (int32_t)o;
    o = align8(o + (size_t)Q * 64 * acc_bytes);
    T->off_hdr = (int32_t)o;
    o = align8(o + (size_t)Q * 4);
    T->off_sync = (int32_t)o;
    o = align8(o + (size_t)(Q + 2) * 4);
    T->lds_bytes = (int32_t)o;
    return o;
}

template <typename TV, typename TA>
static hipError_t stream_launch(const SolveArgs &A, const StreamArgs &T0, bool fwd, hipStream_t s) {
    StreamArgs T = T0;
    const size_t lds = stream_layout(&T, sizeof(TA));
    if (lds > (size_t)kTileLdsMax) return hipErrorInvalidValue;
    if (T.nsteps <= 0 || A.nrhs <= 0) return hipSuccess;
    const void *fn = fwd ? (const void *)k_solve_stream<TV, TA, true> : (const void *)k_solve_stream<TV, TA, false>;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (fwd)
        hipLaunchKernelGGL((k_solve_stream<TV, TA, true>), dim3(A.nrhs), dim3(kStreamBlock), lds, s, A, T);
    else
        hipLaunchKernelGGL((k_solve_stream<TV, TA, false>), dim3(A.nrhs), dim3(kStreamBlock), lds, s, A, T);
    return hipGetLastError();
}

template <int G>
static hipError_t factor_tiled_launch(const FactorArgs &A, const FactorTileArgs &T, hipStream_t s) {
    const size_t lds = (size_t)T.lds_bytes;
    if (lds > (size_t)kFactorTileLdsMax) return hipErrorInvalidValue;
    if (T.ntiles <= 0) return hipSuccess;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void *)k_factor_tiled<G>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // as many blocks as fit the device at once (persistent)
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_factor_tiled<G>, kTileBlock, lds);
    if (e != hipSuccess) return e;
    const int grid = std::max(1, std::min(T.ntiles, cus * std::max(per_cu, 1)));
    hipLaunchKernelGGL((k_factor_tiled<G>), dim3(grid), dim3(kTileBlock), lds, s, A, T);
    return hipGetLastError();
}

hipError_t launch_factor_tiled(const FactorArgs &A, const FactorTileArgs &T, int lanes, hipStream_t s) {
    switch (lanes) {
        case 8: return factor_tiled_launch<8>(A, T, s);
        case 16: return factor_tiled_launch<16>(A, T, s);
        case 32: return factor_tiled_launch<32>(A, T, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve_tiled(const SolveArgs &A, const TileArgs &T, bool forward, int prec, int vec,
                              hipStream_t s) {
    SolveArgs B = A;
    B.vec_f32 = vec;
    switch (prec) {
        case 0: return tiled_dispatch<double, double>(B, T, forward, s);
        case 1: return tiled_dispatch<float, float>(B, T, forward, s);
        case 2: return tiled_dispatch<uint16_t, float>(B, T, forward, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve_stream(const SolveArgs &A, const StreamArgs &T, bool forward, int prec, int vec,
                               hipStream_t s) {
    SolveArgs B = A;
    B.vec_f32 = vec;
    switch (prec) {
        case 0: return stream_launch<double, double>(B, T, forward, s);
        case 1: return stream_launch<float, float>(B, T, forward, s);
        case 2: return stream_launch<uint16_t, float>(B, T, forward, s);
        default: return hipErrorInvalidValue;
    }
}

template <int G>
static hipError_t spmv_dispatch(const SpmvArgs &A, hipStream_t s) {
    dim3 g(grid_for((int64_t)A.n * G, kBlock));
    if (A.perm) hipLaunchKernelGGL((k_spmv<G, true>), g, dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL((k_spmv<G, false>), g, dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

// Long rows of the spmv: one wave per listed row, lanes striding over its entries,
// the wave's partial sums added by the butterfly.
template <bool PERM>
__global__ __launch_bounds__(kBlock) void k_spmv_heavy(SpmvArgs A) {
    const int w = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= A.nheavy) return;
    const int r = A.heavy[w];
    const int rs = A.rp[r], re = A.rp[r + 1];
    const int yr = PERM ? A.perm[r] : r;
    for (int s = 0; s < A.nrhs; ++s) {
        double acc = 0.0;
        for (int p = rs + lane; p < re; p += 64) {
            const int c = PERM ? A.perm[A.ci[p]] : A.ci[p];
            const double prod = A.val[p] * A.x[(int64_t)c * A.ld + s];
            acc = acc + prod;
        }
        acc = group_sum<64>(acc);
        if (lane == 0) {
            double out = A.alpha * acc;
            if (A.beta != 0.0) {
                const double by = A.beta * A.y[(int64_t)yr * A.ld + s];
                out = out + by;
            }
            A.y[(int64_t)yr * A.ld + s] = out;
        }
    }
}

// nnz-balanced spmv (one right-hand side; CSR5-like partition of the entries,
// Sec. II): each lane sums its 16 consecutive entries row segment by row segment
// and writes the rows that start and end among them; a segmented scan over the
// wave's lanes adds up the segments that cross lanes, and the lane (or the end of
// the wave) that closes a segment writes it when it started in this wave.  The
// pieces of rows that reach over a wave boundary go to nz_part (the closing piece
// of the wave's first row, the open piece of its last row) for k_spmv_nz_span.
// Every sum is taken in a fixed order, so the result does not vary between runs.
template <bool PERM>
__global__ __launch_bounds__(kBlock) void k_spmv_nz(SpmvArgs A) {
    const int w = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= A.nz_waves) return;
    const int nnz = A.rp[A.n];
    const int f = w * kNzWave + lane * kNzLane;
    const uint32_t bits = A.nz_bits[(size_t)w * 64 + lane];
    const int cnt = __popc(bits);
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
        const int o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
    }
    const int b0 = __shfl(bits, 0) & 1;
    // the row of the lane's first entry
    const int rf = A.nz_wrow[w] + (inc - cnt) - b0 + (int)(bits & 1);
    auto put = [&](int row, double sum) {
        const int yr = PERM ? A.perm[row] : row;
        double out = A.alpha * sum;
        if (A.beta != 0.0) {
            const double by = A.beta * A.y[yr];
            out = out + by;
        }
        A.y[yr] = out;
    };
    // every load of the lane's entries first (at clamped indices, so that they all
    // issue before any result is needed), then the sums
    double av[kNzLane], xv[kNzLane];
    int cv[kNzLane];
    if (f + kNzLane <= nnz) {
        // 16-byte loads of the lane's 128 bytes of values and 64 bytes of columns
        const double2 *vp = reinterpret_cast<const double2 *>(A.val + f);
        const int4 *cp = reinterpret_cast<const int4 *>(A.ci + f);
#pragma unroll
        for (int i = 0; i < kNzLane / 2; ++i) {
            const double2 v = vp[i];
            av[2 * i] = v.x;
            av[2 * i + 1] = v.y;
        }
#pragma unroll
        for (int i = 0; i < kNzLane / 4; ++i) {
            const int4 c = cp[i];
            cv[4 * i] = c.x;
            cv[4 * i + 1] = c.y;
            cv[4 * i + 2] = c.z;
            cv[4 * i + 3] = c.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kNzLane; ++i) {
            const int p = min(f + i, nnz - 1);
            av[i] = A.val[p];
            cv[i] = A.ci[p];
        }
    }
    if constexpr (PERM) {
#pragma unroll
        for (int i = 0; i < kNzLane; ++i) cv[i] = A.perm[cv[i]];
    }
#pragma unroll
    for (int i = 0; i < kNzLane; ++i) xv[i] = A.x[cv[i]];
    int r = rf;
    double cur = 0.0, head = 0.0;
    bool started = bits & 1;
#pragma unroll
    for (int i = 0; i < kNzLane; ++i) {
        if (f + i < nnz) {
            if (i > 0 && (bits >> i & 1)) {
                if (!started) {
                    head = cur;
                    started = true;
                } else {
                    put(r, cur);   // a row that starts and ends in this lane
                }
                cur = 0.0;
                ++r;
            }
            const double prod = av[i] * xv[i];
            cur = cur + prod;
        }
    }
    // segmented inclusive scan of the open segments: s = sum from the segment's
    // first lane to this one; seen = a segment starts at or before this lane
    const bool has = bits != 0;
    double sc = cur;
    bool seen = has;
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
        const double su = __shfl_up(sc, d);
        const bool fu = __shfl_up((int)seen, d) != 0;
        if (lane >= d && !seen) {
            sc = su + sc;
            seen = fu;
        }
    }
    const double sprev = __shfl_up(sc, 1);
    const bool fprev = __shfl_up((int)seen, 1) != 0 && lane > 0;
    // a lane with a row start closes the segment open before it
    if (has && !(lane == 0 && (bits & 1))) {
        double total = lane > 0 ? sprev : 0.0;
        if (!(bits & 1)) total = total + head;
        const int row = rf - (int)(bits & 1);
        if (fprev) put(row, total);
        else A.nz_part[2 * w] = total;   // the end of a row that began in an earlier wave
    }
    if (lane == 63) {
        const int e = (w + 1) * kNzWave;
        const bool closes = e >= nnz || (A.nz_bits[(size_t)(w + 1) * 64] & 1);
        if (closes) {
            if (seen) put(r, sc);
            else A.nz_part[2 * w] = sc;
        } else {
            A.nz_part[2 * w + 1] = sc;   // the row goes on in the next wave
        }
    }
}

// Rows over several waves: the open pieces of the waves before the last, then the
// last wave's closing piece, in wave order.
template <bool PERM>
__global__ __launch_bounds__(kBlock) void k_spmv_nz_span(SpmvArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.nz_nspan) return;
    const int row = A.nz_span[3 * i], w0 = A.nz_span[3 * i + 1], w1 = A.nz_span[3 * i + 2];
    double sum = A.nz_part[2 * w0 + 1];
    for (int w = w0 + 1; w < w1; ++w) sum = sum + A.nz_part[2 * w + 1];
    sum = sum + A.nz_part[2 * w1];
    const int yr = PERM ? A.perm[row] : row;
    double out = A.alpha * sum;
    if (A.beta != 0.0) {
        const double by = A.beta * A.y[yr];
        out = out + by;
    }
    A.y[yr] = out;
}

hipError_t launch_spmv(const SpmvArgs &A, int lanes, hipStream_t s) {
    hipError_t e;
    if (A.nz_waves > 0 && A.nrhs == 1) {
        dim3 g(grid_for((int64_t)A.nz_waves * 64, kBlock));
        if (A.perm) hipLaunchKernelGGL((k_spmv_nz<true>), g, dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_spmv_nz<false>), g, dim3(kBlock), 0, s, A);
        if ((e = hipGetLastError()) != hipSuccess || A.nz_nspan <= 0) return e;
        dim3 g2(grid_for((int64_t)A.nz_nspan, kBlock));
        if (A.perm) hipLaunchKernelGGL((k_spmv_nz_span<true>), g2, dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_spmv_nz_span<false>), g2, dim3(kBlock), 0, s, A);
        return hipGetLastError();
    }
    switch (lanes) {
        case 1: {
            dim3 g(grid_for((int64_t)A.n, kBlock));
            if (A.perm) hipLaunchKernelGGL((k_spmv_lane<true>), g, dim3(kBlock), 0, s, A);
            else hipLaunchKernelGGL((k_spmv_lane<false>), g, dim3(kBlock), 0, s, A);
            e = hipGetLastError();
            break;
        }
        case 4: e = spmv_dispatch<4>(A, s); break;
        case 8: e = spmv_dispatch<8>(A, s); break;
        case 16: e = spmv_dispatch<16>(A, s); break;
        case 32: e = spmv_dispatch<32>(A, s); break;
        case 64: e = spmv_dispatch<64>(A, s); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || A.nheavy <= 0) return e;
    dim3 g(grid_for((int64_t)A.nheavy * 64, kBlock));
    if (A.perm) hipLaunchKernelGGL((k_spmv_heavy<true>), g, dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL((k_spmv_heavy<false>), g, dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

}  // namespace jv
