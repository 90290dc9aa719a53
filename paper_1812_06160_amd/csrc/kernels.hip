// HIP kernels for gfx950: up-looking ILU factor, triangular solves, spmv, casts.
//
// Every kernel works on groups of G lanes (G in {4, 8, 16, 32, 64}) inside a
// 64-wide wavefront; a group owns one row.  Two launch schemes share the same
// per-row code:
//
//  * level launch: one kernel per level (the kernel boundary is the barrier
//    between levels, the classic level-set scheme the paper compares against,
//    Sec. VI "CSR-LS");
//  * sync-free persistent launch: one kernel for all levels.  Waves take
//    level-homogeneous tasks (up to 64/G consecutive rows of one level) in level
//    order, round-robin; a row reads each value it depends on with an
//    agent-scope atomic load until it is no longer the "pending" bit pattern.
//    This is the GPU form of the paper's point-to-point synchronisation (Sec. III,
//    "Level Scheduling, Upper Stage"): a row waits only for the rows it needs,
//    never for a whole level.  Values are published with agent-scope relaxed
//    atomic stores, so no cache-flushing release fence is needed (coherence of
//    atomics to one address is enough: each consumed value is its own flag).
//
// Deadlock freedom of the persistent scheme: a task only waits on rows of earlier
// levels, i.e. on earlier tasks; the smallest unfinished task always has every
// dependency finished and is being processed by its wave (a wave handles its
// tasks in increasing order), provided every wave of the grid is resident -- the
// host sizes the grid from the occupancy query.  Every wait is bounded
// (kSpinLimit) and raises a device abort flag that stops all waits.
//
// Floating point: the library is compiled with -ffp-contract=off, so a - l*u is
// a rounded multiply then a rounded subtract, and FP64 division is IEEE
// correctly rounded; with the columns of a row taken in ascending order the
// factor reproduces a serial up-looking ILU bit for bit.
#include <hip/hip_runtime.h>
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

// Bounded wait until *p differs from the pending pattern.  On expiry (or when
// another wave has expired) returns a quiet NaN; the host reports ILU_ERR_TIMEOUT.
__device__ uint64_t wait_u64(const uint64_t *p, int32_t *info) {
    uint64_t v = ld_acq_u64(p);
    if (v != kPending64) return v;
    int spins = 0;
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        v = ld_acq_u64(p);
        if (v != kPending64) return v;
        if ((++spins & 31) == 0) {
            if (aborted(info)) return kQNaN64;
            if (spins > kSpinLimit) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return kQNaN64;
            }
        }
    }
}

__device__ uint32_t wait_u32(const uint32_t *p, int32_t *info) {
    uint32_t v = ld_acq_u32(p);
    if (v != kPending32) return v;
    int spins = 0;
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        v = ld_acq_u32(p);
        if (v != kPending32) return v;
        if ((++spins & 31) == 0) {
            if (aborted(info)) return kQNaN32;
            if (spins > kSpinLimit) {
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

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// ---------------------------------------------------------------------------------
// Typed access to published intermediates
// ---------------------------------------------------------------------------------
template <typename TA> struct Pub;
template <> struct Pub<double> {
    __device__ static double wait(const double *p, int32_t *info) {
        return __longlong_as_double((long long)wait_u64(reinterpret_cast<const uint64_t *>(p), info));
    }
    __device__ static void publish(double *p, double v) {
        uint64_t b = (uint64_t)__double_as_longlong(v);
        if (v != v) b = kQNaN64;
        st_pub_u64(reinterpret_cast<uint64_t *>(p), b);
    }
    __device__ static double pending() { return __longlong_as_double((long long)kPending64); }
};
template <> struct Pub<float> {
    __device__ static float wait(const float *p, int32_t *info) {
        return __uint_as_float(wait_u32(reinterpret_cast<const uint32_t *>(p), info));
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
__global__ void k_fill_u32(uint32_t *p, uint32_t value, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
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
// Up-looking ILU on the fixed pattern (paper Sec. III, Fig. 1), one row per group
// ---------------------------------------------------------------------------------
// Lane t of the group holds entry rs+t of row r (the host guarantees row length <= G).
// For each earlier column c of the row, in ascending order: lane e divides its
// entry by the pivot u_cc, the multiplier is broadcast, and every lane whose
// column matches a later column j of row c subtracts l * u_cj.  Row c's upper
// part (diagonal first) is loaded by lanes t < len(U(c)); its structure
// (diag_pos[c], row_ptr[c+1]) is fetched for all c up front.
template <int G, bool SF>
__device__ __forceinline__ void factor_row(const FactorArgs &A, int r, int t, int gi) {
    const int rs = A.rp[r], re = A.rp[r + 1], d = A.diag[r];
    const int nL = d - rs;
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
            if constexpr (SF) uv = Pub<double>::wait(&A.lu[q], A.info);
            else uv = A.lu[q];
        }
        const double piv = __shfl(uv, 0, G);
        if (t == e) {
            v = v / piv;
            if (A.use_tau && fabs(v) < tr) dropped = 1;
        }
        if (__shfl(dropped, e, G)) continue;
        const double l = __shfl(v, e, G);
        for (int j = 1; j < lenU; ++j) {
            const int uc = __shfl(ucol, j, G);
            const double uu = __shfl(uv, j, G);
            const int ua = __shfl(uabs, j, G);
            if (!ua && (uint64_t)__double_as_longlong(uu) != kDropped64 && col == uc && !absent) {
                const double prod = l * uu;
                v = v - prod;
            }
        }
    }
    if (A.use_tau && act && !absent && col > r && fabs(v) < tr) dropped = 1;
    const double pv = __shfl(v, d - rs, G);
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

template <int G>
__global__ __launch_bounds__(kBlock) void k_factor_level(FactorArgs A) {
    const int gid = (blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int t = threadIdx.x % G;
    const int gi = (threadIdx.x & 63) / G;
    const int r = A.row_begin + gid;
    if (r < A.row_end) factor_row<G, false>(A, r, t, gi);
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_factor_syncfree(FactorArgs A) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int t = threadIdx.x % G;
    const int gi = (threadIdx.x & 63) / G;
    for (int task = wave; task < A.ntasks; task += nwaves) {
        const int r = A.task_ptr[task] + gi;
        if (r < A.task_ptr[task + 1]) factor_row<G, true>(A, r, t, gi);
    }
}

// ---------------------------------------------------------------------------------
// Triangular solves (paper Sec. VI), one row per group, lanes over the row's entries
// ---------------------------------------------------------------------------------
// Forward: y_r = (b'_r - sum_{c<r} a_rc y_c) [/ a_rr unless unit]; b' = P b.
// Backward: z_r = (y_r - sum_{c>r} a_rc z_c) [/ a_rr unless unit]; x = P^T z.
// The y and z buffers keep the invariant "all pending" between applies: the
// forward pass re-arms z[r], the backward pass re-arms y[r] after reading it.
template <int G, typename TV, typename TX, typename TA, bool SF, bool FWD>
__device__ __forceinline__ void solve_row(const SolveArgs &A, int r, int t) {
    const TV *val = static_cast<const TV *>(A.val);
    TA *y = static_cast<TA *>(A.y);
    TA *z = static_cast<TA *>(A.z);
    const int rs = A.rp[r], re = A.rp[r + 1], d = A.diag[r];
    const int lo = FWD ? rs : d + 1;
    const int hi = FWD ? d : re;
    TA *dep = FWD ? y : z;
    const int64_t cap = A.cap;
    const int out_row = A.perm ? A.perm[r] : r;
    for (int s = 0; s < A.nrhs; ++s) {
        TA acc = 0;
        for (int p = lo + t; p < hi; p += G) {
            const int c = A.ci[p];
            const TA a = (TA)load_val(val, A.vmap ? A.vmap[p] : p);
            TA xc;
            if constexpr (SF) xc = Pub<TA>::wait(&dep[(int64_t)c * cap + s], A.info);
            else xc = dep[(int64_t)c * cap + s];
            const TA prod = a * xc;
            acc = acc + prod;
        }
        acc = group_sum<G>(acc);
        if (t == 0) {
            TA rhs;
            if constexpr (FWD) rhs = (TA)static_cast<const TX *>(A.b)[(int64_t)out_row * A.ld + s];
            else rhs = y[(int64_t)r * cap + s];
            TA v = rhs - acc;
            if (!A.unit_diag) v = v / (TA)load_val(val, A.vmap ? A.vmap[d] : d);
            if constexpr (FWD) {
                if constexpr (SF) Pub<TA>::publish(&y[(int64_t)r * cap + s], v);
                else y[(int64_t)r * cap + s] = v;
                z[(int64_t)r * cap + s] = Pub<TA>::pending();
                if (A.y_out) static_cast<TA *>(A.y_out)[(int64_t)r * A.ld + s] = v;
            } else {
                if constexpr (SF) Pub<TA>::publish(&z[(int64_t)r * cap + s], v);
                else z[(int64_t)r * cap + s] = v;
                y[(int64_t)r * cap + s] = Pub<TA>::pending();
                static_cast<TX *>(A.x)[(int64_t)out_row * A.ld + s] = (TX)v;
                if (A.z_out) static_cast<TA *>(A.z_out)[(int64_t)r * A.ld + s] = v;
            }
        }
    }
}

template <int G, typename TV, typename TX, typename TA, bool FWD>
__global__ __launch_bounds__(kBlock) void k_solve_level(SolveArgs A) {
    const int pos = A.row_begin + (blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (pos >= A.row_end) return;
    const int r = A.rows ? A.rows[pos] : pos;
    solve_row<G, TV, TX, TA, false, FWD>(A, r, threadIdx.x % G);
}

template <int G, typename TV, typename TX, typename TA, bool FWD>
__global__ __launch_bounds__(kBlock) void k_solve_syncfree(SolveArgs A) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int t = threadIdx.x % G;
    const int gi = (threadIdx.x & 63) / G;
    for (int task = wave; task < A.ntasks; task += nwaves) {
        const int pos = A.task_ptr[task] + gi;
        if (pos < A.task_ptr[task + 1]) {
            const int r = A.rows ? A.rows[pos] : pos;
            solve_row<G, TV, TX, TA, true, FWD>(A, r, t);
        }
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

template <typename F>
int occupancy_grid(F kernel) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
        if (cus <= 0) cus = 1;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    return per_cu * cus;
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

template <int G>
static hipError_t factor_dispatch(const FactorArgs &A, bool syncfree, int grid, hipStream_t s) {
    if (syncfree) {
        hipLaunchKernelGGL(k_factor_syncfree<G>, dim3(grid), dim3(kBlock), 0, s, A);
    } else {
        int64_t rows = A.row_end - A.row_begin;
        if (rows <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_factor_level<G>, dim3(grid_for(rows * G, kBlock)), dim3(kBlock), 0, s, A);
    }
    return hipGetLastError();
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

hipError_t launch_outer(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *perm, const double *W,
                        const double *Bp, const double *x, const double *y, double *glu, int32_t nrhs, int64_t ld,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_outer, dim3(grid_for((int64_t)n * 8, kBlock)), dim3(kBlock), 0, s, n, rp, ci, perm, W, Bp, x,
                       y, glu, nrhs, ld);
    return hipGetLastError();
}

int persistent_grid_factor(int lanes) {
    switch (lanes) {
        case 4: return occupancy_grid(k_factor_syncfree<4>);
        case 8: return occupancy_grid(k_factor_syncfree<8>);
        case 16: return occupancy_grid(k_factor_syncfree<16>);
        case 32: return occupancy_grid(k_factor_syncfree<32>);
        default: return occupancy_grid(k_factor_syncfree<64>);
    }
}

template <int G, typename TV, typename TX, typename TA>
static hipError_t solve_dispatch3(const SolveArgs &A, bool fwd, bool syncfree, int grid, hipStream_t s) {
    if (syncfree) {
        if (fwd) hipLaunchKernelGGL((k_solve_syncfree<G, TV, TX, TA, true>), dim3(grid), dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_solve_syncfree<G, TV, TX, TA, false>), dim3(grid), dim3(kBlock), 0, s, A);
    } else {
        int64_t rows = A.row_end - A.row_begin;
        if (rows <= 0) return hipSuccess;
        dim3 g(grid_for(rows * G, kBlock));
        if (fwd) hipLaunchKernelGGL((k_solve_level<G, TV, TX, TA, true>), g, dim3(kBlock), 0, s, A);
        else hipLaunchKernelGGL((k_solve_level<G, TV, TX, TA, false>), g, dim3(kBlock), 0, s, A);
    }
    return hipGetLastError();
}

template <int G, typename TV, typename TA>
static hipError_t solve_dispatch2(const SolveArgs &A, bool fwd, int vec, bool syncfree, int grid, hipStream_t s) {
    if (vec == 0) return solve_dispatch3<G, TV, double, TA>(A, fwd, syncfree, grid, s);
    return solve_dispatch3<G, TV, float, TA>(A, fwd, syncfree, grid, s);
}

template <int G>
static hipError_t solve_dispatch1(const SolveArgs &A, bool fwd, int prec, int vec, bool syncfree, int grid,
                                  hipStream_t s) {
    switch (prec) {
        case 0: return solve_dispatch2<G, double, double>(A, fwd, vec, syncfree, grid, s);
        case 1: return solve_dispatch2<G, float, float>(A, fwd, vec, syncfree, grid, s);
        case 2: return solve_dispatch2<G, uint16_t, float>(A, fwd, vec, syncfree, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve(const SolveArgs &A, bool forward, int prec, int vec, int lanes, bool syncfree, int grid,
                        hipStream_t s) {
    switch (lanes) {
        case 4: return solve_dispatch1<4>(A, forward, prec, vec, syncfree, grid, s);
        case 8: return solve_dispatch1<8>(A, forward, prec, vec, syncfree, grid, s);
        case 16: return solve_dispatch1<16>(A, forward, prec, vec, syncfree, grid, s);
        case 32: return solve_dispatch1<32>(A, forward, prec, vec, syncfree, grid, s);
        case 64: return solve_dispatch1<64>(A, forward, prec, vec, syncfree, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <int G>
static int solve_grid_g(bool fwd, int prec, int vec) {
    // the persistent solve kernels of one lane count share their resource use;
    // query the FP64 instance of the requested direction
    (void)prec;
    (void)vec;
    if (fwd) return occupancy_grid(k_solve_syncfree<G, double, double, double, true>);
    return occupancy_grid(k_solve_syncfree<G, double, double, double, false>);
}

int persistent_grid_solve(bool forward, int prec, int vec, int lanes) {
    switch (lanes) {
        case 4: return solve_grid_g<4>(forward, prec, vec);
        case 8: return solve_grid_g<8>(forward, prec, vec);
        case 16: return solve_grid_g<16>(forward, prec, vec);
        case 32: return solve_grid_g<32>(forward, prec, vec);
        default: return solve_grid_g<64>(forward, prec, vec);
    }
}

template <int G>
static hipError_t spmv_dispatch(const SpmvArgs &A, hipStream_t s) {
    dim3 g(grid_for((int64_t)A.n * G, kBlock));
    if (A.perm) hipLaunchKernelGGL((k_spmv<G, true>), g, dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL((k_spmv<G, false>), g, dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_spmv(const SpmvArgs &A, int lanes, hipStream_t s) {
    switch (lanes) {
        case 4: return spmv_dispatch<4>(A, s);
        case 8: return spmv_dispatch<8>(A, s);
        case 16: return spmv_dispatch<16>(A, s);
        case 32: return spmv_dispatch<32>(A, s);
        case 64: return spmv_dispatch<64>(A, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace jv
