// Level sets on the device (Sec. II, level scheduling; Sec. III, the dependency
// graph of lower(S) or lower(S + S^T)).
//
// A row's level is 0 when it depends on no row, else one more than the deepest
// row it depends on; the level order lists the rows by (level, row index).  This
// is the same result as the host analysis's frontier peeling, reached in one
// sync-free sweep instead of one pass per level:
//   1. the CSR pattern is checked (monotone row pointers, sorted unique columns in
//      range), so every dependency index read later is in bounds;
//   2. with the symmetric pattern, the strictly upper entries are transposed
//      (column counts, a scan, a scatter), giving each row the earlier rows that
//      list it;
//   3. one persistent sweep: blocks claim 256-row slots in start order, one lane
//      per row; a lane reads its dependencies' levels as they are published (a
//      level is its own ready flag: -1 until written) and publishes its own;
//   4. keys (level << 32 | row) are radix-sorted, which gives the stable order,
//      and the level pointers are read off the sorted keys.
// The same sweep on the strictly upper part, from the last row down, gives the
// backward solve's schedule (Sec. VI) of a permuted factor pattern.
//
// The other device-side analysis calls of this file:
//   - the permuted structure P S P^T in a given order (Sec. III's copy into the
//     level-ordered CSR of L and U): row lengths gathered and scanned, columns
//     renamed, one segmented radix sort by row, diagonal positions;
//   - the transposed structure the adjoint's solves use: column counts, a scan,
//     a scatter, the same segmented sort.
// Every kernel after a call's input check reads the check's error word first
// and does nothing when it is set, so a bad input is never indexed; each call
// makes one scratch allocation and synchronises with the host once, at the end.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>
#include <hipcub/device/device_scan.hpp>
#include <hipcub/device/device_segmented_radix_sort.hpp>

#include <algorithm>
#include <cstdint>
#include <string>

#include "device.h"
#include "handle.h"
#include "javelin.h"

namespace jv {

namespace {

constexpr int kLvBlock = 256;

__device__ __forceinline__ int32_t lv_load(const int32_t *p) {
    return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lv_store(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// err bits: 1 row pointers, 2 column out of range, 4 columns unsorted or repeated
__global__ void k_lv_check(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = rp[i], e = rp[i + 1];
    int bits = 0;
    if ((i == 0 && b != 0) || (i == n - 1 && e != nnz) || b < 0 || e < b || e > nnz) {
        bits = 1;
    } else {
        int32_t prev = -1;
        for (int32_t p = b; p < e; ++p) {
            const int32_t c = ci[p];
            if (c < 0 || c >= n) bits |= 2;
            else if (c <= prev) bits |= 4;
            prev = c;
        }
    }
    if (bits) atomicOr(err, bits);
}

// strictly upper entries (i, j), j > i: row j gains the dependency i
__global__ void k_lv_upper_count(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *cnt, const int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || *err) return;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] > i) atomicAdd(&cnt[ci[p]], 1);
}

__global__ void k_lv_upper_scatter(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *tptr,
                                   int32_t *fill, int32_t *tdep, const int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || *err) return;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
        const int32_t j = ci[p];
        if (j > i) tdep[tptr[j] + atomicAdd(&fill[j], 1)] = (int32_t)i;
    }
}

__global__ void k_lv_fill(int32_t n, int32_t *level, int32_t *cnt, int32_t *fill) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        level[i] = -1;
        if (cnt) cnt[i] = 0;
        if (fill) fill[i] = 0;
    }
    if (i == 0 && cnt) cnt[n] = 0;
}

// One lane per row; blocks claim consecutive 256-row slots in start order, so a
// lane only waits on rows of blocks that started earlier (or of earlier lanes of
// its own block), which always progress.  With the upper pattern the slots run
// from the last row down, so the same holds for dependencies on later rows.  A lane polls without blocking its
// wave.  It scans its dependencies eight at a time (all eight loads in flight
// together), folds the published levels and keeps up to kLvPend pending
// dependencies in registers; later passes re-read only those (one round of
// loads), and the scan resumes when a slot frees up.  The wave leaves when
// every lane has published.  A pass in which some lane of the wave published is
// followed at once by the next (a dependency inside the wave is then ready);
// otherwise the wave sleeps, longer after each pass without progress (up to
// kLvSleepMax), so that waves far from the ready front load the memory system
// less.  Bounded: after kWaitTicks without progress in its wave, or when
// another wave has given up, the lane stops and raises the abort word (the
// host reports ILU_ERR_TIMEOUT).
constexpr int kLvBatch = 8;
constexpr int kLvPend = 8;
constexpr int kLvSleepMax = 32;

// Scans deps [*cur, end): published levels are folded into *lev, pending
// dependencies go to free slots of pend (-1 = free); the scan stops at a pending
// dependency with no free slot (*cur is left there).  idx(u) gives the
// dependency at u, or -1 for an entry that is not one.  Returns true when the
// whole range has been scanned.
template <typename Idx>
__device__ __forceinline__ bool lv_scan(int32_t *cur, int32_t end, int32_t *lev, const int32_t *level, Idx idx,
                                        int32_t (&pend)[kLvPend]) {
    int32_t u = *cur;
    while (u < end) {
        int32_t j[kLvBatch], v[kLvBatch];
#pragma unroll
        for (int k = 0; k < kLvBatch; ++k) j[k] = u + k < end ? idx(u + k) : -1;
#pragma unroll
        for (int k = 0; k < kLvBatch; ++k) v[k] = j[k] >= 0 ? lv_load(level + j[k]) : 0;
        int32_t stop = kLvBatch;
#pragma unroll
        for (int k = 0; k < kLvBatch; ++k) {
            if (stop == kLvBatch && j[k] >= 0) {
                if (v[k] >= 0) {
                    *lev = max(*lev, v[k] + 1);
                } else {
                    bool placed = false;
#pragma unroll
                    for (int s = 0; s < kLvPend; ++s)
                        if (!placed && pend[s] < 0) {
                            pend[s] = j[k];
                            placed = true;
                        }
                    if (!placed) stop = k;
                }
            }
        }
        u += stop;
        if (stop < kLvBatch) {
            *cur = u;
            return false;
        }
    }
    *cur = end;
    return true;
}

__global__ __launch_bounds__(kLvBlock) void k_lv_sweep(int32_t n, const int32_t *rp, const int32_t *ci,
                                                       const int32_t *tptr, const int32_t *tdep,
                                                       int32_t *level, int32_t *counter, int32_t *info,
                                                       uint32_t *maxlev, const int32_t *err, int32_t upper) {
    if (*err) return;   // the pattern failed its check: nothing is read
    __shared__ int32_t slot;
    if (threadIdx.x == 0) slot = atomicAdd(counter, 1);
    __syncthreads();
    // slots run from the first row, or (upper pattern) from the last row down
    const int64_t s64 = (int64_t)slot * kLvBlock + threadIdx.x;
    bool done = s64 >= n;
    const int32_t i = done ? 0 : (int32_t)(upper ? n - 1 - s64 : s64);
    int32_t p = done ? 0 : rp[i], pe = done ? 0 : rp[i + 1];
    int32_t q = (done || !tptr) ? 0 : tptr[i], qe = (done || !tptr) ? 0 : tptr[i + 1];
    int32_t lev = 0;
    int32_t pend[kLvPend];
#pragma unroll
    for (int s = 0; s < kLvPend; ++s) pend[s] = -1;
    bool scanned = false;
    uint64_t t0 = 0;
    int spins = 0, nap = 1;
    for (;;) {
        bool published = false;
        if (!done) {
            int32_t v[kLvPend];
#pragma unroll
            for (int s = 0; s < kLvPend; ++s) v[s] = pend[s] >= 0 ? lv_load(level + pend[s]) : -1;
            bool clear = true;
#pragma unroll
            for (int s = 0; s < kLvPend; ++s) {
                if (pend[s] >= 0 && v[s] >= 0) {
                    lev = max(lev, v[s] + 1);
                    pend[s] = -1;
                }
                clear = clear && pend[s] < 0;
            }
            // row entries (columns below i are dependencies), then the transposed ones
            if (!scanned)
                scanned = lv_scan(&p, pe, &lev, level,
                                  [&](int32_t u) {
                                      const int32_t c = ci[u];
                                      return (upper ? c > i : c < i) ? c : -1;
                                  },
                                  pend) &&
                          lv_scan(&q, qe, &lev, level, [&](int32_t u) { return tdep[u]; }, pend);
            if (scanned) {
                clear = true;
#pragma unroll
                for (int s = 0; s < kLvPend; ++s) clear = clear && pend[s] < 0;
            }
            if (scanned && clear) {
                lv_store(level + i, lev);
                done = published = true;
            }
        }
        if (__all(done)) break;
        if (__any(published)) {
            t0 = 0;   // the bound counts time without progress
            nap = 1;
            continue;
        }
        if ((++spins & 63) == 0) {
            if (__hip_atomic_load(&info[kInfoAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (t0 == 0) {
                t0 = now;
            } else if (now - t0 > kWaitTicks) {
                __hip_atomic_store(&info[kInfoAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        for (int k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(1);
        nap = min(2 * nap, kLvSleepMax);
    }
    // deepest level: one atomic per wave
    int32_t m = s64 < n ? lev : 0;
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(maxlev, (uint32_t)m);
}

__global__ void k_lv_keys(int32_t n, const int32_t *level, uint64_t *keys, const int32_t *err, const int32_t *info) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (*err || info[kInfoAbort]) return;
    if (i < n) keys[i] = (uint64_t)(uint32_t)level[i] << 32 | (uint32_t)i;
}

// sorted keys -> perm, iperm, level_ptr (every level from 0 to the last holds a
// row: a row of level l > 0 depends on one of level l - 1)
__global__ void k_lv_out(int32_t n, const uint64_t *keys, int32_t *perm, int32_t *iperm, int32_t *level_ptr,
                         const int32_t *err, const int32_t *info) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || *err || info[kInfoAbort]) return;
    const uint64_t k = keys[r];
    const int32_t row = (int32_t)(uint32_t)k, lev = (int32_t)(k >> 32);
    perm[r] = row;
    iperm[row] = (int32_t)r;
    if (r == 0 || (int32_t)(keys[r - 1] >> 32) != lev) level_ptr[lev] = (int32_t)r;
    if (r == n - 1) level_ptr[lev + 1] = n;
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kLvBlock - 1) / kLvBlock); }

// Permuted structure P S P^T (Sec. III: the parallel copy into the level-ordered
// CSR of L and U): row r of the result is row perm[r] of S with its columns
// renamed by iperm and sorted.  err bit 8: perm is not a permutation.
__global__ void k_pm_check(int32_t n, const int32_t *perm, const int32_t *iperm, int32_t *err) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t i = perm[r];
    if (i < 0 || i >= n || iperm[i] != (int32_t)r) atomicOr(err, 8);
}

__global__ void k_pm_len(int32_t n, const int32_t *rp, const int32_t *perm, int32_t *len, const int32_t *err) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    // zero lengths after a failed check: the scan and the sort then see empty rows
    len[r] = r < n && !*err ? rp[perm[r] + 1] - rp[perm[r]] : 0;
}

__global__ void k_pm_gather(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *perm,
                            const int32_t *iperm, const int32_t *orp, int32_t *key, int32_t *src, const int32_t *err) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || *err) return;
    const int32_t i = perm[r], o = orp[r];
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
        key[o + (p - rp[i])] = iperm[ci[p]];
        src[o + (p - rp[i])] = p;
    }
}

// Transposed structure: entries counted per column, then scattered to their
// column's range in any order (a segmented sort by row restores the order).
__global__ void k_tr_count(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *cnt, const int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || *err) return;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(&cnt[ci[p]], 1);
}

__global__ void k_tr_scatter(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *trp, int32_t *fill,
                             int32_t *key, int32_t *map, const int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || *err) return;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
        const int32_t j = ci[p];
        const int32_t o = trp[j] + atomicAdd(&fill[j], 1);
        key[o] = (int32_t)i;
        map[o] = p;
    }
}

// position of column r in row r (binary search of the sorted row), -1 if absent
__global__ void k_pm_diag(int32_t n, const int32_t *orp, const int32_t *oci, int32_t *diag, const int32_t *err) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || *err) return;
    int32_t lo = orp[r], hi = orp[r + 1];
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (oci[mid] < r) lo = mid + 1;
        else hi = mid;
    }
    diag[r] = lo < orp[r + 1] && oci[lo] == r ? lo : -1;
}

}  // namespace

}  // namespace jv

using namespace jv;

extern "C" ilu_status ilu_levels_device(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                        int32_t pattern, int32_t *level_ptr, int32_t *perm, int32_t *iperm,
                                        int32_t *n_levels, hipStream_t stream) {
    if (n <= 0 || n >= (1 << 30) || nnz < 0 || nnz >= ((int64_t)1 << 31) || !row_ptr || (nnz > 0 && !col_idx) ||
        !level_ptr || !perm || !iperm || !n_levels)
        return fail(ILU_ERR_ARG, "ilu_levels_device: bad argument");
    if (pattern != ILU_PATTERN_LOWER_SYM && pattern != ILU_PATTERN_LOWER_A && pattern != ILU_PATTERN_UPPER_A)
        return fail(ILU_ERR_ARG, "ilu_levels_device: unknown pattern");
    const bool sym = pattern == ILU_PATTERN_LOWER_SYM, upper = pattern == ILU_PATTERN_UPPER_A;
    // Levels are below n < 2^30, so the sort keys need 32 + bits(n - 1) bits.
    int end_bit = 32;
    while (end_bit < 62 && ((int64_t)(n - 1) >> (end_bit - 32)) != 0) ++end_bit;
    // Scratch sizes, then one allocation: control words, levels, two key arrays,
    // and with the symmetric pattern the counts, their scan, the fill cursors and
    // the transposed lists (at most nnz entries), plus the library temporaries.
    hipError_t e;
    size_t scan_b = 0, sort_b = 0;
    if (sym && (e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_b, (int32_t *)nullptr, (int32_t *)nullptr, n + 1,
                                                     stream)) != hipSuccess)
        return hip_fail(e, "ilu_levels_device: scan size");
    if ((e = hipcub::DeviceRadixSort::SortKeys(nullptr, sort_b, (uint64_t *)nullptr, (uint64_t *)nullptr, n, 0,
                                               end_bit, stream)) != hipSuccess)
        return hip_fail(e, "ilu_levels_device: sort size");
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_level = 256, o_keys = o_level + al((size_t)n * 4), o_keys2 = o_keys + al((size_t)n * 8),
                 o_cnt = o_keys2 + al((size_t)n * 8), o_tptr = o_cnt + (sym ? al(((size_t)n + 1) * 4) : 0),
                 o_fill = o_tptr + (sym ? al(((size_t)n + 1) * 4) : 0), o_tdep = o_fill + (sym ? al((size_t)n * 4) : 0),
                 o_scan = o_tdep + (sym ? al((size_t)std::max<int64_t>(nnz, 1) * 4) : 0), o_sort = o_scan + al(scan_b),
                 total = o_sort + al(std::max<size_t>(sort_b, 1));
    char *base = nullptr;
    if ((e = hipMalloc((void **)&base, total)) != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(ILU_ERR_NOMEM, "ilu_levels_device: device memory")
                                        : hip_fail(e, "ilu_levels_device: allocate");
    struct Guard {
        void *p;
        hipStream_t s;
        ~Guard() {
            (void)hipStreamSynchronize(s);
            (void)hipFree(p);
        }
    } g{base, stream};
    int32_t *ctl = reinterpret_cast<int32_t *>(base);
    int32_t *err = ctl, *info = ctl + 16, *counter = ctl + 32;
    uint32_t *maxlev = reinterpret_cast<uint32_t *>(ctl + 48);
    int32_t *level = reinterpret_cast<int32_t *>(base + o_level);
    uint64_t *keys = reinterpret_cast<uint64_t *>(base + o_keys), *keys2 = reinterpret_cast<uint64_t *>(base + o_keys2);
    int32_t *cnt = sym ? reinterpret_cast<int32_t *>(base + o_cnt) : nullptr;
    int32_t *tptr = sym ? reinterpret_cast<int32_t *>(base + o_tptr) : nullptr;
    int32_t *fill = sym ? reinterpret_cast<int32_t *>(base + o_fill) : nullptr;
    int32_t *tdep = sym ? reinterpret_cast<int32_t *>(base + o_tdep) : nullptr;
    // Every kernel after the check reads the error word first and does nothing
    // when it is set, so an invalid pattern is never indexed; the sort then runs
    // on keys nobody reads.  One synchronisation at the end.
    if ((e = hipMemsetAsync(ctl, 0, 64 * sizeof(int32_t), stream)) != hipSuccess)
        return hip_fail(e, "ilu_levels_device: clear");
    k_lv_check<<<grid_of(n), kLvBlock, 0, stream>>>(n, nnz, row_ptr, col_idx, err);
    k_lv_fill<<<grid_of((int64_t)n + 1), kLvBlock, 0, stream>>>(n, level, cnt, fill);
    if (sym) {
        k_lv_upper_count<<<grid_of(n), kLvBlock, 0, stream>>>(n, row_ptr, col_idx, cnt, err);
        if ((e = hipcub::DeviceScan::ExclusiveSum(base + o_scan, scan_b, cnt, tptr, n + 1, stream)) != hipSuccess)
            return hip_fail(e, "ilu_levels_device: scan");
        k_lv_upper_scatter<<<grid_of(n), kLvBlock, 0, stream>>>(n, row_ptr, col_idx, tptr, fill, tdep, err);
    }
    k_lv_sweep<<<grid_of(n), kLvBlock, 0, stream>>>(n, row_ptr, col_idx, tptr, tdep, level, counter, info, maxlev,
                                                    err, upper ? 1 : 0);
    k_lv_keys<<<grid_of(n), kLvBlock, 0, stream>>>(n, level, keys, err, info);
    if ((e = hipcub::DeviceRadixSort::SortKeys(base + o_sort, sort_b, keys, keys2, n, 0, end_bit, stream)) !=
        hipSuccess)
        return hip_fail(e, "ilu_levels_device: sort");
    k_lv_out<<<grid_of(n), kLvBlock, 0, stream>>>(n, keys2, perm, iperm, level_ptr, err, info);
    int32_t h[64];
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(h, ctl, sizeof(h), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return hip_fail(e, "ilu_levels_device: run");
    if (h[0] & 1) return fail(ILU_ERR_CSR, "ilu_levels_device: row_ptr not monotone or not ending at nnz");
    if (h[0] & 2) return fail(ILU_ERR_CSR, "ilu_levels_device: column index out of range");
    if (h[0] & 4) return fail(ILU_ERR_CSR, "ilu_levels_device: columns unsorted or repeated");
    if (h[16 + kInfoAbort]) return fail(ILU_ERR_TIMEOUT, "ilu_levels_device: a dependency wait expired");
    *n_levels = h[48] + 1;
    return ILU_OK;
}

extern "C" ilu_status ilu_permute_device(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                         const int32_t *perm, const int32_t *iperm, int32_t *out_row_ptr,
                                         int32_t *out_col_idx, int32_t *out_src, int32_t *diag_pos,
                                         hipStream_t stream) {
    if (n <= 0 || n >= (1 << 30) || nnz < 0 || nnz >= ((int64_t)1 << 31) || !row_ptr || (nnz > 0 && !col_idx) ||
        !perm || !iperm || !out_row_ptr || (nnz > 0 && (!out_col_idx || !out_src)) || !diag_pos)
        return fail(ILU_ERR_ARG, "ilu_permute_device: bad argument");
    int kbits = 1;
    while (kbits < 31 && ((int64_t)(n - 1) >> kbits) != 0) ++kbits;
    hipError_t e;
    size_t scan_b = 0, sort_b = 0;
    if ((e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_b, (int32_t *)nullptr, (int32_t *)nullptr, n + 1,
                                              stream)) != hipSuccess)
        return hip_fail(e, "ilu_permute_device: scan size");
    if (nnz > 0 &&
        (e = hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, sort_b, (int32_t *)nullptr, (int32_t *)nullptr,
                                                         (int32_t *)nullptr, (int32_t *)nullptr, (int)nnz, n,
                                                         (int32_t *)nullptr, (int32_t *)nullptr, 0, kbits,
                                                         stream)) != hipSuccess)
        return hip_fail(e, "ilu_permute_device: sort size");
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_len = 256, o_key = o_len + al(((size_t)n + 1) * 4), o_src = o_key + al((size_t)nnz * 4 + 4),
                 o_scan = o_src + al((size_t)nnz * 4 + 4), o_sort = o_scan + al(scan_b),
                 total = o_sort + al(std::max<size_t>(sort_b, 1));
    char *base = nullptr;
    if ((e = hipMalloc((void **)&base, total)) != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(ILU_ERR_NOMEM, "ilu_permute_device: device memory")
                                        : hip_fail(e, "ilu_permute_device: allocate");
    struct Guard {
        void *p;
        hipStream_t s;
        ~Guard() {
            (void)hipStreamSynchronize(s);
            (void)hipFree(p);
        }
    } g{base, stream};
    int32_t *err = reinterpret_cast<int32_t *>(base);
    int32_t *len = reinterpret_cast<int32_t *>(base + o_len);
    int32_t *key = reinterpret_cast<int32_t *>(base + o_key), *src = reinterpret_cast<int32_t *>(base + o_src);
    // as for the level sets: every kernel after the checks does nothing once one
    // has failed, and one synchronisation at the end reports it
    if ((e = hipMemsetAsync(err, 0, 64 * sizeof(int32_t), stream)) != hipSuccess)
        return hip_fail(e, "ilu_permute_device: clear");
    k_lv_check<<<grid_of(n), kLvBlock, 0, stream>>>(n, nnz, row_ptr, col_idx, err);
    k_pm_check<<<grid_of(n), kLvBlock, 0, stream>>>(n, perm, iperm, err);
    k_pm_len<<<grid_of((int64_t)n + 1), kLvBlock, 0, stream>>>(n, row_ptr, perm, len, err);
    if ((e = hipcub::DeviceScan::ExclusiveSum(base + o_scan, scan_b, len, out_row_ptr, n + 1, stream)) != hipSuccess)
        return hip_fail(e, "ilu_permute_device: scan");
    if (nnz > 0) {
        k_pm_gather<<<grid_of(n), kLvBlock, 0, stream>>>(n, row_ptr, col_idx, perm, iperm, out_row_ptr, key, src, err);
        if ((e = hipcub::DeviceSegmentedRadixSort::SortPairs(base + o_sort, sort_b, key, out_col_idx, src, out_src,
                                                             (int)nnz, n, out_row_ptr, out_row_ptr + 1, 0, kbits,
                                                             stream)) != hipSuccess)
            return hip_fail(e, "ilu_permute_device: sort");
    }
    k_pm_diag<<<grid_of(n), kLvBlock, 0, stream>>>(n, out_row_ptr, out_col_idx, diag_pos, err);
    int32_t h = 0;
    if ((e = hipGetLastError()) != hipSuccess || (e = hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return hip_fail(e, "ilu_permute_device: run");
    if (h & 1) return fail(ILU_ERR_CSR, "ilu_permute_device: row_ptr not monotone or not ending at nnz");
    if (h & 2) return fail(ILU_ERR_CSR, "ilu_permute_device: column index out of range");
    if (h & 4) return fail(ILU_ERR_CSR, "ilu_permute_device: columns unsorted or repeated");
    if (h & 8) return fail(ILU_ERR_ARG, "ilu_permute_device: perm / iperm not a permutation and its inverse");
    return ILU_OK;
}

extern "C" ilu_status ilu_transpose_device(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                           int32_t *t_row_ptr, int32_t *t_col_idx, int32_t *t_map, int32_t *t_diag,
                                           hipStream_t stream) {
    if (n <= 0 || n >= (1 << 30) || nnz < 0 || nnz >= ((int64_t)1 << 31) || !row_ptr || (nnz > 0 && !col_idx) ||
        !t_row_ptr || (nnz > 0 && (!t_col_idx || !t_map)) || !t_diag)
        return fail(ILU_ERR_ARG, "ilu_transpose_device: bad argument");
    int kbits = 1;
    while (kbits < 31 && ((int64_t)(n - 1) >> kbits) != 0) ++kbits;
    hipError_t e;
    size_t scan_b = 0, sort_b = 0;
    if ((e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_b, (int32_t *)nullptr, (int32_t *)nullptr, n + 1,
                                              stream)) != hipSuccess)
        return hip_fail(e, "ilu_transpose_device: scan size");
    if (nnz > 0 &&
        (e = hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, sort_b, (int32_t *)nullptr, (int32_t *)nullptr,
                                                         (int32_t *)nullptr, (int32_t *)nullptr, (int)nnz, n,
                                                         (int32_t *)nullptr, (int32_t *)nullptr, 0, kbits,
                                                         stream)) != hipSuccess)
        return hip_fail(e, "ilu_transpose_device: sort size");
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_cnt = 256, o_fill = o_cnt + al(((size_t)n + 1) * 4), o_key = o_fill + al((size_t)n * 4),
                 o_map = o_key + al((size_t)nnz * 4 + 4), o_scan = o_map + al((size_t)nnz * 4 + 4),
                 o_sort = o_scan + al(scan_b), total = o_sort + al(std::max<size_t>(sort_b, 1));
    char *base = nullptr;
    if ((e = hipMalloc((void **)&base, total)) != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(ILU_ERR_NOMEM, "ilu_transpose_device: device memory")
                                        : hip_fail(e, "ilu_transpose_device: allocate");
    struct Guard {
        void *p;
        hipStream_t s;
        ~Guard() {
            (void)hipStreamSynchronize(s);
            (void)hipFree(p);
        }
    } g{base, stream};
    int32_t *err = reinterpret_cast<int32_t *>(base);
    int32_t *cnt = reinterpret_cast<int32_t *>(base + o_cnt), *fill = reinterpret_cast<int32_t *>(base + o_fill);
    int32_t *key = reinterpret_cast<int32_t *>(base + o_key), *map = reinterpret_cast<int32_t *>(base + o_map);
    if ((e = hipMemsetAsync(err, 0, 64 * sizeof(int32_t), stream)) != hipSuccess)
        return hip_fail(e, "ilu_transpose_device: clear");
    k_lv_check<<<grid_of(n), kLvBlock, 0, stream>>>(n, nnz, row_ptr, col_idx, err);
    k_lv_fill<<<grid_of((int64_t)n + 1), kLvBlock, 0, stream>>>(n, t_diag, cnt, fill);   // t_diag is overwritten below
    k_tr_count<<<grid_of(n), kLvBlock, 0, stream>>>(n, row_ptr, col_idx, cnt, err);
    if ((e = hipcub::DeviceScan::ExclusiveSum(base + o_scan, scan_b, cnt, t_row_ptr, n + 1, stream)) != hipSuccess)
        return hip_fail(e, "ilu_transpose_device: scan");
    if (nnz > 0) {
        k_tr_scatter<<<grid_of(n), kLvBlock, 0, stream>>>(n, row_ptr, col_idx, t_row_ptr, fill, key, map, err);
        if ((e = hipcub::DeviceSegmentedRadixSort::SortPairs(base + o_sort, sort_b, key, t_col_idx, map, t_map, (int)nnz,
                                                             n, t_row_ptr, t_row_ptr + 1, 0, kbits, stream)) !=
            hipSuccess)
            return hip_fail(e, "ilu_transpose_device: sort");
    }
    k_pm_diag<<<grid_of(n), kLvBlock, 0, stream>>>(n, t_row_ptr, t_col_idx, t_diag, err);
    int32_t h = 0;
    if ((e = hipGetLastError()) != hipSuccess || (e = hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return hip_fail(e, "ilu_transpose_device: run");
    if (h & 1) return fail(ILU_ERR_CSR, "ilu_transpose_device: row_ptr not monotone or not ending at nnz");
    if (h & 2) return fail(ILU_ERR_CSR, "ilu_transpose_device: column index out of range");
    if (h & 4) return fail(ILU_ERR_CSR, "ilu_transpose_device: columns unsorted or repeated");
    return ILU_OK;
}
