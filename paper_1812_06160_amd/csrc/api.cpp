// C ABI of the incomplete-LU hot path (declared in include/javelin.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "analysis.h"
#include "blas.h"
#include "device.h"
#include "handle.h"
#include "par.h"
#include "javelin.h"

using namespace jv;

namespace jv {

thread_local std::string g_last_error;

ilu_status fail(ilu_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

ilu_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return ILU_ERR_HIP;
}

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc(dst, src.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

int pow2_lanes(int len, int lo, int hi) {
    int g = lo;
    while (g < len && g < hi) g <<= 1;
    return g;
}

// Task list of the persistent kernels: level-homogeneous runs of up to `per`
// consecutive positions, in level order.
std::vector<int32_t> make_tasks(const std::vector<int32_t> &level_ptr, int per) {
    std::vector<int32_t> t;
    for (size_t l = 0; l + 1 < level_ptr.size(); ++l)
        for (int32_t p = level_ptr[l]; p < level_ptr[l + 1]; p += per) t.push_back(p);
    t.push_back(level_ptr.empty() ? 0 : level_ptr.back());
    return t;
}

int Profiler::begin(int st, hipStream_t s) {
    if (!enabled || 2 * (used + 1) > pool.size()) return -1;
    if (hipEventRecord(pool[2 * used], s) != hipSuccess) return -1;
    stage.push_back(st);
    closed.push_back(0);
    return (int)used++;
}

void Profiler::end(int pair, hipStream_t s) {
    if (pair < 0 || (size_t)pair >= used) return;
    if (hipEventRecord(pool[2 * pair + 1], s) == hipSuccess) closed[pair] = 1;
}

void Profiler::release() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
    stage.clear();
    closed.clear();
    used = 0;
    enabled = false;
}

}  // namespace jv

ilu_handle_s::~ilu_handle_s() {
    prof.release();

    for (void *p : allocs) (void)hipFree(p);
    if (h_kry_pin) (void)hipHostFree(h_kry_pin);
    if (kry_ev) (void)hipEventDestroy(kry_ev);
    for (auto &kv : tasks) {
        (void)hipFree(kv.second.ptr);
        (void)hipFree(kv.second.stream_tasks);
        (void)hipFree(kv.second.stream_ptr);
    }
}

hipError_t ilu_handle_s::alloc_bytes(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
}

const TaskList *ilu_handle_s::task_list(int which, int lanes, int32_t levels) {
    const int64_t key = task_key(which, lanes, levels);
    auto it = tasks.find(key);
    if (it != tasks.end()) return &it->second;
    const std::vector<int32_t> *ptr = nullptr;
    switch (which) {
        case kTasksForward: ptr = &H.level_ptr; break;
        case kTasksBackward: ptr = &H.ulevel_ptr; break;
        case kTasksTForward: ptr = &H.tlevel_ptr; break;
        default: ptr = &H.tulevel_ptr; break;
    }
    // tasks: level-homogeneous runs of up to 64/lanes positions; each level's tasks
    // are cut into kStreams contiguous slices, slice x going to stream x
    const int per = 64 / lanes;
    const int S = nstreams;
    std::vector<int32_t> t;
    std::vector<std::vector<int32_t>> streams(S);
    const size_t nl = levels < 0 ? ptr->size() - 1 : std::min<size_t>((size_t)levels, ptr->size() - 1);
    for (size_t l = 0; l < nl; ++l) {
        const int32_t t0 = (int32_t)t.size();
        for (int32_t p = (*ptr)[l]; p < (*ptr)[l + 1]; p += per) t.push_back(p);
        const int32_t t1 = (int32_t)t.size();
        for (int x = 0; x < S; ++x) {
            const int32_t a = t0 + (int32_t)((int64_t)(t1 - t0) * x / S);
            const int32_t b = t0 + (int32_t)((int64_t)(t1 - t0) * (x + 1) / S);
            for (int32_t k = a; k < b; ++k) streams[x].push_back(k);
        }
    }
    t.push_back(ptr->empty() ? 0 : (*ptr)[nl]);
    std::vector<int32_t> st, sp(S + 1, 0);
    int32_t max_slots = 0;
    const int wpb = 4;   // waves per block: one task each
    for (int x = 0; x < S; ++x) {
        st.insert(st.end(), streams[x].begin(), streams[x].end());
        sp[x + 1] = (int32_t)st.size();
        max_slots = std::max<int32_t>(max_slots, ((int32_t)streams[x].size() + wpb - 1) / wpb);
    }
    TaskList tl;
    tl.ntasks = (int32_t)t.size() - 1;
    tl.max_slots = max_slots;
    auto up = [](int32_t **d, const std::vector<int32_t> &v) {
        if (hipMalloc(d, std::max<size_t>(1, v.size()) * sizeof(int32_t)) != hipSuccess) return false;
        if (v.empty()) return true;
        return hipMemcpy(*d, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(&tl.ptr, t) || !up(&tl.stream_tasks, st) || !up(&tl.stream_ptr, sp)) {
        (void)hipFree(tl.ptr);
        (void)hipFree(tl.stream_tasks);
        (void)hipFree(tl.stream_ptr);
        return nullptr;
    }
    tasks[key] = tl;
    return &tasks[key];
}

hipError_t ilu_handle_s::ensure_workspace(int nrhs, int prec_class, hipStream_t s) {
    // prec_class 0: FP64 intermediates, 1: FP32 intermediates
    int &cap = prec_class == 0 ? cap64 : cap32;
    void *&y = prec_class == 0 ? y64 : y32;
    void *&z = prec_class == 0 ? z64 : z32;
    if (cap >= nrhs) return hipSuccess;
    int newcap = std::max(nrhs, cap * 2);
    if (newcap < 1) newcap = 1;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (y) { (void)hipFree(y); allocs.erase(std::find(allocs.begin(), allocs.end(), y)); y = nullptr; }
    if (z) { (void)hipFree(z); allocs.erase(std::find(allocs.begin(), allocs.end(), z)); z = nullptr; }
    const size_t elt = prec_class == 0 ? 8 : 4;
    const size_t count = (size_t)H.n * (size_t)newcap;
    if ((e = alloc_bytes(&y, count * elt)) != hipSuccess) return e;
    if ((e = alloc_bytes(&z, count * elt)) != hipSuccess) return e;
    if (prec_class == 0) {
        if ((e = launch_fill_u64((uint64_t *)y, kPending64, (int64_t)count, s)) != hipSuccess) return e;
        if ((e = launch_fill_u64((uint64_t *)z, kPending64, (int64_t)count, s)) != hipSuccess) return e;
    } else {
        if ((e = launch_fill_u32((uint32_t *)y, kPending32, (int64_t)count, s)) != hipSuccess) return e;
        if ((e = launch_fill_u32((uint32_t *)z, kPending32, (int64_t)count, s)) != hipSuccess) return e;
    }
    cap = newcap;
    return hipStreamSynchronize(s);
}

// re-arms every published intermediate after an expired wait
hipError_t ilu_handle_s::rearm(hipStream_t s) {
    hipError_t e = hipSuccess;
    if (y64) e = launch_fill_u64((uint64_t *)y64, kPending64, (int64_t)H.n * cap64, s);
    if (e == hipSuccess && z64) e = launch_fill_u64((uint64_t *)z64, kPending64, (int64_t)H.n * cap64, s);
    if (e == hipSuccess && y32) e = launch_fill_u32((uint32_t *)y32, kPending32, (int64_t)H.n * cap32, s);
    if (e == hipSuccess && z32) e = launch_fill_u32((uint32_t *)z32, kPending32, (int64_t)H.n * cap32, s);
    return e;
}

// resets the factor's slots (bad row, abort, drop count); the timeout count and
// the guard's counter are left alone
hipError_t ilu_handle_s::reset_info(hipStream_t s) {
    static const int32_t init[kInfoTimeouts] = {INT_MAX, 0, 0, 0};
    return hipMemcpyAsync(d_info, init, sizeof(init), hipMemcpyHostToDevice, s);
}

hipError_t ilu_handle_s::guard(hipStream_t s) {
    return launch_solve_guard(d_info, (uint64_t *)y64, (uint64_t *)z64, (int64_t)H.n * cap64, (uint32_t *)y32,
                              (uint32_t *)z32, (int64_t)H.n * cap32, s);
}

// Reads the abort flag and the timeout count (synchronises s).  Either one set:
// re-arms the intermediates, clears both and returns ILU_ERR_TIMEOUT.
ilu_status ilu_handle_s::take_timeout(hipStream_t s, const char *who) {
    int32_t w[kInfoSlots];
    hipError_t e = hipMemcpyAsync(w, d_info, sizeof(w), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, who);
    if (!w[kInfoAbort] && !w[kInfoTimeouts]) return ILU_OK;
    static const int32_t zero2[2] = {0, 0};
    e = rearm(s);
    if (e == hipSuccess) e = hipMemcpyAsync(&d_info[kInfoAbort], zero2, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&d_info[kInfoTimeouts], zero2, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, who);
    return fail(ILU_ERR_TIMEOUT, std::string(who) + ": a dependency wait of an apply expired (its outputs are invalid)");
}

static const int32_t kDefaultTileRows = 512;

static const int kComplement[kPasses] = {-1,          kPassBackward, kPassForward, kPassTBackward,
                                         kPassTForward, kPassTileB,   kPassTileF,   -1};

hipError_t ilu_handle_s::prepare_claims(int pass, const TaskList *tl, Claims *c, hipStream_t s) {
    int32_t *mine = d_counters + (size_t)pass * kStreams * kCounterStride;
    if (counters_dirty[pass]) {
        hipError_t e = launch_zero_counters(mine, s);
        if (e != hipSuccess) return e;
    }
    c->task_ptr = tl->ptr;
    c->stream_tasks = tl->stream_tasks;
    c->stream_ptr = tl->stream_ptr;
    c->counters = mine;
    const int comp = kComplement[pass];
    c->zero_counters = comp >= 0 ? d_counters + (size_t)comp * kStreams * kCounterStride : nullptr;
    c->xcc_stream = d_xcc_stream;
    counters_dirty[pass] = true;
    if (comp >= 0) counters_dirty[comp] = false;
    return hipSuccess;
}

hipError_t ilu_handle_s::prepare_tile_claims(int pass, TileArgs *t, hipStream_t s) {
    int32_t *mine = d_counters + (size_t)pass * kStreams * kCounterStride;
    if (counters_dirty[pass]) {
        hipError_t e = launch_zero_counters(mine, s);
        if (e != hipSuccess) return e;
    }
    const int comp = kComplement[pass];
    t->counter = mine;
    t->zero_counter = comp >= 0 ? d_counters + (size_t)comp * kStreams * kCounterStride : nullptr;
    counters_dirty[pass] = true;
    if (comp >= 0) counters_dirty[comp] = false;
    return hipSuccess;
}

// rows the tiled solve can take at all (dependencies per row), whatever the tile size
static bool tile_rows_ok(const TileSet &T) { return T.kmax <= (T.unit == 64 ? kTileShortRow : 4 * kTileLongJ); }

static bool tiles_fit(const TileSet &T, size_t budget = kTileLdsMax) {
    return tile_lds_bytes(T.max_rows, T.max_slots, T.max_pos, T.max_imps, T.kmax, 1, 8) <= budget &&
           T.max_slots + 1 <= 65535 && T.max_pos <= 32767 && tile_rows_ok(T);
}

// LDS budget of the default tile size.  Narrow levels (median under 256 rows) leave
// little parallelism per level, and large tiles -- fewer crossings -- win even at
// one block per CU; wide levels want three blocks per CU (64 KB).
static size_t default_tile_budget(const HostAnalysis &H) {
    std::vector<int32_t> sizes(H.n_levels);
    for (int32_t l = 0; l < H.n_levels; ++l) sizes[l] = H.level_ptr[l + 1] - H.level_ptr[l];
    if (sizes.empty()) return 65536;
    std::nth_element(sizes.begin(), sizes.begin() + sizes.size() / 2, sizes.end());
    return sizes[sizes.size() / 2] < 256 ? (size_t)kTileLdsMax : (size_t)65536;
}

// Default rows per tile of the tiled factor.  A tile's life is its rows' update
// work (each L entry of a row subtracts the dependency row's U part), and the
// factor runs fewer tiles at once than the solves, so tiles shrink from the
// solves' size by halves until they carry at most 8192 multiply-subtracts: 512
// rows for ILU(0) on a 7-point grid (about 9 per row), 128 for ILU(1) there
// (about 36).
static int32_t default_factor_rows(const HostAnalysis &H, int32_t tile_rows) {
    if (H.n == 0) return tile_rows;
    double work = 0.0;
    for (int32_t r = 0; r < H.n; ++r)
        for (int32_t p = H.lu_rp[r]; p < H.diag[r]; ++p) {
            const int32_t c = H.lu_ci[p];
            work += (double)(H.lu_rp[c + 1] - H.diag[c] - 1);
        }
    work /= H.n;
    constexpr double kTileWork = 8192.0;   // multiply-subtracts per tile: a 512-row tile of 7-point
                                           // ILU(0) does about 4600, one of ILU(1) about 18000
    int32_t rows = tile_rows;
    while (rows > 64 && (double)rows * work > kTileWork) rows /= 2;
    return rows;
}

// LDS slot of every position of a tiling (-1 for padding)
static std::vector<int16_t> position_slots(const TileSet &T) {
    std::vector<int16_t> pslot(T.row.size());
    for (int32_t t = 0; t < T.ntiles; ++t) {
        int32_t k = 0;
        for (int32_t q = T.ptr[t]; q < T.ptr[t + 1]; ++q) pslot[q] = (int16_t)(T.row[q] >= 0 ? k++ : -1);
    }
    return pslot;
}

ilu_status ilu_handle_s::make_tiles(int32_t rows, bool shrink) {
    spare_fwd = jv::TileSet();
    try {
        const size_t budget = default_tile_budget(H);
        // 3D grid boxes: the default size doubled (fewer crossings on the critical
        // path of both solves) when such a tile still fits a CU's LDS and the grid
        // makes a tile per CU and more; measured faster on 7-point ILU(0), two tiles
        // per CU, and on ILU(1), whose doubled tiles leave room for one.  The
        // doubled candidate is built beside the default one.
        const bool try_double = shrink && rows == kDefaultTileRows && (int64_t)H.n >= 256 * 2 * (int64_t)rows;
        TileSet t0, t1;
        std::vector<int32_t> sci2;
        int dim = 0, dim2 = 0;
        for (bool first = true;; first = false) {
            if (first && try_double)
                run_pair([&] { dim = build_tiles(H, rows, kTileShortRow, tile_lattice, &tiles[0], &tiles[1], &sci); },
                         [&] { dim2 = build_tiles(H, 2 * rows, kTileShortRow, tile_lattice, &t0, &t1, &sci2); });
            else
                dim = build_tiles(H, rows, kTileShortRow, tile_lattice, &tiles[0], &tiles[1], &sci);
            if (!shrink || rows <= 16 || (tiles_fit(tiles[0], budget) && tiles_fit(tiles[1], budget))) break;
            rows /= 2;
        }
        tiles_on_lattice = dim > 0;
        const size_t budget2 = (size_t)kTileLdsMax;
        if (try_double && dim == 3 && rows == kDefaultTileRows && dim2 == 3 && tiles_fit(t0, budget2) &&
            tiles_fit(t1, budget2)) {
            spare_fwd = std::move(tiles[0]);
            tiles[0] = std::move(t0);
            tiles[1] = std::move(t1);
            sci = std::move(sci2);
            rows *= 2;
        }
    } catch (const std::bad_alloc &) {
        return fail(ILU_ERR_NOMEM, "tiles: out of host memory");
    }
    tile_rows = rows;
    if (host_only) return make_factor_tiles();
    auto drop = [&](int32_t *&d) {
        if (d) {
            (void)hipFree(d);
            allocs_erase(this, d);
            d = nullptr;
        }
    };
    auto drop16 = [&](int16_t *&d) {
        if (d) {
            (void)hipFree(d);
            allocs_erase(this, d);
            d = nullptr;
        }
    };
    auto put = [&](int32_t *&d, const std::vector<int32_t> &v) -> hipError_t {
        drop(d);
        hipError_t e = upload(&d, v);
        if (e == hipSuccess && d) allocs.push_back(d);
        return e;
    };
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "tiles: synchronize");
    for (int dir = 0; dir < 2; ++dir) {
        const TileSet &T = tiles[dir];
        const std::vector<int16_t> pslot = position_slots(T);
        std::vector<int32_t> meta(T.rows.size() * 4);
        for (size_t i = 0; i < T.rows.size(); ++i) {
            const int32_t r = T.rows[i], d = H.diag[r];
            meta[4 * i] = r;
            meta[4 * i + 1] = dir == 0 ? H.lu_rp[r] : d + 1;
            meta[4 * i + 2] = dir == 0 ? d : H.lu_rp[r + 1];
            meta[4 * i + 3] = d;
        }
        DevTiles &D = dtiles[dir];
        drop16(D.pslot);
        if ((e = upload(&D.pslot, pslot)) != hipSuccess) return hip_fail(e, "tiles: upload");
        if (D.pslot) allocs.push_back(D.pslot);
        if ((e = put(D.ptr, T.ptr)) != hipSuccess ||
            (e = put(D.rows_ptr, T.rows_ptr)) != hipSuccess || (e = put(D.meta, meta)) != hipSuccess ||
            (e = put(D.imp_ptr, T.imp_ptr)) != hipSuccess || (e = put(D.imp, T.imp)) != hipSuccess)
            return hip_fail(e, "tiles: upload");
    }
    if ((e = put(d_sci, sci)) != hipSuccess) return hip_fail(e, "tiles: upload");
    return make_factor_tiles();
}

// The tiled factor needs the forward tiles, rows of at most kFactorMaxLanes
// entries and a tile image that fits LDS (the modified form's masks included).
ilu_status ilu_handle_s::make_factor_tiles() {
    ftiles_ok = false;
    arm_built = false;
    ftset_own = false;
    if (H.max_row_lu > kFactorMaxLanes || tiles[0].ntiles == 0) return ILU_OK;
    const int32_t lanes = H.max_row_lu <= 8 ? 8 : H.max_row_lu <= 16 ? 16 : 32;
    auto fits = [&](const TileSet &S) {
        build_factor_tiles(H, S, lanes, &ftiles);
        return ftiles.lds_need[3] <= (size_t)kFactorTileLdsMax;
    };
    try {
        // the solves' forward tiles unless another size is asked for; too large an
        // LDS image: a forward tiling of its own, halving the tile size
        const int32_t want = factor_rows > 0 ? factor_rows : default_factor_rows(H, tile_rows);
        bool ok = false;
        if (want == tile_rows) {
            ok = fits(tiles[0]);
        } else {
            // the same tiling as build_forward_tiles(want) when it was kept from make_tiles
            if (spare_fwd.ntiles > 0 && spare_fwd.cap == want)
                ftset = spare_fwd;
            else
                build_forward_tiles(H, want, kTileShortRow, tile_lattice, &ftset);
            ok = ftset_own = fits(ftset);
        }
        for (int32_t rows = want / 2; !ok && rows >= 16; rows /= 2) {
            build_forward_tiles(H, rows, kTileShortRow, tile_lattice, &ftset);
            ok = fits(ftset);
            ftset_own = ok;
        }
        if (!ok) return ILU_OK;
    } catch (const std::bad_alloc &) {
        return fail(ILU_ERR_NOMEM, "factor tiles: out of host memory");
    }
    if (host_only) {
        ftiles_ok = true;
        return ILU_OK;
    }
    auto drop = [&](auto *&d) {
        if (d) {
            (void)hipFree(d);
            allocs_erase(this, d);
            d = nullptr;
        }
    };
    auto put = [&](auto *&d, const auto &v) -> hipError_t {
        drop(d);
        hipError_t e = upload(&d, v);
        if (e == hipSuccess && d) allocs.push_back(d);
        return e;
    };
    hipError_t e;
    {   // the U parts other tiles import (diagonal entry, length), once each
        std::vector<std::pair<int32_t, int32_t>> ranges;
        for (size_t i = 0; i + 3 < ftiles.imp.size(); i += 4) ranges.push_back({ftiles.imp[i], ftiles.imp[i + 1]});
        std::sort(ranges.begin(), ranges.end());
        ranges.erase(std::unique(ranges.begin(), ranges.end()), ranges.end());
        std::vector<int32_t> flat;
        flat.reserve(2 * ranges.size());
        for (const auto &r : ranges) {
            flat.push_back(r.first);
            flat.push_back(r.second);
        }
        if ((e = put(d_arm, flat)) != hipSuccess) return hip_fail(e, "factor tiles: upload");
        n_arm = (int32_t)ranges.size();
        arm_built = true;
    }
    if ((e = put(dft.hdr, ftiles.hdr)) != hipSuccess || (e = put(dft.blob, ftiles.blob)) != hipSuccess ||
        (e = put(dft.vsrc, ftiles.vsrc)) != hipSuccess || (e = put(dft.cmask, ftiles.cmask)) != hipSuccess)
        return hip_fail(e, "factor tiles: upload");
    ftiles_ok = true;
    return ILU_OK;
}

ilu_status ilu_handle_s::make_tail(int32_t min_rows) {
    constexpr int32_t kTailMinLevels = 64;
    try {
        build_tail(H, 0, min_rows, kTailMinLevels, &tail[0]);
        build_tail(H, 1, min_rows, kTailMinLevels, &tail[1]);
    } catch (const std::bad_alloc &) {
        return fail(ILU_ERR_NOMEM, "tail: out of host memory");
    }
    tail_min_rows = min_rows;
    if (host_only) return make_factor_tail();
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "tail: synchronize");
    for (int d = 0; d < 2; ++d) {
        for (int32_t **pp : {&dtail[d].hdr, &dtail[d].rec}) {
            if (*pp) {
                (void)hipFree(*pp);
                allocs_erase(this, *pp);
                *pp = nullptr;
            }
        }
        if (tail[d].nsteps == 0) continue;
        if ((e = upload(&dtail[d].hdr, tail[d].hdr)) != hipSuccess || (e = upload(&dtail[d].rec, tail[d].rec)) != hipSuccess)
            return hip_fail(e, "tail: upload");
        if (dtail[d].hdr) allocs.push_back(dtail[d].hdr);
        if (dtail[d].rec) allocs.push_back(dtail[d].rec);
    }
    return make_factor_tail();
}

// The factor's lower stage follows the forward solve's tail.
ilu_status ilu_handle_s::make_factor_tail() {
    ftail_ok = false;
    try {
        ftail_ok = build_factor_tail(H, tail[0], &ftail);
    } catch (const std::bad_alloc &) {
        return fail(ILU_ERR_NOMEM, "factor tail: out of host memory");
    }
    if (host_only) return ILU_OK;
    auto drop = [&](auto *&d) {
        if (d) {
            (void)hipFree(d);
            allocs_erase(this, d);
            d = nullptr;
        }
    };
    drop(dftail.hdr);
    drop(dftail.rows);
    drop(dftail.lsrc);
    drop(dftail.match);
    drop(dftail.lmap);
    if (!ftail_ok) return ILU_OK;
    hipError_t e;
    auto put = [&](auto *&d, const auto &v) -> hipError_t {
        hipError_t r = upload(&d, v);
        if (r == hipSuccess && d) allocs.push_back(d);
        return r;
    };
    if ((e = put(dftail.hdr, ftail.hdr)) != hipSuccess || (e = put(dftail.rows, ftail.rows)) != hipSuccess ||
        (e = put(dftail.lsrc, ftail.lsrc)) != hipSuccess || (e = put(dftail.match, ftail.match)) != hipSuccess ||
        (e = put(dftail.lmap, ftail.lmap)) != hipSuccess) {
        ftail_ok = false;
        return hip_fail(e, "factor tail: upload");
    }
    return ILU_OK;
}

// XCC ids present on the current device (one probe per process): id -> stream
static hipError_t xcc_streams(std::vector<int8_t> *map, int *nstreams) {
    static std::vector<int8_t> cached;
    static int cached_n = 0;
    if (!cached_n) {
        const int blocks = 512;
        std::vector<int32_t> ids(blocks);
        hipError_t e = probe_xcc_ids(blocks, ids.data());
        if (e != hipSuccess) return e;
        std::vector<int8_t> m(16, -1);
        int n = 0;
        for (int id = 0; id < 16; ++id)
            if (std::find(ids.begin(), ids.end(), id) != ids.end()) m[id] = (int8_t)n++;
        if (n < 1 || n > kStreams) {
            std::fill(m.begin(), m.end(), 0);
            n = 1;
        }
        for (auto &v : m)
            if (v < 0) v = 0;   // ids never seen share stream 0
        cached = m;
        cached_n = n;
    }
    *map = cached;
    *nstreams = cached_n;
    return hipSuccess;
}

// -------------------------------------------------------------------------------------
// Analysis
// -------------------------------------------------------------------------------------

static ilu_status finish_analysis(ilu_handle_s *h) {
    HostAnalysis &H = h->H;
    hipError_t e;
#define UPLOAD_ONE(dst, src)                                                   \
    do {                                                                       \
        if ((e = upload(&dst, src)) != hipSuccess) return hip_fail(e, "upload " #src); \
        if (dst) h->allocs.push_back(dst);                                     \
    } while (0)
#define UP(dst, src)                                                   \
    do {                                                               \
        if ((e = upload(&dst, src)) != hipSuccess) return hip_fail(e, "upload " #src); \
        if (dst) h->allocs.push_back(dst);                             \
    } while (0)
    UP(h->d_in_rp, H.in_rp);
    UP(h->d_perm, H.perm);
    UP(h->d_lu_rp, H.lu_rp);
    UP(h->d_lu_ci, H.lu_ci);
    UP(h->d_diag, H.diag);
    UP(h->d_lu_src, H.lu_src);
    UP(h->d_flev, H.flev);
    UP(h->d_b_rp, H.b_rp);
    UP(h->d_b_ci, H.b_ci);
    UP(h->d_b_src, H.b_src);
    UP(h->d_ulevel_rows, H.ulevel_rows);
    UP(h->d_t_rp, H.t_rp);
    UP(h->d_t_ci, H.t_ci);
    UP(h->d_t_map, H.t_map);
    UP(h->d_t_diag, H.t_diag);
    UP(h->d_tlevel_rows, H.tlevel_rows);
    UP(h->d_tulevel_rows, H.tulevel_rows);
#undef UP
    const size_t nz = H.lu_rp[H.n];
    void *p;
    if ((e = h->alloc_bytes(&p, nz * 8)) != hipSuccess) return hip_fail(e, "alloc factor");
    h->d_lu = (double *)p;
    if ((e = h->alloc_bytes(&p, (size_t)H.b_rp[H.n] * 8)) != hipSuccess) return hip_fail(e, "alloc spmv values");
    h->d_bval = (double *)p;
    if ((e = h->alloc_bytes(&p, (size_t)H.n * 8)) != hipSuccess) return hip_fail(e, "alloc row tau");
    h->d_row_tau = (double *)p;
    if ((e = h->alloc_bytes(&p, kInfoSlots * 4)) != hipSuccess) return hip_fail(e, "alloc info");
    h->d_info = (int32_t *)p;
    if ((e = hipMemset(h->d_info, 0, kInfoSlots * 4)) != hipSuccess) return hip_fail(e, "zero info");
    if ((e = h->alloc_bytes(&p, kDotWorkBytes)) != hipSuccess) return hip_fail(e, "alloc dot work");
    h->d_dotwork = (double *)p;
    const size_t cbytes = (size_t)kPasses * kStreams * kCounterStride * 4;
    if ((e = h->alloc_bytes(&p, cbytes)) != hipSuccess) return hip_fail(e, "alloc counters");
    h->d_counters = (int32_t *)p;
    if ((e = hipMemset(h->d_counters, 0, cbytes)) != hipSuccess) return hip_fail(e, "zero counters");
    // the permuted copy of A has the factor's pattern when there is no fill (the
    // tiled factor then writes its values)
    h->b_same = H.b_rp == H.lu_rp && H.b_ci == H.lu_ci;
    std::vector<int8_t> xmap;
    if ((e = xcc_streams(&xmap, &h->nstreams)) != hipSuccess) return hip_fail(e, "xcc probe");
    UPLOAD_ONE(h->d_xcc_stream, xmap);
    // LDS staging of the factor: the dependency rows' upper parts, summed per row
    int64_t tcap = 0;
    for (int32_t r = 0; r < H.n; ++r) {
        int64_t t = 0;
        for (int32_t q = H.lu_rp[r]; q < H.diag[r]; ++q) {
            const int32_t c = H.lu_ci[q];
            t += H.lu_rp[c + 1] - H.diag[c];
        }
        tcap = std::max(tcap, t);
    }
    h->factor_tcap = (int32_t)std::min<int64_t>(tcap, 1 << 20);
    h->lanes_factor = pow2_lanes(H.max_row_lu, 4, 64);
    h->lanes_solve = pow2_lanes(std::max(H.max_lower_lu, H.max_upper_lu), 4, 64);
    // spmv: rows longer than one wave go to a one-wave-per-row pass; the rest take one
    // lane per row when they average at most 8 entries (every load of a row in
    // flight at once), else a lane group of half their mean length, rounded up to a
    // power of two (two entries per lane)
    {
        constexpr int32_t kHeavy = 64;
        std::vector<int32_t> heavy;
        int64_t light_nnz = 0;
        for (int32_t r = 0; r < H.n; ++r) {
            const int32_t len = H.b_rp[r + 1] - H.b_rp[r];
            if (len > kHeavy) heavy.push_back(r);
            else light_nnz += len;
        }
        const int64_t light_rows = std::max<int64_t>(1, H.n - (int64_t)heavy.size());
        const int64_t mean = std::max<int64_t>(1, (light_nnz + light_rows - 1) / light_rows);
        h->lanes_spmv = mean <= 8 ? 1 : std::max(4, pow2_lanes((int)mean, 4, 64) / 2);
        if (!heavy.empty()) {
            UPLOAD_ONE(h->d_spmv_heavy, heavy);
            h->n_spmv_heavy = (int32_t)heavy.size();
            h->spmv_heavy_min = kHeavy;
        }
        // with long rows, the nnz-balanced pass (every row must hold an entry)
        bool nonempty = true;
        for (int32_t r = 0; r < H.n && nonempty; ++r) nonempty = H.b_rp[r + 1] > H.b_rp[r];
        const int64_t nnzb = H.b_rp[H.n];
        if (!heavy.empty() && nonempty && nnzb > 0) {
            const int32_t nw = (int32_t)((nnzb + kNzWave - 1) / kNzWave);
            std::vector<int32_t> wrow(nw), span;
            std::vector<uint16_t> bits((size_t)(nw + 1) * 64, 0);
            for (int32_t r = 0; r < H.n; ++r) {
                const int32_t p = H.b_rp[r];
                bits[p / kNzLane] |= (uint16_t)(1u << (p % kNzLane));
                const int32_t w0 = p / kNzWave, w1 = (H.b_rp[r + 1] - 1) / kNzWave;
                if (w1 > w0) span.insert(span.end(), {r, w0, w1});
            }
            for (int32_t w = 0, r = 0; w < nw; ++w) {
                while (H.b_rp[r + 1] <= (int64_t)w * kNzWave) ++r;
                wrow[w] = r;
            }
            UPLOAD_ONE(h->d_nz_wrow, wrow);
            UPLOAD_ONE(h->d_nz_bits, bits);
            if (!span.empty()) UPLOAD_ONE(h->d_nz_span, span);
            void *pp = nullptr;
            if ((e = h->alloc_bytes(&pp, (size_t)2 * nw * sizeof(double))) != hipSuccess)
                return hip_fail(e, "spmv pieces");
            h->d_nz_part = (double *)pp;
            h->nz_waves = nw;
            h->nz_nspan = (int32_t)(span.size() / 3);
            // by default only for rows so long that one wave per row would walk
            // them for more than 64 rounds (the autotuner times both)
            int32_t longest = 0;
            for (int32_t r = 0; r < H.n; ++r) longest = std::max(longest, H.b_rp[r + 1] - H.b_rp[r]);
            h->spmv_nz = longest > 4 * kNzWave;
        }
    }
#undef UPLOAD_ONE
    return ILU_OK;
}

extern "C" ilu_status ilu_analyze(const ilu_csr *A, const ilu_analyze_opts *opts, ilu_handle *out) {
    if (!A || !out) return fail(ILU_ERR_ARG, "ilu_analyze: NULL argument");
    *out = nullptr;
    ilu_analyze_opts o{};
    if (opts) o = *opts;
    for (int i = 0; i < 2; ++i)
        if (o.reserved[i]) return fail(ILU_ERR_ARG, "ilu_analyze: reserved option fields must be 0");
    if (o.tail_min_rows < 0 || o.tail_min_rows > 65536)
        return fail(ILU_ERR_ARG, "ilu_analyze: tail_min_rows must be in [0, 65536]");
    if (o.tile_rows != 0 && (o.tile_rows < 16 || o.tile_rows > 65536))
        return fail(ILU_ERR_ARG, "ilu_analyze: tile_rows must be 0 or in [16, 65536]");
    if (o.host_only != 0 && o.host_only != 1) return fail(ILU_ERR_ARG, "ilu_analyze: host_only must be 0 or 1");
    if (A->n <= 0 || A->n >= (1 << 30)) return fail(ILU_ERR_ARG, "ilu_analyze: n must be in [1, 2^30)");
    std::unique_ptr<ilu_handle_s> h(new (std::nothrow) ilu_handle_s());
    if (!h) return fail(ILU_ERR_NOMEM, "ilu_analyze: out of host memory");
    std::string err;
    ilu_status st;
    try {
        st = analyze_host(A->n, A->row_ptr, A->col_idx, A->nnz, o.k_max, o.pattern, o.ordering, &h->H, &err);
    } catch (const std::bad_alloc &) {
        return fail(ILU_ERR_NOMEM, "ilu_analyze: out of host memory");
    }
    if (st != ILU_OK) return fail(st, err);
    h->row_off = {0, (int64_t)A->n};
    h->nnz_off = {0, A->nnz};
    h->host_only = o.host_only != 0;
    h->pattern_sym = h->H.t_rp == h->H.lu_rp && h->H.t_ci == h->H.lu_ci;
    if (!h->host_only && (st = finish_analysis(h.get())) != ILU_OK) return st;
    if ((st = h->make_tiles(o.tile_rows ? o.tile_rows : kDefaultTileRows, o.tile_rows == 0)) != ILU_OK) return st;
    if ((st = h->make_tail(o.tail_min_rows)) != ILU_OK) return st;
    // the solves default to the tiled launch wherever the tiles fit LDS
    h->sched_solve = tiles_fit(h->tiles[0]) && tiles_fit(h->tiles[1]) ? ILU_SCHED_TILED : ILU_SCHED_SYNCFREE;
    h->sched_factor = h->ftiles_ok ? ILU_SCHED_TILED : ILU_SCHED_SYNCFREE;
    *out = h.release();
    return ILU_OK;
}

extern "C" ilu_status ilu_analyze_batched(int32_t count, const ilu_csr *As, const ilu_analyze_opts *opts,
                                          ilu_handle *out) {
    if (!As || !out || count <= 0) return fail(ILU_ERR_ARG, "ilu_analyze_batched: bad arguments");
    *out = nullptr;
    ilu_analyze_opts o{};
    if (opts) o = *opts;
    if (o.ordering != ILU_ORDER_NATURAL)
        return fail(ILU_ERR_UNSUPPORTED, "ilu_analyze_batched: a preordering would mix the matrices' rows");
    std::vector<int64_t> roff(count + 1, 0), zoff(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        if (As[i].n <= 0 || !As[i].row_ptr || !As[i].col_idx) return fail(ILU_ERR_ARG, "ilu_analyze_batched: bad matrix");
        roff[i + 1] = roff[i] + As[i].n;
        zoff[i + 1] = zoff[i] + As[i].nnz;
    }
    if (roff[count] >= (1 << 30) || zoff[count] >= ((int64_t)1 << 31) - roff[count])
        return fail(ILU_ERR_UNSUPPORTED, "ilu_analyze_batched: batch too large for int32 indices");
    std::vector<int32_t> rp((size_t)roff[count] + 1), ci((size_t)zoff[count]);
    rp[0] = 0;
    for (int i = 0; i < count; ++i) {
        const ilu_csr &M = As[i];
        if (M.row_ptr[0] != 0 || M.row_ptr[M.n] != M.nnz)
            return fail(ILU_ERR_CSR, "ilu_analyze_batched: matrix " + std::to_string(i) + " row_ptr inconsistent");
        for (int32_t r = 0; r < M.n; ++r) rp[roff[i] + r + 1] = (int32_t)(zoff[i] + M.row_ptr[r + 1]);
        for (int64_t p = 0; p < M.nnz; ++p) {
            if (M.col_idx[p] < 0 || M.col_idx[p] >= M.n)
                return fail(ILU_ERR_CSR, "ilu_analyze_batched: matrix " + std::to_string(i) + " column out of range");
            ci[zoff[i] + p] = (int32_t)(M.col_idx[p] + roff[i]);
        }
    }
    ilu_csr big{(int32_t)roff[count], zoff[count], rp.data(), ci.data()};
    ilu_status st = ilu_analyze(&big, &o, out);
    if (st != ILU_OK) return st;
    (*out)->row_off = roff;
    (*out)->nnz_off = zoff;
    (*out)->batch_count = count;
    return ILU_OK;
}

extern "C" ilu_status ilu_batch_offsets(ilu_handle h, int64_t *row_off, int64_t *nnz_off) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_batch_offsets: NULL handle");
    if (row_off) std::copy(h->row_off.begin(), h->row_off.end(), row_off);
    if (nnz_off) std::copy(h->nnz_off.begin(), h->nnz_off.end(), nnz_off);
    return ILU_OK;
}

extern "C" ilu_status ilu_get_info(ilu_handle h, ilu_info *out) {
    if (!h || !out) return fail(ILU_ERR_ARG, "ilu_get_info: NULL argument");
    const HostAnalysis &H = h->H;
    ilu_info I{};
    I.n = H.n;
    I.n_levels = H.n_levels;
    I.n_ulevels = H.n_ulevels;
    I.max_row_lu = H.max_row_lu;
    I.nnz_a = H.nnz_in;
    I.nnz_lu = H.lu_rp[H.n];
    I.nnz_b = H.b_rp[H.n];
    std::vector<int32_t> sizes(H.n_levels);
    for (int l = 0; l < H.n_levels; ++l) sizes[l] = H.level_ptr[l + 1] - H.level_ptr[l];
    std::sort(sizes.begin(), sizes.end());
    I.level_min = sizes.front();
    I.level_max = sizes.back();
    const size_t m = sizes.size();
    I.level_median = (m % 2) ? sizes[m / 2] : 0.5 * ((double)sizes[m / 2 - 1] + sizes[m / 2]);
    I.batch_count = h->batch_count;
    I.n_tiles = h->tiles[0].ntiles;
    I.n_utiles = h->tiles[1].ntiles;
    I.tile_rows = h->tile_rows;
    I.max_tile = std::max(h->tiles[0].max_rows, h->tiles[1].max_rows);
    I.tail_rows = h->tail[0].nsteps ? H.n - h->tail[0].pos0 : 0;
    I.tail_urows = h->tail[1].nsteps ? H.n - h->tail[1].pos0 : 0;
    *out = I;
    return ILU_OK;
}

extern "C" ilu_status ilu_copy_schedule(ilu_handle h, int32_t *level_ptr, int32_t *perm, int32_t *lu_row_ptr,
                                        int32_t *lu_col_idx, int32_t *diag_pos, int32_t *ulevel_ptr,
                                        int32_t *ulevel_rows, int8_t *fill_lev, int32_t *lu_src,
                                        int32_t *b_row_ptr, int32_t *b_col_idx) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_copy_schedule: NULL handle");
    const HostAnalysis &H = h->H;
    auto cp = [](auto *dst, const auto &v) {
        if (dst) std::copy(v.begin(), v.end(), dst);
    };
    cp(level_ptr, H.level_ptr);
    cp(perm, H.perm);
    cp(lu_row_ptr, H.lu_rp);
    cp(lu_col_idx, H.lu_ci);
    cp(diag_pos, H.diag);
    cp(ulevel_ptr, H.ulevel_ptr);
    cp(ulevel_rows, H.ulevel_rows);
    cp(fill_lev, H.flev);
    cp(lu_src, H.lu_src);
    cp(b_row_ptr, H.b_rp);
    cp(b_col_idx, H.b_ci);
    return ILU_OK;
}

extern "C" ilu_status ilu_copy_tiles(ilu_handle h, int32_t dir, int32_t *tile_ptr, int32_t *tile_row, int32_t *sci) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_copy_tiles: NULL handle");
    if (dir != 0 && dir != 1) return fail(ILU_ERR_ARG, "ilu_copy_tiles: dir must be 0 or 1");
    const TileSet &T = h->tiles[dir];
    if (tile_ptr) std::copy(T.ptr.begin(), T.ptr.end(), tile_ptr);
    if (tile_row) std::copy(T.row.begin(), T.row.end(), tile_row);
    if (sci) std::copy(h->sci.begin(), h->sci.end(), sci);
    return ILU_OK;
}

extern "C" ilu_status ilu_copy_tail(ilu_handle h, int32_t dir, int32_t *sizes, int32_t *hdr, int32_t *rec) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_copy_tail: NULL handle");
    if (dir != 0 && dir != 1) return fail(ILU_ERR_ARG, "ilu_copy_tail: dir must be 0 or 1");
    const TailPlan &T = h->tail[dir];
    if (sizes) {
        sizes[0] = T.level0;
        sizes[1] = T.pos0;
        sizes[2] = T.nsteps;
        sizes[3] = (int32_t)T.rec.size();
    }
    if (hdr) std::copy(T.hdr.begin(), T.hdr.end(), hdr);
    if (rec) std::copy(T.rec.begin(), T.rec.end(), rec);
    return ILU_OK;
}

extern "C" ilu_status ilu_copy_factor_tail(ilu_handle h, int32_t *sizes, int32_t *hdr, int32_t *rows, int32_t *lsrc,
                                           uint8_t *match, uint8_t *lmap) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_copy_factor_tail: NULL handle");
    const FactorTailPlan &T = h->ftail;
    const bool ok = h->ftail_ok;
    if (sizes) {
        const int32_t v[10] = {ok ? T.level0 : -1, ok ? T.pos0 : 0, ok ? T.nsteps : 0, ok ? T.umax : 0,
                               ok ? T.ring_rows : 0, ok ? T.q : 0, ok ? (int32_t)(T.rows.size() / 8) : 0,
                               ok ? (int32_t)T.lsrc.size() : 0, ok ? (int32_t)T.match.size() : 0,
                               ok ? (int32_t)T.lmap.size() : 0};
        std::copy(v, v + 10, sizes);
    }
    if (!ok) return ILU_OK;
    if (hdr) std::copy(T.hdr.begin(), T.hdr.end(), hdr);
    if (rows) std::copy(T.rows.begin(), T.rows.end(), rows);
    if (lsrc) std::copy(T.lsrc.begin(), T.lsrc.end(), lsrc);
    if (match) std::copy(T.match.begin(), T.match.end(), match);
    if (lmap) std::copy(T.lmap.begin(), T.lmap.end(), lmap);
    return ILU_OK;
}

// -------------------------------------------------------------------------------------
// Factor
// -------------------------------------------------------------------------------------

extern "C" ilu_status ilu_factor(ilu_handle h, const double *a_val, int32_t k, double tau, int32_t casts,
                                 ilu_factor_info *info, hipStream_t s) {
    if (!h) return fail(ILU_ERR_STATE, "ilu_factor: no analysis (NULL handle)");
    if (h->host_only) return fail(ILU_ERR_STATE, "ilu_factor: host-only analysis");
    if (!a_val && h->H.nnz_in > 0) return fail(ILU_ERR_ARG, "ilu_factor: NULL values");
    if (k < 0 || k > h->H.k_max) return fail(ILU_ERR_ARG, "ilu_factor: k must be in [0, k_max]");
    if (!(tau >= 0.0)) return fail(ILU_ERR_ARG, "ilu_factor: tau must be >= 0");
    if (casts & ~(ILU_CAST_F32 | ILU_CAST_BF16 | ILU_FACTOR_MODIFIED))
        return fail(ILU_ERR_ARG, "ilu_factor: unknown flag bits");
    const bool milu = (casts & ILU_FACTOR_MODIFIED) != 0;
    const HostAnalysis &H = h->H;
    if (H.max_row_lu > kFactorLongMax)
        return fail(ILU_ERR_UNSUPPORTED, "ilu_factor: factor rows longer than 4096 entries are not supported");
    // rows longer than 64 entries: one wave per row with the row in LDS
    const bool long_rows = H.max_row_lu > 64;
    const int lanes = long_rows ? 64 : h->lanes_factor;
    const bool sf = h->sched_factor != ILU_SCHED_LEVEL;
    hipError_t e;
    h->factored = false;
    if (info) {
        info->bad_row = info->bad_row_original = info->bad_matrix = -1;
        info->n_dropped = 0;
    }
    const bool use_tau = tau > 0.0;
    // the lower stage (a tail set, plain ILU(k) at k = k_max, rows of at most 64
    // entries): the rows before the tail sync-free, the tail streamed
    const bool stream = h->factor_lower && h->ftail_ok && h->tail_min_rows > 0 && k == H.k_max && !use_tau &&
                        !milu && !long_rows;
    // the tiled factor covers ILU(k, tau), plain or modified, at k = k_max (no
    // absent entries); anything else runs the sync-free factor
    const bool tiled = !stream && h->sched_factor == ILU_SCHED_TILED && h->ftiles_ok && k == H.k_max;
    // storage copies are allocated before the first launch of the call
    void *p;
    if ((casts & ILU_CAST_F32) && !h->d_lu32) {
        if ((e = h->alloc_bytes(&p, (size_t)H.lu_rp[H.n] * 4)) != hipSuccess) return hip_fail(e, "alloc f32");
        h->d_lu32 = (float *)p;
    }
    if ((casts & ILU_CAST_BF16) && !h->d_lu16) {
        if ((e = h->alloc_bytes(&p, (size_t)H.lu_rp[H.n] * 2)) != hipSuccess) return hip_fail(e, "alloc bf16");
        h->d_lu16 = (uint16_t *)p;
    }
    int32_t *tile_counter = h->d_counters + (size_t)kPassFactorTile * kStreams * kCounterStride;
    const int pcall = h->prof.begin(ILU_STAGE_FACTOR_CALL, s);
    // an apply that timed out and was never reported leaves its intermediates
    // half published: the prologue re-arms them before the abort flag is cleared,
    // resets the status slots and the tiled factor's claim counter
    if ((e = launch_factor_prologue(h->d_info, (uint64_t *)h->y64, (uint64_t *)h->z64, (int64_t)H.n * h->cap64,
                                    (uint32_t *)h->y32, (uint32_t *)h->z32, (int64_t)H.n * h->cap32,
                                    tiled ? tile_counter : nullptr, s)) != hipSuccess)
        return hip_fail(e, "ilu_factor: prologue");

    if (use_tau && (e = launch_row_tau(H.n, h->d_in_rp, a_val, h->d_perm, tau, h->d_row_tau, s)) != hipSuccess)
        return hip_fail(e, "ilu_factor: row tau");
    FactorArgs A{};
    A.n = H.n;
    A.rp = h->d_lu_rp;
    A.ci = h->d_lu_ci;
    A.diag = h->d_diag;
    A.src = h->d_lu_src;
    A.flev = h->d_flev;
    A.k = k;
    A.use_flev = k < H.k_max;
    A.use_tau = use_tau;
    A.milu = milu;
    A.a = a_val;
    A.lu = h->d_lu;
    A.row_tau = h->d_row_tau;
    A.info = h->d_info;
    A.tcap = (h->factor_staged && factor_lds_bytes(lanes, h->factor_tcap)) ? h->factor_tcap : 0;
    A.max_lower = H.max_lower_lu;
    A.lcap = long_rows ? H.max_row_lu : 0;
    if (stream) {
        if ((e = launch_fill_u64((uint64_t *)h->d_lu, kPending64, H.lu_rp[H.n], s)) != hipSuccess)
            return hip_fail(e, "ilu_factor: arm");
        const int pp_ = h->prof.begin(ILU_STAGE_FACTOR, s);
        if (h->ftail.level0 > 0) {
            const TaskList *tl = h->task_list(kTasksForward, lanes, h->ftail.level0);
            if (!tl) return fail(ILU_ERR_NOMEM, "ilu_factor: task list");
            if ((e = h->prepare_claims(kPassFactor, tl, &A.claims, s)) != hipSuccess)
                return hip_fail(e, "ilu_factor: claims");
            A.nstreams = h->nstreams;
            A.poll_sleep = h->poll_sleep;
            if ((e = launch_factor(A, lanes, true, h->grid_syncfree(tl), s)) != hipSuccess)
                return hip_fail(e, "ilu_factor: upper stage");
        }
        FactorStreamArgs F{};
        F.hdr = reinterpret_cast<const int4 *>(h->dftail.hdr);
        F.rows = reinterpret_cast<const int4 *>(h->dftail.rows);
        F.lsrc = h->dftail.lsrc;
        F.match = h->dftail.match;
        F.lmap = h->dftail.lmap;
        F.nsteps = h->ftail.nsteps;
        F.q = h->ftail.q;
        A.poll_sleep = h->poll_sleep;
        e = launch_factor_stream(A, F, s);
        h->prof.end(pp_, s);
        if (e != hipSuccess) return hip_fail(e, "ilu_factor: lower stage");
    } else if (tiled) {
        const TileSet &T0 = h->ftset_own ? h->ftset : h->tiles[0];
        FactorTileArgs T{};
        T.hdr = h->dft.hdr;
        T.blob = reinterpret_cast<const int4 *>(h->dft.blob);
        T.vsrc = h->dft.vsrc;
        T.cmask = h->dft.cmask;
        T.ntiles = T0.ntiles;
        T.lds_bytes = (int32_t)h->ftiles.lds_need[(use_tau ? 1 : 0) + (milu ? 2 : 0)];
        T.counter = tile_counter;
        A.poll_sleep = h->poll_sleep;
        // only U parts that other tiles import are polled: arm just those
        e = h->arm_built ? launch_arm_ranges((uint64_t *)h->d_lu, reinterpret_cast<const int2 *>(h->d_arm), h->n_arm, s)
                     : launch_fill_u64((uint64_t *)h->d_lu, kPending64, H.lu_rp[H.n], s);
        if (e != hipSuccess) return hip_fail(e, "ilu_factor: arm");
        // the storage copies are written as each row is published, the spmv
        // operand as the rows' input values are staged
        A.lu32 = (casts & ILU_CAST_F32) ? h->d_lu32 : nullptr;
        A.lu16 = (casts & ILU_CAST_BF16) ? h->d_lu16 : nullptr;
        A.bval = h->b_same ? h->d_bval : nullptr;
        const int pp_ = h->prof.begin(ILU_STAGE_FACTOR, s);
        e = launch_factor_tiled(A, T, h->ftiles.lanes, s);
        h->prof.end(pp_, s);
        if (e != hipSuccess) return hip_fail(e, "ilu_factor: tiled launch");
    } else if (sf) {
        const TaskList *tl = h->task_list(kTasksForward, lanes);
        if (!tl) return fail(ILU_ERR_NOMEM, "ilu_factor: task list");
        if ((e = launch_fill_u64((uint64_t *)h->d_lu, kPending64, H.lu_rp[H.n], s)) != hipSuccess)
            return hip_fail(e, "ilu_factor: arm");
        if ((e = h->prepare_claims(kPassFactor, tl, &A.claims, s)) != hipSuccess) return hip_fail(e, "ilu_factor: claims");
        A.nstreams = h->nstreams;
        A.poll_sleep = h->poll_sleep;
        const int pp_ = h->prof.begin(ILU_STAGE_FACTOR, s);
        e = long_rows ? launch_factor_long(A, true, h->grid_syncfree(tl), s)
                      : launch_factor(A, lanes, true, h->grid_syncfree(tl), s);
        h->prof.end(pp_, s);
        if (e != hipSuccess) return hip_fail(e, "ilu_factor: launch");
    } else {
        const int pp_ = h->prof.begin(ILU_STAGE_FACTOR, s);
        for (int l = 0; l < H.n_levels; ++l) {
            A.row_begin = H.level_ptr[l];
            A.row_end = H.level_ptr[l + 1];
            e = long_rows ? launch_factor_long(A, false, 0, s) : launch_factor(A, lanes, false, 0, s);
            if (e != hipSuccess) return hip_fail(e, "ilu_factor: launch");
        }
        h->prof.end(pp_, s);
    }
    h->tracked = use_tau || A.use_flev;
    if (h->tracked) {
        if (!h->d_stat) {
            void *p;
            if ((e = h->alloc_bytes(&p, (size_t)H.lu_rp[H.n])) != hipSuccess) return hip_fail(e, "alloc state");
            h->d_stat = (int8_t *)p;
        }
        if ((e = launch_factor_fixup(H.lu_rp[H.n], h->d_lu, h->d_flev, k, A.use_flev, h->d_stat, h->d_info, s)) !=
            hipSuccess)
            return hip_fail(e, "ilu_factor: fixup");
    }
    if ((!tiled || !h->b_same) && (e = launch_gather(H.b_rp[H.n], h->d_b_src, a_val, h->d_bval, s)) != hipSuccess)
        return hip_fail(e, "ilu_factor: spmv values");
    h->bvals = true;
    if (!tiled && (casts & ILU_CAST_F32) &&
        (e = launch_cast_f32(H.lu_rp[H.n], h->d_lu, h->d_lu32, s)) != hipSuccess)
        return hip_fail(e, "cast f32");
    if (!tiled && (casts & ILU_CAST_BF16) &&
        (e = launch_cast_bf16(H.lu_rp[H.n], h->d_lu, h->d_lu16, s)) != hipSuccess)
        return hip_fail(e, "cast bf16");
    h->prof.end(pcall, s);
    int32_t hinfo[kInfoSlots];
    if ((e = hipMemcpyAsync(hinfo, h->d_info, sizeof(hinfo), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "ilu_factor: info readback");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ilu_factor: synchronize");
    h->has32 = casts & 1;
    h->has16 = (casts & 2) != 0;
    h->k_used = k;
    h->tau_used = tau;
    h->flags_used = casts;
    int64_t dropped = 0;
    std::memcpy(&dropped, &hinfo[kInfoDropLo], 8);
    if (info) info->n_dropped = dropped;
    if (hinfo[kInfoAbort]) {
        (void)h->reset_info(s);
        (void)h->rearm(s);
        (void)hipStreamSynchronize(s);
        return fail(ILU_ERR_TIMEOUT, "ilu_factor: a dependency wait expired");
    }
    if (hinfo[kInfoBadKey] != INT_MAX) {
        const int row = hinfo[kInfoBadKey] >> 1;
        if (info) {
            info->bad_row = row;
            info->bad_row_original = H.perm[row];
            const int64_t orig = H.perm[row];
            info->bad_matrix =
                (int32_t)(std::upper_bound(h->row_off.begin(), h->row_off.end(), orig) - h->row_off.begin()) - 1;
        }
        h->factored = true;  // values exist (garbage after the failing row); callers see the status
        h->factor_ok = false;
        return fail((hinfo[kInfoBadKey] & 1) ? ILU_ERR_NONFINITE : ILU_ERR_ZERO_PIVOT,
                    std::string("ilu_factor: ") + ((hinfo[kInfoBadKey] & 1) ? "non-finite value" : "zero pivot") +
                        " in row " + std::to_string(row) + " (level order), " + std::to_string(H.perm[row]) +
                        " (input order)");
    }
    h->factored = true;
    h->factor_ok = true;
    return ILU_OK;
}

extern "C" ilu_status ilu_factor_values(ilu_handle h, int32_t prec, const void **dev_ptr) {
    if (!h || !dev_ptr) return fail(ILU_ERR_ARG, "ilu_factor_values: NULL argument");
    if (!h->factored) return fail(ILU_ERR_STATE, "ilu_factor_values: no factor");
    switch (prec) {
        case ILU_PREC_F64: *dev_ptr = h->d_lu; return ILU_OK;
        case ILU_PREC_F32:
            if (!h->has32) return fail(ILU_ERR_STATE, "ilu_factor_values: no FP32 copy");
            *dev_ptr = h->d_lu32;
            return ILU_OK;
        case ILU_PREC_BF16:
            if (!h->has16) return fail(ILU_ERR_STATE, "ilu_factor_values: no BF16 copy");
            *dev_ptr = h->d_lu16;
            return ILU_OK;
        default: return fail(ILU_ERR_ARG, "ilu_factor_values: unknown precision");
    }
}

extern "C" ilu_status ilu_copy_factor(ilu_handle h, double *lu_val, int8_t *state) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_copy_factor: NULL handle");
    if (!h->factored) return fail(ILU_ERR_STATE, "ilu_copy_factor: no factor");
    const size_t nz = h->H.lu_rp[h->H.n];
    hipError_t e;
    if (lu_val && (e = hipMemcpy(lu_val, h->d_lu, nz * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "ilu_copy_factor");
    if (state) {
        if (h->tracked) {
            if ((e = hipMemcpy(state, h->d_stat, nz, hipMemcpyDeviceToHost)) != hipSuccess)
                return hip_fail(e, "ilu_copy_factor");
        } else {
            std::memset(state, 0, nz);
        }
    }
    return ILU_OK;
}

extern "C" ilu_status ilu_copy_factor_prec(ilu_handle h, int32_t prec, void *host) {
    if (!h || !host) return fail(ILU_ERR_ARG, "ilu_copy_factor_prec: NULL argument");
    const void *src = nullptr;
    ilu_status st = ilu_factor_values(h, prec, &src);
    if (st != ILU_OK) return st;
    const size_t esz = prec == ILU_PREC_F64 ? 8 : (prec == ILU_PREC_F32 ? 4 : 2);
    hipError_t e = hipMemcpy(host, src, (size_t)h->H.lu_rp[h->H.n] * esz, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "ilu_copy_factor_prec");
    return ILU_OK;
}

// -------------------------------------------------------------------------------------
// Solves
// -------------------------------------------------------------------------------------

namespace jv {

// One forward + backward pass.  view: 0 = the factor (L then U), 1 = the
// transposed factor (U^T then L^T, adjoint).
ilu_status run_solves(ilu_handle_s *h, int view, const void *val, int prec, int vec, const void *b, void *x,
                      void *y_out, void *z_out, int nrhs, int64_t ld, int flags, hipStream_t s, const SolveWork *ws,
                      bool guard) {
    const HostAnalysis &H = h->H;
    const int pc = prec == ILU_PREC_F64 ? 0 : 1;
    hipError_t e;
    if (!ws && (e = h->ensure_workspace(nrhs, pc, s)) != hipSuccess) return hip_fail(e, "workspace");
    const int pcall = h->prof.begin(ILU_STAGE_APPLY_CALL, s);
    // an earlier apply that timed out: re-arm, clear and count it (reported by
    // ilu_get_status and the Krylov drivers)
    if (guard && (e = h->guard(s)) != hipSuccess) return hip_fail(e, "solve guard");
    if (ws && ws->fill) {
        // caller-provided intermediates start all pending
        const int64_t cnt = (int64_t)H.n * ws->cap;
        e = pc == 0 ? launch_fill_u64((uint64_t *)ws->y, kPending64, cnt, s)
                    : launch_fill_u32((uint32_t *)ws->y, kPending32, cnt, s);
        if (e == hipSuccess)
            e = pc == 0 ? launch_fill_u64((uint64_t *)ws->z, kPending64, cnt, s)
                        : launch_fill_u32((uint32_t *)ws->z, kPending32, cnt, s);
        if (e != hipSuccess) return hip_fail(e, "solve workspace fill");
    }
    if (h->force_abort) {
        h->force_abort = false;
        if ((e = launch_raise_abort(h->d_info, s)) != hipSuccess) return hip_fail(e, "raise abort");
    }
    // after a completed forward pass, an error leaves y published: re-arm it
    auto after_fwd = [&](ilu_status st, int pass) -> ilu_status {
        if (pass == 1) {
            if (ws) {
                const int64_t cnt = (int64_t)H.n * ws->cap;
                (void)(pc == 0 ? launch_fill_u64((uint64_t *)ws->y, kPending64, cnt, s)
                               : launch_fill_u32((uint32_t *)ws->y, kPending32, cnt, s));
            } else {
                (void)h->rearm(s);
            }
        }
        return st;
    };
    const bool sf = h->sched_solve != ILU_SCHED_LEVEL;
    const int lanes = h->lanes_solve;
    SolveArgs A{};
    A.n = H.n;
    A.val = val;
    A.perm = (flags & ILU_PERMUTED_SPACE) ? nullptr : h->d_perm;
    A.b = b;
    A.x = x;
    A.y = ws ? ws->y : (pc == 0 ? h->y64 : h->y32);
    A.z = ws ? ws->z : (pc == 0 ? h->z64 : h->z32);
    A.y_out = y_out;
    A.z_out = z_out;
    A.ld = ld;
    A.cap = ws ? ws->cap : (pc == 0 ? h->cap64 : h->cap32);
    A.nrhs = nrhs;
    A.info = h->d_info;
    for (int pass = 0; pass < 2; ++pass) {
        const bool fwd = pass == 0;
        int which;
        const std::vector<int32_t> *lptr;
        if (view == 0) {
            A.rp = h->d_lu_rp;
            A.ci = h->d_lu_ci;
            A.diag = h->d_diag;
            A.vmap = nullptr;
            A.rows = fwd ? nullptr : h->d_ulevel_rows;
            A.unit_diag = fwd ? 1 : 0;
            which = fwd ? kTasksForward : kTasksBackward;
            lptr = fwd ? &H.level_ptr : &H.ulevel_ptr;
        } else {
            A.rp = h->d_t_rp;
            A.ci = h->d_t_ci;
            A.diag = h->d_t_diag;
            A.vmap = h->d_t_map;
            A.rows = fwd ? h->d_tlevel_rows : h->d_tulevel_rows;
            A.unit_diag = fwd ? 0 : 1;
            which = fwd ? kTasksTForward : kTasksTBackward;
            lptr = fwd ? &H.tlevel_ptr : &H.tulevel_ptr;
        }
        // a lower stage: the levels before it sync-free (or one launch per level),
        // then one streaming workgroup per right-hand side for the tail
        const TailPlan &TP = h->tail[fwd ? 0 : 1];
        if (view == 0 && TP.nsteps > 0) {
            const int pp_ = h->prof.begin(fwd ? ILU_STAGE_FORWARD : ILU_STAGE_BACKWARD, s);
            if (TP.level0 > 0 && h->sched_solve == ILU_SCHED_LEVEL) {
                for (int32_t l = 0; l < TP.level0; ++l) {
                    A.row_begin = (*lptr)[l];
                    A.row_end = (*lptr)[l + 1];
                    if ((e = launch_solve(A, fwd, prec, vec, lanes, false, 0, s)) != hipSuccess)
                        return after_fwd(hip_fail(e, "solve launch"), pass);
                }
            } else if (TP.level0 > 0) {
                const TaskList *tl = ws ? h->cached_task_list(which, lanes, TP.level0) : h->task_list(which, lanes, TP.level0);
                if (!tl)
                    return after_fwd(ws ? fail(ILU_ERR_STATE, "solve: the sync-free task list is built by a first ilu_apply")
                                        : fail(ILU_ERR_NOMEM, "task list"),
                                     pass);
                if ((e = h->prepare_claims(fwd ? kPassForward : kPassBackward, tl, &A.claims, s)) != hipSuccess)
                    return after_fwd(hip_fail(e, "solve claims"), pass);
                A.nstreams = h->nstreams;
                A.poll_sleep = h->poll_sleep;
                if ((e = launch_solve(A, fwd, prec, vec, lanes, true, h->grid_syncfree(tl), s)) != hipSuccess)
                    return after_fwd(hip_fail(e, "solve launch"), pass);
            }
            StreamArgs sa{};
            sa.hdr = reinterpret_cast<const int4 *>(h->dtail[fwd ? 0 : 1].hdr);
            sa.rec = h->dtail[fwd ? 0 : 1].rec;
            sa.nsteps = TP.nsteps;
            A.poll_sleep = h->poll_sleep;
            e = launch_solve_stream(A, sa, fwd, prec, vec, s);
            h->prof.end(pp_, s);
            if (e != hipSuccess) return after_fwd(hip_fail(e, "tail launch"), pass);
            continue;
        }
        // the tiled schedule; a direction whose rows are too long for it runs
        // sync-free, and so do the transposed views of an unsymmetric pattern
        if ((view == 0 || h->pattern_sym) && h->sched_solve == ILU_SCHED_TILED && tile_rows_ok(h->tiles[fwd ? 0 : 1])) {
            const TileSet &T = h->tiles[fwd ? 0 : 1];
            const ilu_handle_s::DevTiles &D = h->dtiles[fwd ? 0 : 1];
            TileArgs ta{};
            ta.tile_ptr = D.ptr;
            ta.pslot = D.pslot;
            ta.rows_ptr = D.rows_ptr;
            ta.meta = reinterpret_cast<const int4 *>(D.meta);
            ta.imp_ptr = D.imp_ptr;
            ta.imp = D.imp;
            ta.sci = h->d_sci;
            ta.ntiles = T.ntiles;
            ta.max_rows = T.max_rows;
            ta.max_slots = T.max_slots;
            ta.max_pos = T.max_pos;
            ta.max_imps = T.max_imps;
            ta.kmax = T.kmax;
            ta.unit = T.unit;
            ta.blocks_per_cu = h->solve_bpc;
            if ((e = h->prepare_tile_claims(fwd ? kPassTileF : kPassTileB, &ta, s)) != hipSuccess)
                return after_fwd(hip_fail(e, "tile claims"), pass);
            A.poll_sleep = h->poll_sleep;
            const int pp_ = h->prof.begin(fwd ? ILU_STAGE_FORWARD : ILU_STAGE_BACKWARD, s);
            e = launch_solve_tiled(A, ta, fwd, prec, vec, s);
            h->prof.end(pp_, s);
            if (e == hipErrorInvalidValue)
                return after_fwd(fail(ILU_ERR_UNSUPPORTED, "tiled solve: the largest tile does not fit LDS (lower tile_rows)"),
                                 pass);
            if (e != hipSuccess) return after_fwd(hip_fail(e, "tiled solve launch"), pass);
        } else if (sf) {
            const TaskList *tl = ws ? h->cached_task_list(which, lanes) : h->task_list(which, lanes);
            if (!tl)
                return after_fwd(ws ? fail(ILU_ERR_STATE, "solve: the sync-free task list is built by a first ilu_apply")
                                    : fail(ILU_ERR_NOMEM, "task list"),
                                 pass);
            const int cpass = view == 0 ? (fwd ? kPassForward : kPassBackward) : (fwd ? kPassTForward : kPassTBackward);
            if ((e = h->prepare_claims(cpass, tl, &A.claims, s)) != hipSuccess)
                return after_fwd(hip_fail(e, "solve claims"), pass);
            A.nstreams = h->nstreams;
            A.poll_sleep = h->poll_sleep;
            const int pp_ = h->prof.begin(fwd ? ILU_STAGE_FORWARD : ILU_STAGE_BACKWARD, s);
            e = launch_solve(A, fwd, prec, vec, lanes, true, h->grid_syncfree(tl), s);
            h->prof.end(pp_, s);
            if (e != hipSuccess) return after_fwd(hip_fail(e, "solve launch"), pass);
        } else {
            const int pp_ = h->prof.begin(fwd ? ILU_STAGE_FORWARD : ILU_STAGE_BACKWARD, s);
            for (size_t l = 0; l + 1 < lptr->size(); ++l) {
                A.row_begin = (*lptr)[l];
                A.row_end = (*lptr)[l + 1];
                if ((e = launch_solve(A, fwd, prec, vec, lanes, false, 0, s)) != hipSuccess)
                    return after_fwd(hip_fail(e, "solve launch"), pass);
            }
            h->prof.end(pp_, s);
        }
    }
    h->prof.end(pcall, s);
    return ILU_OK;
}

}  // namespace jv

extern "C" ilu_status ilu_apply(ilu_handle h, const void *b, void *x, int32_t nrhs, int64_t ld, int32_t fac_prec,
                                int32_t vec_prec, int32_t flags, hipStream_t s) {
    if (!h) return fail(ILU_ERR_STATE, "ilu_apply: NULL handle");
    if (!h->factored) return fail(ILU_ERR_STATE, "ilu_apply: no factor");
    if (!b || !x || nrhs < 1 || ld < nrhs) return fail(ILU_ERR_ARG, "ilu_apply: bad vectors or sizes");
    if (vec_prec != ILU_PREC_F64 && vec_prec != ILU_PREC_F32) return fail(ILU_ERR_ARG, "ilu_apply: vec_prec");
    if (flags & ~ILU_PERMUTED_SPACE) return fail(ILU_ERR_ARG, "ilu_apply: unknown flags");
    const void *val;
    switch (fac_prec) {
        case ILU_PREC_F64: val = h->d_lu; break;
        case ILU_PREC_F32:
            if (!h->has32) return fail(ILU_ERR_STATE, "ilu_apply: factor has no FP32 copy");
            val = h->d_lu32;
            break;
        case ILU_PREC_BF16:
            if (!h->has16) return fail(ILU_ERR_STATE, "ilu_apply: factor has no BF16 copy");
            val = h->d_lu16;
            break;
        default: return fail(ILU_ERR_ARG, "ilu_apply: fac_prec");
    }
    return run_solves(h, 0, val, fac_prec, vec_prec == ILU_PREC_F64 ? 0 : 1, b, x, nullptr, nullptr, nrhs, ld, flags,
                      s);
}

extern "C" ilu_status ilu_get_status(ilu_handle h, hipStream_t s) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_get_status: NULL handle");
    if (h->host_only) return ILU_OK;
    return h->take_timeout(s, "ilu_get_status");
}

extern "C" ilu_status ilu_apply_ex(ilu_handle h, const double *lu_val, const double *b, double *x, double *y_out,
                                   int32_t nrhs, int64_t ld, int32_t flags, hipStream_t s) {
    if (!h) return fail(ILU_ERR_STATE, "ilu_apply_ex: NULL handle");
    if (h->host_only) return fail(ILU_ERR_STATE, "ilu_apply_ex: host-only analysis");
    if (!lu_val && !h->factored) return fail(ILU_ERR_STATE, "ilu_apply_ex: no factor");
    if (!b || !x || nrhs < 1 || ld < nrhs) return fail(ILU_ERR_ARG, "ilu_apply_ex: bad vectors or sizes");
    if (flags & ~ILU_PERMUTED_SPACE) return fail(ILU_ERR_ARG, "ilu_apply_ex: unknown flags");
    return run_solves(h, 0, lu_val ? lu_val : h->d_lu, ILU_PREC_F64, 0, b, x, y_out, nullptr, nrhs, ld, flags, s);
}

// -------------------------------------------------------------------------------------
// Graph capture of an apply
// -------------------------------------------------------------------------------------

struct ilu_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ilu_handle h = nullptr;
    ~ilu_graph_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

extern "C" ilu_status ilu_apply_graph_create(ilu_handle h, const void *b, void *x, int32_t nrhs, int64_t ld,
                                             int32_t fac_prec, int32_t vec_prec, int32_t flags, ilu_graph *out) {
    if (!h || !out) return fail(ILU_ERR_ARG, "ilu_apply_graph_create: NULL argument");
    *out = nullptr;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "ilu_apply_graph_create: stream");
    // an eager apply first: allocates workspaces and builds the task lists outside the capture
    ilu_status st = ilu_apply(h, b, x, nrhs, ld, fac_prec, vec_prec, flags, cs);
    if (st == ILU_OK && (e = hipStreamSynchronize(cs)) != hipSuccess) st = hip_fail(e, "ilu_apply_graph_create");
    const bool prof = h->prof.enabled;
    h->prof.enabled = false;
    std::unique_ptr<ilu_graph_s> g(new (std::nothrow) ilu_graph_s());
    if (st == ILU_OK && !g) st = fail(ILU_ERR_NOMEM, "ilu_apply_graph_create");
    if (st == ILU_OK) {
        if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            st = hip_fail(e, "ilu_apply_graph_create: begin capture");
        } else {
            ilu_status st2 = ilu_apply(h, b, x, nrhs, ld, fac_prec, vec_prec, flags, cs);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(cs, &graph);
            if (st2 != ILU_OK) st = st2;
            else if (e != hipSuccess) st = hip_fail(e, "ilu_apply_graph_create: end capture");
            g->graph = graph;
            if (st == ILU_OK && (e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0)) != hipSuccess)
                st = hip_fail(e, "ilu_apply_graph_create: instantiate");
        }
    }
    h->prof.enabled = prof;
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
    if (st != ILU_OK) return st;
    g->h = h;
    *out = g.release();
    return ILU_OK;
}

extern "C" ilu_status ilu_graph_launch(ilu_graph g, hipStream_t s) {
    if (!g || !g->exec) return fail(ILU_ERR_ARG, "ilu_graph_launch: NULL graph");
    hipError_t e = hipGraphLaunch(g->exec, s);
    if (e != hipSuccess) return hip_fail(e, "ilu_graph_launch");
    return ILU_OK;
}

extern "C" ilu_status ilu_graph_destroy(ilu_graph g) {
    delete g;
    return ILU_OK;
}

// spmv
extern "C" ilu_status ilu_set_values(ilu_handle h, const double *a_val, hipStream_t s) {
    if (!h) return fail(ILU_ERR_STATE, "ilu_set_values: NULL handle");
    if (h->host_only) return fail(ILU_ERR_STATE, "ilu_set_values: host-only analysis");
    if (!a_val && h->H.nnz_in) return fail(ILU_ERR_ARG, "ilu_set_values: NULL values");
    hipError_t e = launch_gather(h->H.b_rp[h->H.n], h->d_b_src, a_val, h->d_bval, s);
    if (e != hipSuccess) return hip_fail(e, "ilu_set_values");
    h->bvals = true;
    return ILU_OK;
}

extern "C" ilu_status ilu_spmv(ilu_handle h, double alpha, const double *x, double beta, double *y, int32_t nrhs,
                               int64_t ld, int32_t flags, hipStream_t s) {
    if (!h) return fail(ILU_ERR_STATE, "ilu_spmv: NULL handle");
    if (!h->bvals) return fail(ILU_ERR_STATE, "ilu_spmv: no values loaded");
    if (!x || !y || nrhs < 1 || ld < nrhs) return fail(ILU_ERR_ARG, "ilu_spmv: bad vectors or sizes");
    if (x == y) return fail(ILU_ERR_ARG, "ilu_spmv: x and y must not alias");
    SpmvArgs A{};
    A.n = h->H.n;
    A.rp = h->d_b_rp;
    A.ci = h->d_b_ci;
    A.val = h->d_bval;
    A.perm = (flags & ILU_PERMUTED_SPACE) ? nullptr : h->d_perm;
    A.x = x;
    A.y = y;
    A.alpha = alpha;
    A.beta = beta;
    A.ld = ld;
    A.nrhs = nrhs;
    A.heavy_min = h->spmv_heavy_min;
    A.heavy = h->d_spmv_heavy;
    A.nheavy = h->n_spmv_heavy;
    if (h->spmv_nz) {
        A.nz_waves = h->nz_waves;
        A.nz_wrow = h->d_nz_wrow;
        A.nz_bits = h->d_nz_bits;
        A.nz_span = h->d_nz_span;
        A.nz_nspan = h->nz_nspan;
        A.nz_part = h->d_nz_part;
    }
    const int pp_ = h->prof.begin(ILU_STAGE_SPMV, s);
    hipError_t e = launch_spmv(A, h->lanes_spmv, s);
    h->prof.end(pp_, s);
    if (e != hipSuccess) return hip_fail(e, "ilu_spmv");
    return ILU_OK;
}

// -------------------------------------------------------------------------------------
// Adjoint
// -------------------------------------------------------------------------------------

extern "C" ilu_status ilu_apply_adjoint(ilu_handle h, const double *lu_val, const double *gx, const double *x,
                                        const double *y, double *gb, double *glu, int32_t nrhs, int64_t ld,
                                        hipStream_t s) {
    if (!h) return fail(ILU_ERR_STATE, "ilu_apply_adjoint: NULL handle");
    if (h->host_only) return fail(ILU_ERR_STATE, "ilu_apply_adjoint: host-only analysis");
    if (!lu_val && !h->factored) return fail(ILU_ERR_STATE, "ilu_apply_adjoint: no factor");
    if (!gx || nrhs < 1 || ld < nrhs) return fail(ILU_ERR_ARG, "ilu_apply_adjoint: bad vectors or sizes");
    if (glu && (!x || !y)) return fail(ILU_ERR_ARG, "ilu_apply_adjoint: glu needs the saved x and y");
    const HostAnalysis &H = h->H;
    hipError_t e;
    const size_t vec_bytes = (size_t)H.n * (size_t)ld * 8;
    if (h->adj_bytes < vec_bytes) {
        void *p;
        if (h->d_adj_w) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(h->d_adj_w);
            allocs_erase(h, h->d_adj_w);
            (void)hipFree(h->d_adj_bp);
            allocs_erase(h, h->d_adj_bp);
            (void)hipFree(h->d_adj_gb);
            allocs_erase(h, h->d_adj_gb);
        }
        if ((e = h->alloc_bytes(&p, vec_bytes)) != hipSuccess) return hip_fail(e, "adjoint workspace");
        h->d_adj_w = (double *)p;
        if ((e = h->alloc_bytes(&p, vec_bytes)) != hipSuccess) return hip_fail(e, "adjoint workspace");
        h->d_adj_bp = (double *)p;
        if ((e = h->alloc_bytes(&p, vec_bytes)) != hipSuccess) return hip_fail(e, "adjoint workspace");
        h->d_adj_gb = (double *)p;
        h->adj_bytes = vec_bytes;
    }
    const double *val = lu_val ? lu_val : h->d_lu;
    double *gb_out = gb ? gb : h->d_adj_gb;
    ilu_status st = run_solves(h, 1, val, ILU_PREC_F64, 0, gx, gb_out, h->d_adj_w, h->d_adj_bp, nrhs, ld, 0, s);
    if (st != ILU_OK) return st;
    if (glu) {
        e = launch_outer(H.n, h->d_lu_rp, h->d_lu_ci, h->d_perm, h->d_adj_w, h->d_adj_bp, x, y, glu, nrhs, ld, s);
        if (e != hipSuccess) return hip_fail(e, "ilu_apply_adjoint: outer products");
    }
    return ILU_OK;
}

// -------------------------------------------------------------------------------------
// Scheduling
// -------------------------------------------------------------------------------------

static bool valid_lanes(int l) { return l == 0 || l == 4 || l == 8 || l == 16 || l == 32 || l == 64; }

extern "C" ilu_status ilu_set_schedule(ilu_handle h, int32_t factor_sched, int32_t solve_sched, int32_t lanes_factor,
                                       int32_t lanes_solve) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_set_schedule: NULL handle");
    if (factor_sched < 0 || factor_sched > 3 || solve_sched < 0 || solve_sched > 3 || !valid_lanes(lanes_factor) ||
        !valid_lanes(lanes_solve))
        return fail(ILU_ERR_ARG, "ilu_set_schedule: bad value");
    if (factor_sched) h->sched_factor = factor_sched;
    if (solve_sched) h->sched_solve = solve_sched;
    if (lanes_factor) {
        if (lanes_factor < h->H.max_row_lu)
            return fail(ILU_ERR_ARG, "ilu_set_schedule: factor lanes must cover the longest factor row");
        h->lanes_factor = lanes_factor;
    }
    if (lanes_solve) h->lanes_solve = lanes_solve;
    return ILU_OK;
}

extern "C" ilu_status ilu_get_schedule(ilu_handle h, int32_t *factor_sched, int32_t *solve_sched,
                                       int32_t *lanes_factor, int32_t *lanes_solve) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_get_schedule: NULL handle");
    if (factor_sched) *factor_sched = h->sched_factor;
    if (solve_sched) *solve_sched = h->sched_solve;
    if (lanes_factor) *lanes_factor = h->lanes_factor;
    if (lanes_solve) *lanes_solve = h->lanes_solve;
    return ILU_OK;
}

extern "C" ilu_status ilu_set_tuning(ilu_handle h, const char *key, int64_t value) {
    if (!h || !key) return fail(ILU_ERR_ARG, "ilu_set_tuning: NULL argument");
    const std::string k(key);
    if (k == "poll_sleep") {
        if (value < 0 || value > 64) return fail(ILU_ERR_ARG, "ilu_set_tuning: poll_sleep must be in [0, 64]");
        h->poll_sleep = (int32_t)value;
        return ILU_OK;
    }
    if (k == "tile_rows") {
        if (value < 16 || value > 65536) return fail(ILU_ERR_ARG, "ilu_set_tuning: tile_rows must be in [16, 65536]");
        return h->make_tiles((int32_t)value, false);
    }
    if (k == "spmv_lanes") {
        if (value != 1 && value != 4 && value != 8 && value != 16 && value != 32 && value != 64)
            return fail(ILU_ERR_ARG, "ilu_set_tuning: spmv_lanes must be 1, 4, 8, 16, 32 or 64");
        h->lanes_spmv = (int32_t)value;
        return ILU_OK;
    }
    if (k == "factor_tile_rows") {
        if (value != 0 && (value < 16 || value > 65536))
            return fail(ILU_ERR_ARG, "ilu_set_tuning: factor_tile_rows must be 0 or in [16, 65536]");
        if (!h->host_only) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "factor tiles: synchronize");
        }
        h->factor_rows = (int32_t)value;
        return h->make_factor_tiles();
    }
    if (k == "tile_lattice") {
        if (value != 0 && value != 1) return fail(ILU_ERR_ARG, "ilu_set_tuning: tile_lattice must be 0 or 1");
        h->tile_lattice = value != 0;
        return h->make_tiles(h->tile_rows, false);
    }
    if (k == "factor_lower_stage") {
        if (value != 0 && value != 1) return fail(ILU_ERR_ARG, "ilu_set_tuning: factor_lower_stage must be 0 or 1");
        h->factor_lower = value != 0;
        return ILU_OK;
    }
    if (k == "spmv_nz") {
        if (value != 0 && value != 1) return fail(ILU_ERR_ARG, "ilu_set_tuning: spmv_nz must be 0 or 1");
        h->spmv_nz = value != 0;
        return ILU_OK;
    }
    if (k == "solve_blocks_per_cu") {
        if (value < 0 || value > 8) return fail(ILU_ERR_ARG, "ilu_set_tuning: solve_blocks_per_cu must be in [0, 8]");
        h->solve_bpc = (int32_t)value;
        return ILU_OK;
    }
    if (k == "factor_staged") {
        if (value != 0 && value != 1) return fail(ILU_ERR_ARG, "ilu_set_tuning: factor_staged must be 0 or 1");
        h->factor_staged = value != 0;
        return ILU_OK;
    }
    if (k == "tail_min_rows") {
        if (value < 0 || value > 65536) return fail(ILU_ERR_ARG, "ilu_set_tuning: tail_min_rows must be in [0, 65536]");
        return h->make_tail((int32_t)value);
    }
    if (k == "force_abort") {
        // failure-path tests: 1 raises the abort flag now (as an apply that timed
        // out and was not reported would leave it); 2 raises it inside the next
        // apply, after its guard, so its kernels leave through their bounded waits
        if (value != 1 && value != 2) return fail(ILU_ERR_ARG, "ilu_set_tuning: force_abort must be 1 or 2");
        if (h->host_only) return fail(ILU_ERR_STATE, "ilu_set_tuning: host-only analysis");
        if (value == 2) {
            h->force_abort = true;
            return ILU_OK;
        }
        hipError_t e = launch_raise_abort(h->d_info, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        return e == hipSuccess ? ILU_OK : hip_fail(e, "ilu_set_tuning: force_abort");
    }
    return fail(ILU_ERR_ARG, "ilu_set_tuning: unknown key " + k);
}

extern "C" ilu_status ilu_get_tuning(ilu_handle h, const char *key, int64_t *value) {
    if (!h || !key || !value) return fail(ILU_ERR_ARG, "ilu_get_tuning: NULL argument");
    const std::string k(key);
    if (k == "poll_sleep") { *value = h->poll_sleep; return ILU_OK; }
    if (k == "nstreams") { *value = h->nstreams; return ILU_OK; }
    if (k == "factor_tcap") { *value = h->factor_tcap; return ILU_OK; }
    if (k == "tile_rows") { *value = h->tile_rows; return ILU_OK; }
    if (k == "tile_lattice") { *value = h->tiles_on_lattice ? 1 : 0; return ILU_OK; }
    if (k == "spmv_lanes") { *value = h->lanes_spmv; return ILU_OK; }
    if (k == "factor_tile_rows") {
        *value = !h->ftiles_ok ? 0 : h->ftset_own ? h->ftset.cap : h->tile_rows;
        return ILU_OK;
    }
    if (k == "solve_blocks_per_cu") { *value = h->solve_bpc; return ILU_OK; }
    if (k == "spmv_nz") { *value = (h->spmv_nz && h->nz_waves > 0) ? 1 : 0; return ILU_OK; }
    if (k == "factor_lower_stage") { *value = h->factor_lower ? 1 : 0; return ILU_OK; }
    if (k == "factor_lower_planned") { *value = h->ftail_ok ? 1 : 0; return ILU_OK; }
    if (k == "factor_tiled") { *value = h->ftiles_ok ? 1 : 0; return ILU_OK; }
    if (k == "factor_staged") { *value = h->factor_staged ? 1 : 0; return ILU_OK; }
    if (k == "tail_min_rows") { *value = h->tail_min_rows; return ILU_OK; }
    return fail(ILU_ERR_ARG, "ilu_get_tuning: unknown key " + k);
}

// -------------------------------------------------------------------------------------
// Kernel timing
// -------------------------------------------------------------------------------------

extern "C" ilu_status ilu_profile_enable(ilu_handle h, int32_t enable, int32_t capacity) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_profile_enable: NULL handle");
    if (!enable) {
        h->prof.enabled = false;
        return ILU_OK;
    }
    if (capacity < 1 || capacity > (1 << 20)) return fail(ILU_ERR_ARG, "ilu_profile_enable: capacity");
    if (h->prof.pool.size() < (size_t)2 * capacity) {
        h->prof.release();
        h->prof.pool.resize((size_t)2 * capacity);
        for (auto &ev : h->prof.pool) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) {
                ev = nullptr;
                h->prof.release();
                return hip_fail(e, "ilu_profile_enable: events");
            }
        }
    }
    h->prof.stage.clear();
    h->prof.closed.clear();
    h->prof.used = 0;
    h->prof.enabled = true;
    return ILU_OK;
}

extern "C" ilu_status ilu_profile_read(ilu_handle h, double *ms, int64_t *launches) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_profile_read: NULL handle");
    double acc[ILU_STAGE_COUNT] = {0};
    int64_t cnt[ILU_STAGE_COUNT] = {0};
    for (size_t i = 0; i < h->prof.used; ++i) {
        if (!h->prof.closed[i]) continue;
        hipError_t e = hipEventSynchronize(h->prof.pool[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "ilu_profile_read");
        float t = 0.f;
        e = hipEventElapsedTime(&t, h->prof.pool[2 * i], h->prof.pool[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "ilu_profile_read");
        acc[h->prof.stage[i]] += t;
        cnt[h->prof.stage[i]] += 1;
    }
    h->prof.stage.clear();
    h->prof.closed.clear();
    h->prof.used = 0;
    for (int i = 0; i < ILU_STAGE_COUNT; ++i) {
        if (ms) ms[i] = acc[i];
        if (launches) launches[i] = cnt[i];
    }
    return ILU_OK;
}

// -------------------------------------------------------------------------------------
// Lifetime
// -------------------------------------------------------------------------------------

extern "C" ilu_status ilu_destroy(ilu_handle h) {
    delete h;
    return ILU_OK;
}

extern "C" const char *ilu_version(void) { return "javelin-mi355x 0.1 (gfx950)"; }

extern "C" const char *ilu_status_str(ilu_status s) {
    switch (s) {
        case ILU_OK: return "ILU_OK";
        case ILU_ERR_ARG: return "ILU_ERR_ARG";
        case ILU_ERR_CSR: return "ILU_ERR_CSR";
        case ILU_ERR_NOMEM: return "ILU_ERR_NOMEM";
        case ILU_ERR_HIP: return "ILU_ERR_HIP";
        case ILU_ERR_ZERO_PIVOT: return "ILU_ERR_ZERO_PIVOT";
        case ILU_ERR_NONFINITE: return "ILU_ERR_NONFINITE";
        case ILU_ERR_NOCONV: return "ILU_ERR_NOCONV";
        case ILU_ERR_BREAKDOWN: return "ILU_ERR_BREAKDOWN";
        case ILU_ERR_STATE: return "ILU_ERR_STATE";
        case ILU_ERR_UNSUPPORTED: return "ILU_ERR_UNSUPPORTED";
        case ILU_ERR_TIMEOUT: return "ILU_ERR_TIMEOUT";
        default: return "ILU_ERR_UNKNOWN";
    }
}

extern "C" ilu_status ilu_last_error(char *buf, int32_t len) {
    if (!buf || len <= 0) return ILU_ERR_ARG;
    std::strncpy(buf, g_last_error.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
    return ILU_OK;
}
