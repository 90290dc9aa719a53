// The analysis handle behind ilu_handle: host schedule, device arrays, workspaces.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "analysis.h"
#include "device.h"
#include "javelin.h"

namespace jv {

enum { kTasksForward = 0, kTasksBackward = 1, kTasksTForward = 2, kTasksTBackward = 3 };

// Event pairs around stage launches (ilu_profile_*).  Pairs may nest: a whole
// call is bracketed around the brackets of its kernels.
struct Profiler {
    bool enabled = false;
    std::vector<hipEvent_t> pool;      // 2 * capacity events
    std::vector<int> stage;            // stage of each pair handed out
    std::vector<char> closed;          // its end event was recorded
    size_t used = 0;                   // pairs handed out
    int begin(int st, hipStream_t s);  // pair index, -1 when not recording
    void end(int pair, hipStream_t s);
    void release();
};

struct TaskList {
    int32_t *ptr = nullptr;            // device, ntasks + 1 positions
    int32_t *stream_tasks = nullptr;   // device, task ids in stream order
    int32_t *stream_ptr = nullptr;     // device, nstreams + 1
    int32_t ntasks = 0;
    int32_t max_slots = 0;             // block slots of the longest stream
};

// claim-counter sets of the persistent passes
enum {
    kPassFactor = 0, kPassForward = 1, kPassBackward = 2, kPassTForward = 3, kPassTBackward = 4,
    kPassTileF = 5, kPassTileB = 6, kPassFactorTile = 7, kPasses = 8
};

ilu_status fail(ilu_status s, const std::string &msg);
ilu_status hip_fail(hipError_t e, const char *what);

}  // namespace jv

struct ilu_handle_s {
    jv::HostAnalysis H;
    int32_t batch_count = 1;
    std::vector<int64_t> row_off, nnz_off;

    // structure on the device
    int32_t *d_in_rp = nullptr, *d_perm = nullptr;
    int32_t *d_lu_rp = nullptr, *d_lu_ci = nullptr, *d_diag = nullptr, *d_lu_src = nullptr;
    int8_t *d_flev = nullptr;
    int32_t *d_b_rp = nullptr, *d_b_ci = nullptr, *d_b_src = nullptr;
    int32_t *d_ulevel_rows = nullptr;
    int32_t *d_t_rp = nullptr, *d_t_ci = nullptr, *d_t_map = nullptr, *d_t_diag = nullptr;
    int32_t *d_tlevel_rows = nullptr, *d_tulevel_rows = nullptr;

    // values
    double *d_lu = nullptr, *d_bval = nullptr, *d_row_tau = nullptr;
    float *d_lu32 = nullptr;
    uint16_t *d_lu16 = nullptr;
    int8_t *d_stat = nullptr;
    int32_t *d_info = nullptr;
    double *d_dotwork = nullptr;     // dot work area: kDotParts partials, kDotScalars scalar slots

    // published solve intermediates [n][cap], kept "all pending" between calls
    int cap64 = 0, cap32 = 0;
    void *y64 = nullptr, *z64 = nullptr, *y32 = nullptr, *z32 = nullptr;

    // adjoint workspaces [n][ld]
    size_t adj_bytes = 0;
    double *d_adj_w = nullptr, *d_adj_bp = nullptr, *d_adj_gb = nullptr;

    // Krylov workspace
    size_t kry_bytes = 0;
    double *d_kry = nullptr;
    // pinned host block the drivers read their scalars and the info words into, and
    // the event that marks a posted readback complete
    double *h_kry_pin = nullptr;
    hipEvent_t kry_ev = nullptr;

    std::map<int64_t, jv::TaskList> tasks;

    // tiles of the tiled solves (direction 0: L, 1: U) and the solve column encoding
    jv::TileSet tiles[2];
    std::vector<int32_t> sci;
    int32_t tile_rows = 0;             // rows per tile of the current tiles
    bool tile_lattice = true;          // box tiles on structured grids (else greedy growth)
    int32_t factor_rows = 0;           // rows per tile of the tiled factor (0: the solves' size)
    bool tiles_on_lattice = false;     // the current tiles are lattice boxes
    bool pattern_sym = false;          // factor pattern symmetric: the transposed views (adjoint)
                                       // have the same rows and columns and use the same tiles
    struct DevTiles {
        int32_t *ptr = nullptr, *rows_ptr = nullptr, *meta = nullptr, *imp_ptr = nullptr, *imp = nullptr;
        int16_t *pslot = nullptr;
    } dtiles[2];
    int32_t *d_sci = nullptr;
    // tiled factor (plain ILU) on the forward tiles
    jv::FactorTiles ftiles;
    bool ftiles_ok = false;            // built and fits LDS
    // the factor's own forward tiling, when the solves' tiles make too large an LDS
    // image for it (ftset_own); otherwise the factor uses tiles[0] / dtiles[0]
    jv::TileSet ftset;
    bool ftset_own = false;
    // the forward tiling of the size the default tiles were doubled from, kept
    // for the factor (whose default tile size is often that one); empty otherwise
    jv::TileSet spare_fwd;
    struct DevFactorTiles {
        int32_t *hdr = nullptr, *blob = nullptr, *vsrc = nullptr;
        uint32_t *cmask = nullptr;
    } dft;
    int32_t *d_arm = nullptr;          // tiled factor: (diagonal entry, U length) of every imported row
    int32_t n_arm = 0;
    bool arm_built = false;            // d_arm / n_arm describe the current factor tiles
    bool b_same = false;               // the permuted copy of A has the factor's pattern
    // lower stage of each solve direction (0: L, 1: U) and its device copy
    jv::TailPlan tail[2];
    int32_t tail_min_rows = 0;
    struct DevTail {
        int32_t *hdr = nullptr, *rec = nullptr;
    } dtail[2];
    // the factor's lower stage (rows of the forward tail; plain ILU(k) at k_max)
    jv::FactorTailPlan ftail;
    bool ftail_ok = false;
    bool factor_lower = false;         // factor through the lower stage when planned (tunable)
    struct DevFTail {
        int32_t *hdr = nullptr, *rows = nullptr, *lsrc = nullptr;
        uint8_t *match = nullptr, *lmap = nullptr;
    } dftail;
    jv::Profiler prof;
    int32_t *d_counters = nullptr;     // kPasses sets of claim counters
    bool counters_dirty[jv::kPasses] = {false, false, false, false, false, false, false, false};
    int32_t factor_tcap = 0;           // LDS staging entries per factor row (0: unstaged)
    bool factor_staged = true;         // stage dependency rows in LDS when they fit
    int32_t nstreams = 1;              // task streams (one per XCD)
    int32_t poll_sleep = 1;            // s_sleep(1) steps between polls (tunable)
    int32_t solve_bpc = 2;             // tiled solves: resident tiles per CU cap (0: none; tunable)
    int8_t *d_xcc_stream = nullptr;    // XCC id -> stream
    int32_t *d_spmv_heavy = nullptr;   // rows of the permuted copy of A longer than spmv_heavy_min
    int32_t n_spmv_heavy = 0, spmv_heavy_min = INT32_MAX;
    // nnz-balanced spmv (when long rows exist and no row is empty): per wave its
    // first entry's row, the row-start bits, the rows over several waves, pieces
    int32_t *d_nz_wrow = nullptr, *d_nz_span = nullptr;
    uint16_t *d_nz_bits = nullptr;
    double *d_nz_part = nullptr;
    int32_t nz_waves = 0, nz_nspan = 0;
    bool spmv_nz = false;              // use it (when built; tunable)
    std::vector<void *> allocs;

    // state
    bool host_only = false;
    bool factored = false, factor_ok = false, tracked = false, bvals = false, has32 = false, has16 = false;
    bool force_abort = false;          // raise the abort flag inside the next apply (tests)
    int32_t k_used = 0;                // k, tau and flags of the last factor (the tuner re-runs it)
    double tau_used = 0.0;
    int32_t flags_used = 0;
    int32_t sched_factor = ILU_SCHED_SYNCFREE, sched_solve = ILU_SCHED_SYNCFREE;
    int32_t lanes_factor = 8, lanes_solve = 4, lanes_spmv = 8;

    ~ilu_handle_s();
    hipError_t alloc_bytes(void **p, size_t bytes);
    // task list of the first `levels` levels of a direction (-1: all)
    const jv::TaskList *task_list(int which, int lanes, int32_t levels = -1);
    hipError_t ensure_workspace(int nrhs, int prec_class, hipStream_t s);
    hipError_t rearm(hipStream_t s);
    hipError_t reset_info(hipStream_t s);
    // launches the solve guard over the handle's intermediates (see launch_solve_guard)
    hipError_t guard(hipStream_t s);
    // synchronous check of the abort flag and the timeout count (ILU_ERR_TIMEOUT
    // after re-arming and clearing them)
    ilu_status take_timeout(hipStream_t s, const char *who);
    // the task list if it has been built already (no allocation), else nullptr
    static int64_t task_key(int which, int lanes, int32_t levels) {
        return ((int64_t)(levels + 1) << 16) | (int64_t)(which << 8) | lanes;
    }
    const jv::TaskList *cached_task_list(int which, int lanes, int32_t levels = -1) const {
        auto it = tasks.find(task_key(which, lanes, levels));
        return it == tasks.end() ? nullptr : &it->second;
    }
    // fills the claims of one sync-free pass (launching a counter reset when needed)
    hipError_t prepare_claims(int pass, const jv::TaskList *tl, jv::Claims *c, hipStream_t s);
    // blocks of a sync-free launch: every stream's slots plus one spare per stream
    int grid_syncfree(const jv::TaskList *tl) const { return nstreams * (tl->max_slots + 1); }
    // (re)builds the tiles on the host and, unless host-only, uploads them; with
    // shrink, halves the tile size until the tiles fit the LDS budget
    ilu_status make_tiles(int32_t rows, bool shrink);
    ilu_status make_factor_tiles();
    // (re)builds the lower stage of both solve directions (min_rows 0: none)
    ilu_status make_tail(int32_t min_rows);
    // (re)builds the factor's lower stage from the forward tail (called by make_tail)
    ilu_status make_factor_tail();
    // claim counter of a tiled pass (launching a counter reset when needed)
    hipError_t prepare_tile_claims(int pass, jv::TileArgs *t, hipStream_t s);
};

inline void allocs_erase(ilu_handle_s *h, void *p) {
    auto it = std::find(h->allocs.begin(), h->allocs.end(), p);
    if (it != h->allocs.end()) h->allocs.erase(it);
}

namespace jv {
// Published intermediates supplied by the caller instead of the handle's: y and z
// of [n][cap] elements of the accumulate type; fill: arm them at the start.
struct SolveWork {
    void *y, *z;
    int32_t cap;
    bool fill;
};
ilu_status run_solves(ilu_handle_s *h, int view, const void *val, int prec, int vec, const void *b, void *x,
                      void *y_out, void *z_out, int nrhs, int64_t ld, int flags, hipStream_t s,
                      const SolveWork *ws = nullptr, bool guard = true);
}
