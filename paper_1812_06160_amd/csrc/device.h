// Device-side declarations shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "analysis.h"

namespace jv {

// Bit patterns published into factor values and solve intermediates.  Both are
// signalling NaNs with a payload: arithmetic never produces them (a NaN result
// is quiet), and stored values that happen to be NaN are canonicalised before
// they are published.
constexpr uint64_t kPending64 = 0x7FF40000DEADBEEFull;   // value not yet computed
constexpr uint64_t kDropped64 = 0x7FF400000D50D50Dull;   // entry dropped by the tau test
constexpr uint32_t kPending32 = 0x7FA0BEEFu;
constexpr uint64_t kQNaN64 = 0x7FF8000000000000ull;
constexpr uint32_t kQNaN32 = 0x7FC00000u;

// info word layout (int32 slots)
enum : int {
    kInfoBadKey = 0,      // atomicMin of 2*row + (0 zero pivot | 1 non-finite); INT32_MAX if none
    kInfoAbort = 1,       // a bounded wait expired: every persistent kernel stops
    kInfoDropLo = 2,      // dropped-entry count (uint64 in slots 2-3)
    kInfoTimeouts = 4,    // applies whose start found the abort flag raised (cleared by a status query)
    kInfoGuardDone = 5,   // blocks of the solve guard that have finished re-arming
    kInfoSlots = 8
};

// Bound on a single dependency wait: 10 s of the 100 MHz realtime counter.  A
// wait that long means a value that will never be published (the device abort
// flag then stops every wait and the call reports ILU_ERR_TIMEOUT).
constexpr uint64_t kWaitTicks = 1000000000ull;

// Sync-free kernels take their work from task streams, one per XCD.  Each level's
// tasks are cut into contiguous slices, slice x of every level going to stream x,
// so level-to-level dependencies mostly stay inside one XCD's L2.  A block that
// starts on XCD x claims the next block slot of stream x with one atomic add on
// that XCD's counter (start order), and each of its waves runs one task of the
// slot.  A block waits only on tasks of earlier-claimed slots, which belong to
// blocks that already run or have finished, so progress never depends on how
// many blocks are resident.
constexpr int kStreams = 8;          // maximum XCD count handled
constexpr int kCounterStride = 32;   // int32 slots between counters (128 bytes)

struct Claims {
    const int32_t *task_ptr;      // positions of task t: [task_ptr[t], task_ptr[t + 1])
    const int32_t *stream_tasks;  // task ids in stream order (stream, level, position)
    const int32_t *stream_ptr;    // nstreams + 1 offsets into stream_tasks
    int32_t *counters;            // this pass's claim counters (kStreams * kCounterStride)
    int32_t *zero_counters;       // counters of another pass to clear at launch (may be null)
    const int8_t *xcc_stream;     // hardware XCC id (0..15) -> stream
};

struct FactorArgs {
    int32_t n;
    const int32_t *rp, *ci, *diag, *src;
    const int8_t *flev;
    int32_t k;
    int32_t use_flev;     // k < k_max: entries with fill level > k are absent
    int32_t use_tau;
    int32_t milu;         // modified ILU: what a row loses is added to its diagonal
    const double *a;      // input values (input entry order)
    double *lu;           // factor values (factor order)
    const double *row_tau;
    int32_t *info;
    // level-launch range or persistent claims
    int32_t row_begin, row_end;
    Claims claims;
    int32_t nstreams;
    int32_t tcap;         // LDS entries per group for the dependency rows (0: no staging)
    int32_t max_lower;    // longest strictly lower part of a row
    int32_t poll_sleep;   // s_sleep(1) steps between polls of a pending value
    int32_t lcap;         // long rows (more than 64 entries): LDS entries per wave (0: not used)
    float *lu32;          // tiled factor: FP32 copy written with each published row (may be null)
    uint16_t *lu16;       // tiled factor: BF16 copy written with each published row (may be null)
    double *bval;         // tiled factor, when the permuted copy of A has the factor's pattern:
                          // A's values written into it as each row starts (may be null)
};

struct SolveArgs {
    int32_t n;
    const int32_t *rp, *ci, *diag;
    const void *val;          // TV[nnz]
    const int32_t *rows;      // row list (nullptr: identity)
    const int32_t *perm;      // nullptr: permuted space
    const void *b;            // [n][ld] double or float (forward input)
    void *x;                  // [n][ld] double or float (backward output)
    void *y;                  // TA[n][cap] forward intermediate (published)
    void *z;                  // TA[n][cap] backward intermediate (published)
    void *y_out;              // optional copy of y (TA) [n][ld], level ordering
    void *z_out;              // optional copy of z (TA) [n][ld], level ordering
    int64_t ld;
    int32_t cap;              // columns of the y/z buffers
    int32_t nrhs;
    int32_t vec_f32;          // b and x are float (1) or double (0)
    int32_t unit_diag;        // forward: 1 (L), 0 (U^T); backward: 1 (L^T) or 0 (U)
    int32_t *info;
    int32_t row_begin, row_end;   // level-launch range over `rows` positions
    Claims claims;
    int32_t nstreams;
    int32_t poll_sleep;
    const int32_t *vmap;      // optional value gather map (transposed views): val[vmap[p]]
};

// Tiled solve: one workgroup per tile, tiles claimed in start order (tile order is
// topological, so a block only waits on tiles of blocks that started earlier).
// A block stages its tile (rows, dependency slots and values, pivots, right-hand
// sides) into LDS, one poller wave copies the tile's imports (dependencies in
// other tiles) from the published y/z buffers into their LDS slots as they
// appear, and the compute waves solve the tile's rows reading LDS only.
struct TileArgs {
    const int32_t *tile_ptr;  // [ntiles + 1] positions (rows + padding)
    const int16_t *pslot;     // LDS slot of each position, -1 for padding
    const int32_t *rows_ptr;  // [ntiles + 1] offsets into meta
    const int4 *meta;         // per row of each tile in slot order: row, first and end entry of the
                              // direction's part of the row, diagonal entry
    const int32_t *imp_ptr;   // [ntiles + 1] offsets into imp
    const int32_t *imp;       // imported rows (slot = tile rows + index)
    const int32_t *sci;       // per factor entry: LDS slot of the dependency
    int32_t ntiles;
    int32_t max_rows, max_slots, max_pos, max_imps, kmax;
    int32_t unit;             // positions per chunk (64: one lane per row, 16: four)
    // LDS carve-up (bytes), set by the launcher
    int32_t off_rhs, off_piv, off_eval, off_eslot, off_rowid, off_pslot, off_imp, off_orow, lds_bytes;
    int32_t *counter;         // claim counter of this pass
    int32_t *zero_counter;    // counter of the complementary pass, cleared at launch (may be null)
    int32_t blocks_per_cu;    // at most this many tiles resident per CU (0: as many as fit)
};

// Tiled solve blocks: kTileComputeWaves compute waves and 1 poller wave (imports);
// all of them stage the tile.  A tile
// whose rows have at most kTileShortRow dependencies is solved with one lane per
// row (chunks of 64 positions); longer rows get 4 lanes each (chunks of 16, at
// most 4 * kTileLongJ dependencies).  The chunk size is fixed by the tiling.
constexpr int kTileComputeWaves = 8;
constexpr int kTileShortRow = 1;
constexpr int kTileLongJ = 8;
constexpr int kTileBlock = 64 * (kTileComputeWaves + 1);
// Compute waves of a tiled solve block by accumulate type.  Seven for FP64 gives
// eight-wave blocks, two waves on every SIMD; FP32 (fewer registers per lane)
// measured faster with eight.
template <typename TA>
constexpr int solve_waves() { return sizeof(TA) == 8 ? 7 : 8; }
template <typename TA>
constexpr int solve_block() { return 64 * (solve_waves<TA>() + 1); }
constexpr int kTileLdsMax = 163840;   // dynamic LDS bytes a tiled solve may use (the whole LDS of a CU)
constexpr int kFactorTileLdsMax = 163840;   // the whole LDS of a compute unit (opt-in above 64 KB)
constexpr int kFactorMaxLanes = 32;         // longest factor row of the tiled factor
// LDS a tiling needs with `nr` right-hand sides per pass of `acc_bytes` each
size_t tile_lds_bytes(int max_rows, int max_slots, int max_pos, int max_imps, int kmax, int nr, int acc_bytes);

// Lower stage (tail) of a solve direction, streamed by one workgroup per
// right-hand side: wave 0 computes the steps in order, the other waves stage them
// kTailQ steps ahead (see TailPlan in analysis.h for the record format).
struct StreamArgs {
    const int4 *hdr;          // [nsteps + 1] per step: record offset, packed counts, entries, 0
    const int32_t *rec;       // step records
    int32_t nsteps;
    // LDS carve-up (bytes), set by the launcher
    int32_t off_vals, off_a, off_c, off_lane, off_rhs, off_piv, off_hdr, off_sync, lds_bytes;
};
constexpr int kStreamStagers = 15;
// The factor's lower stage (one block): the plan of build_factor_tail.
struct FactorStreamArgs {
    const int4 *hdr;          // [nsteps + 1] per step: first row record, rows, most L entries, lane map offset
    const int4 *rows;         // 2 per row record
    const int32_t *lsrc;      // per L entry: ring base of U(c) (>= 0) or -(diag(c) + 1)
    const uint8_t *match;     // per L entry and row entry: position in U(c), 255 none
    const uint8_t *lmap;      // 64 per step: lane -> row of the step (255 idle)
    int32_t nsteps, q;        // steps; steps staged ahead (<= kFTailQ)
};
// factor's lower stage: rows of the tail in steps; every row before the tail must
// be final in A.lu, the tail rows' entries armed with the pending pattern
hipError_t launch_factor_stream(const FactorArgs &A, const FactorStreamArgs &T, hipStream_t s);
// The stream launch: A.nrhs blocks (block b solves right-hand side b of the
// direction's tail); the direction's rows before the tail must be finished.
hipError_t launch_solve_stream(const SolveArgs &A, const StreamArgs &T, bool forward, int prec, int vec,
                               hipStream_t s);

// Tiled factor (plain ILU: every pattern entry kept, no dropping) on the forward
// tiles; see FactorTiles in analysis.h for the data.
// One tile's tables live in a blob in the layout they take in LDS (FactorHdr
// gives the offsets): per tile row meta (row, first entry, end entry, diagonal
// entry; the row complemented when its L entries are independent) and off
// (value-area offset, L-entry offset); per L entry the LDS location and ready
// flag of its U row and, per lane, the position of the lane's column in that U
// row; per import (diagonal entry, U length, value-area offset); per position
// the row slot (-1: padding).
struct FactorTileArgs {
    const int32_t *hdr;       // kFactorHdr words per tile
    const int4 *blob;
    const int32_t *vsrc;      // input entry of each row value slot, -1 for fill
    const uint32_t *cmask;    // per L entry: U(c) positions whose update goes to the diagonal (modified ILU)
    int32_t ntiles;
    int32_t lds_bytes;        // LDS of the largest tile image
    int32_t *counter;         // claim counter (zero at launch)
};

struct SpmvArgs {
    int32_t n;
    const int32_t *rp, *ci;
    const double *val;
    const int32_t *perm;      // nullptr: permuted space
    const double *x;
    double *y;
    double alpha, beta;
    int64_t ld;
    int32_t nrhs;
    // rows with more than heavy_min entries are left to a second pass with one wave
    // per row over the list heavy[0 .. nheavy) (load balance for long rows)
    int32_t heavy_min;
    const int32_t *heavy;
    int32_t nheavy;
    // nnz-balanced pass (one right-hand side, rows all nonempty): wave w takes
    // entries [w * kNzWave, (w + 1) * kNzWave), 16 consecutive entries per lane;
    // nz_bits marks the entries that start a row (16 bits per lane, one chunk of 64
    // spare at the end), nz_wrow[w] is the row of the wave's first entry, and the
    // rows whose entries reach over several waves (nz_span: row, first wave, last
    // wave) are added up from the waves' pieces in nz_part by a second kernel
    int32_t nz_waves;
    const int32_t *nz_wrow;
    const uint16_t *nz_bits;
    const int32_t *nz_span;
    int32_t nz_nspan;
    double *nz_part;          // [2 * nz_waves]: closing piece, open piece of each wave
};
constexpr int kNzLane = 16;
constexpr int kNzWave = 64 * kNzLane;

// launchers (kernels.hip); all return hipError_t of the launch
hipError_t launch_fill_u64(uint64_t *p, uint64_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_zero_counters(int32_t *counters, hipStream_t s);
// Start of every apply: when the device abort flag is raised (a bounded wait of an
// earlier call expired), re-arms the published intermediates (y/z of both
// precision classes: n64 FP64 and n32 FP32 elements each), clears the flag and
// counts the event in info[kInfoTimeouts]; otherwise every block returns at once.
hipError_t launch_solve_guard(int32_t *info, uint64_t *y64, uint64_t *z64, int64_t n64, uint32_t *y32, uint32_t *z32,
                              int64_t n32, hipStream_t s);
// The guard of a factor call, which also resets the factor's status slots (bad row,
// drop count; the abort flag is clear after the guard) and, when `counters` is not
// null, zeroes that pass's claim counters -- one launch instead of three.
hipError_t launch_factor_prologue(int32_t *info, uint64_t *y64, uint64_t *z64, int64_t n64, uint32_t *y32,
                                  uint32_t *z32, int64_t n32, int32_t *counters, hipStream_t s);
// Writes the pending pattern into `count` ranges of the factor buffer: range i is
// entries [ranges[i].x, ranges[i].x + ranges[i].y) (the U parts other tiles import).
hipError_t launch_arm_ranges(uint64_t *lu, const int2 *ranges, int32_t count, hipStream_t s);
// Raises the device abort flag from the stream (failure-path tests: every wait of
// the kernels that follow gives up within its next 64 polls).
hipError_t launch_raise_abort(int32_t *info, hipStream_t s);
hipError_t launch_row_tau(int32_t n, const int32_t *in_rp, const double *a, const int32_t *perm, double tau,
                          double *row_tau, hipStream_t s);
hipError_t launch_gather(int64_t m, const int32_t *src, const double *a, double *out, hipStream_t s);
hipError_t launch_factor(const FactorArgs &A, int lanes, bool syncfree, int grid, hipStream_t s);
// factor with one wave per row and the row's values in LDS (A.lcap entries per wave),
// for patterns with rows longer than 64 entries; hipErrorInvalidValue when the rows
// do not fit LDS
hipError_t launch_factor_long(const FactorArgs &A, bool syncfree, int grid, hipStream_t s);
constexpr int kFactorLongMax = 4096;   // longest factor row of the long-row factor
hipError_t launch_factor_fixup(int64_t nnz, double *lu, const int8_t *flev, int32_t k, int32_t use_flev,
                               int8_t *stat, int32_t *info, hipStream_t s);
hipError_t launch_cast_f32(int64_t m, const double *x, float *y, hipStream_t s);
hipError_t launch_cast_bf16(int64_t m, const double *x, uint16_t *y, hipStream_t s);
// prec: 0 f64 values / f64 arithmetic, 1 f32 values, 2 bf16 values (f32 arithmetic);
// vec: 0 double vectors, 1 float vectors
hipError_t launch_solve(const SolveArgs &A, bool forward, int prec, int vec, int lanes, bool syncfree,
                        int grid, hipStream_t s);
hipError_t launch_spmv(const SpmvArgs &A, int lanes, hipStream_t s);
// tiled factor with `lanes` (8, 16 or 32) lanes per row; hipErrorInvalidValue when it
// does not fit LDS
hipError_t launch_factor_tiled(const FactorArgs &A, const FactorTileArgs &T, int lanes, hipStream_t s);
// tiled solve; returns hipErrorInvalidValue when no right-hand-side blocking fits LDS
hipError_t launch_solve_tiled(const SolveArgs &A, const TileArgs &T, bool forward, int prec, int vec,
                              hipStream_t s);
// adjoint outer products on the factor pattern: for entry p = (i, j) of row i,
// glu[p] = -sum_s W[i][s] x[perm[j]][s] (j >= i) or -sum_s Bp[i][s] y[j][s] (j < i)
hipError_t launch_outer(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *perm, const double *W,
                        const double *Bp, const double *x, const double *y, double *glu, int32_t nrhs, int64_t ld,
                        hipStream_t s);
// capacity queries for persistent launches (blocks), and the dynamic LDS the factor
// needs per block for a given staging capacity (0 if it does not fit)
size_t factor_lds_bytes(int lanes, int tcap);
// XCC ids seen by the first `blocks` blocks of a launch (host array of `blocks`)
hipError_t probe_xcc_ids(int blocks, int32_t *host_ids);

}  // namespace jv
