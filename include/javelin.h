/*
 * javelin.h -- C ABI of the MI355X (gfx950) incomplete-LU hot path.
 *
 * The method is the one of Booth & Bolet, "Javelin: A Scalable Implementation
 * for Sparse Incomplete LU Factorization" (arXiv:1812.06160): the fill pattern of
 * A and a level ordering are found once (Sec. III, "Level Scheduling, Upper
 * Stage"), A is copied into one CSR that holds L and U in level order, the
 * numeric factor runs up-looking on that fixed pattern (Sec. III, Fig. 1), and
 * the same structure serves the sparse triangular solves and the sparse
 * matrix-vector product that apply M^{-1} = U^{-1} L^{-1} inside CG/GMRES
 * (Sec. I, Sec. VI).
 *
 * Conventions (all calls):
 *  - Every function returns an ilu_status; ILU_OK is 0.  No C++ exception crosses
 *    this boundary.  ilu_status_str() names a status, ilu_last_error() gives the
 *    detail of the last failure on the calling thread.
 *  - Indices are 0-based int32; nnz must be below 2^31 (ILU_ERR_UNSUPPORTED).
 *  - "device" pointers are HIP device memory owned by the caller and borrowed for
 *    the duration of the call (asynchronous calls: until the stream reaches them).
 *    "host" pointers are ordinary host memory, read or written before the call
 *    returns.
 *  - A handle owns every buffer it allocates (hipMalloc at analysis time, freed by
 *    ilu_destroy).  Handles are not thread-safe; distinct handles are independent.
 *  - Calls are ordered on the given hipStream_t (0 = the null stream).
 *  - Dense vectors are row-major [n][ld] with nrhs <= ld columns ("RHS interleaved").
 */
#ifndef JAVELIN_H
#define JAVELIN_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ilu_status;
enum {
    ILU_OK = 0,
    ILU_ERR_ARG = 1,          /* NULL pointer, bad size or option value */
    ILU_ERR_CSR = 2,          /* row_ptr not monotone, columns unsorted / duplicate / out of range */
    ILU_ERR_NOMEM = 3,        /* host or device allocation failed */
    ILU_ERR_HIP = 4,          /* a HIP runtime call failed (detail in ilu_last_error) */
    ILU_ERR_ZERO_PIVOT = 5,   /* u_rr == 0 in the first failing row (no pivoting, Sec. III) */
    ILU_ERR_NONFINITE = 6,    /* a non-finite value in the first failing row */
    ILU_ERR_NOCONV = 7,       /* Krylov iteration limit reached (x still holds the last iterate) */
    ILU_ERR_BREAKDOWN = 8,    /* Krylov breakdown (zero curvature) */
    ILU_ERR_STATE = 9,        /* call out of order (e.g. apply before factor) */
    ILU_ERR_UNSUPPORTED = 10, /* size or row length beyond what the kernels support */
    ILU_ERR_TIMEOUT = 11      /* a dependency wait in a persistent kernel exceeded its bound (or a
                                 test raised the abort flag through "force_abort") */
};

/* Dependency pattern used to build level sets (Sec. III; Sec. VII recommends the
 * symmetric one by default).  ILU_PATTERN_UPPER_A (ilu_levels_device only): row
 * i depends on every j > i of its own row, levels counted from the last row --
 * the backward solve's schedule (Sec. VI) when the CSR is the permuted factor
 * pattern. */
enum { ILU_PATTERN_LOWER_SYM = 0, ILU_PATTERN_LOWER_A = 1, ILU_PATTERN_UPPER_A = 2 };

/* Storage precision of the factor values used by an apply. */
enum { ILU_PREC_F64 = 0, ILU_PREC_F32 = 1, ILU_PREC_BF16 = 2 };

/* Bits of `flags`. */
enum {
    ILU_PERMUTED_SPACE = 1    /* b, x (apply) and x, y (spmv) are in the level ordering */
};

/* Scheduling of the factor and the triangular solves. */
enum {
    ILU_SCHED_AUTO = 0,       /* the handle's current choice: after analysis the factor and the
                                 solves are tiled where their tiles fit LDS, else sync-free */
    ILU_SCHED_LEVEL = 1,      /* one kernel launch per level: the launch boundary is the barrier */
    ILU_SCHED_SYNCFREE = 2,   /* one launch for all levels; rows wait on per-row published values */
    ILU_SCHED_TILED = 3       /* one launch; rows grouped into tiles, one workgroup per tile,
                                 dependencies inside a tile resolved in LDS (Sec. III's
                                 point-to-point waits, kept on-chip where the tile allows) */
};

typedef struct ilu_handle_s *ilu_handle;

/* Host CSR of A (values are passed to ilu_factor instead). */
typedef struct {
    int32_t n;                /* rows = columns, > 0 */
    int64_t nnz;              /* row_ptr[n] */
    const int32_t *row_ptr;   /* host, n + 1 entries, row_ptr[0] = 0, non-decreasing */
    const int32_t *col_idx;   /* host, nnz entries, sorted and unique within a row */
} ilu_csr;

typedef struct {
    int32_t k_max;            /* largest level of fill that ilu_factor may use (>= 0) */
    int32_t pattern;          /* ILU_PATTERN_LOWER_SYM (default) or ILU_PATTERN_LOWER_A */
    int32_t host_only;        /* 1: analysis on the host only, nothing uploaded (inspection and
                                 planning without a device); numeric calls then fail with
                                 ILU_ERR_STATE */
    int32_t tile_rows;        /* rows per tile of the tiled solves (0 = default: 512, halved until a
                                 tile fits the LDS budget, or doubled to 1024 on a 3D grid read as a
                                 lattice when such a tile fits a CU's LDS and the grid makes 256 of
                                 them; else 16..65536, used as given) */
    int32_t ordering;         /* ILU_ORDER_NATURAL (default: A as given) or ILU_ORDER_RCM */
    int32_t tail_min_rows;    /* lower stage of the triangular solves (Sec. III-B, "Lower Stage";
                                 Fig. 7): 0 = none; M > 0: in each direction the longest suffix of
                                 the level order whose levels all hold fewer than M rows (at least
                                 64 levels) is solved by one streaming workgroup per right-hand
                                 side after the rows before it */
    int32_t reserved[2];      /* must be 0 */
} ilu_analyze_opts;

/* Preorderings applied before the analysis (Sec. VII compares orderings; the
 * method itself only imposes the level ordering).  ILU_ORDER_RCM: reverse
 * Cuthill-McKee on the graph of A + A^T -- components in order of their smallest
 * vertex, each started from a pseudo-peripheral vertex (George-Liu search seeded
 * with the vertex of least degree, ties to the smaller index), neighbours queued
 * by (degree, index), the whole sweep reversed.  The levels are then those of
 * Q A Q^T; perm (ilu_copy_schedule) and every call keep using the input ordering,
 * so callers see no difference except the schedule and the factor.  Not
 * available for batched handles (ILU_ERR_UNSUPPORTED). */
enum { ILU_ORDER_NATURAL = 0, ILU_ORDER_RCM = 1 };

typedef struct {
    int32_t n;
    int32_t n_levels;         /* forward (factor / L solve) levels */
    int32_t n_ulevels;        /* backward (U solve) levels */
    int32_t max_row_lu;       /* longest row of the factor pattern */
    int64_t nnz_a;            /* input nnz */
    int64_t nnz_lu;           /* factor pattern nnz (fill included) */
    int64_t nnz_b;            /* nnz of the permuted copy of A (input + inserted diagonals) */
    int32_t level_min, level_max;   /* rows per forward level */
    double level_median;
    int32_t batch_count;      /* matrices in a batched handle (1 otherwise) */
    int32_t n_tiles;          /* tiles of the forward (L) tiled solve */
    int32_t n_utiles;         /* tiles of the backward (U) tiled solve */
    int32_t tile_rows;        /* rows per tile requested */
    int32_t max_tile;         /* most rows in one tile of either direction */
    int32_t tail_rows;        /* rows in the lower stage of the forward solve (0: none) */
    int32_t tail_urows;       /* rows in the lower stage of the backward solve (0: none) */
    int32_t reserved[1];
} ilu_info;

typedef struct {
    int32_t bad_row;          /* first failing row in the level ordering, -1 if none */
    int32_t bad_row_original; /* the same row in the input ordering, -1 if none */
    int32_t bad_matrix;       /* batched handles: index of the matrix holding bad_row */
    int32_t reserved;
    int64_t n_dropped;        /* entries dropped by the tau test */
} ilu_factor_info;

typedef struct {
    int32_t iters;            /* inner iterations (CG steps, GMRES Arnoldi steps) */
    int32_t status;           /* ILU_OK, ILU_ERR_NOCONV or ILU_ERR_BREAKDOWN */
    double relres;            /* last recursive residual norm / ||b|| */
    double true_relres;       /* ||b - A x|| / ||b|| recomputed at exit */
} ilu_solve_info;

/* ---------------------------------------------------------------------------- */
/* Analysis (setup; the paper leaves it out of the timed factor, Sec. V).        */
/* ---------------------------------------------------------------------------- */

/* Validates A, inserts missing diagonals, finds the ILU(k_max) pattern S by level
 * of fill in the input ordering (Sec. III: the pattern with its fill is found
 * first, then permuted), the level sets of lower(S) or lower(S + S^T) (Sec. II,
 * Sec. III), the stable level-order permutation, the permuted factor structure
 * P S P^T with diagonal positions, the permuted copy of A for spmv, and the
 * backward-solve schedule; uploads all of it.  opts may be NULL (k_max = 0,
 * LOWER_SYM).  Synchronous.  Errors: ILU_ERR_ARG, ILU_ERR_CSR, ILU_ERR_NOMEM,
 * ILU_ERR_HIP, ILU_ERR_UNSUPPORTED. */
ilu_status ilu_analyze(const ilu_csr *A, const ilu_analyze_opts *opts, ilu_handle *out);

/* Block-diagonal batch of `count` matrices analysed as one: the level sets of all
 * matrices merge level by level, so a single factor / apply / spmv call (one
 * persistent launch per stage) serves the whole batch.  Values, right-hand sides
 * and solutions are the per-matrix arrays concatenated in order. */
ilu_status ilu_analyze_batched(int32_t count, const ilu_csr *As, const ilu_analyze_opts *opts,
                               ilu_handle *out);

/* Level sets computed on the device (Sec. II, level scheduling; Sec. III, the
 * dependency graph): row i depends on every j < i with (i, j) in the pattern,
 * and with ILU_PATTERN_LOWER_SYM also on every j < i with (j, i) in it; with
 * ILU_PATTERN_UPPER_A on every j > i with (i, j) in it.  Level 0 holds the rows
 * with no dependency; a row's level is one more than the deepest level it
 * depends on.  Outputs (device, caller-owned): perm[r] = the row at
 * position r of the order by (level, row index), iperm its inverse (both n),
 * level_ptr[l] = first position of level l, level_ptr[n_levels] = n (capacity
 * n + 1); *n_levels (host).  These equal the schedule ilu_analyze computes on
 * the host for the same pattern (its ILU(k) fill pattern S passed here as the
 * CSR; for ILU_PATTERN_UPPER_A, the permuted factor pattern, whose result is
 * the backward schedule ulevel_ptr / ulevel_rows).  row_ptr (n + 1) and col_idx (nnz) are device arrays, checked first:
 * ILU_ERR_CSR for row pointers that do not run monotonically from 0 to nnz, or
 * columns unsorted, repeated or out of range.  The diagonal is optional.
 * Allocates one scratch block (about 20 bytes per row; with the symmetric
 * pattern 12 more per row and 4 per stored entry; plus the sort's
 * temporaries) and frees it; returns after the work on `stream` has finished.
 * ILU_ERR_TIMEOUT if a dependency wait exceeded its bound.  On either error
 * nothing is written to the outputs. */
ilu_status ilu_levels_device(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                             int32_t pattern, int32_t *level_ptr, int32_t *perm, int32_t *iperm,
                             int32_t *n_levels, hipStream_t stream);

/* Permuted structure on the device (Sec. III: A copied into the level-ordered
 * CSR of L and U): row r of the output is row perm[r] of the input pattern, its
 * columns renamed c -> iperm[c] and sorted ascending; out_src[q] is the input
 * entry that output entry q came from, diag_pos[r] the position of column r in
 * output row r (-1 if absent).  With the ILU(k) pattern S and the level order
 * of ilu_levels_device this is the factor pattern P S P^T, its diagonal
 * positions and its entry map, as ilu_analyze builds them on the host.  All
 * arrays are device, caller-owned: row_ptr (n + 1), col_idx (nnz), perm and
 * iperm (n), out_row_ptr (n + 1), out_col_idx and out_src (nnz), diag_pos (n).
 * ILU_ERR_CSR for an invalid pattern (as ilu_levels_device), ILU_ERR_ARG when
 * perm is not a permutation with inverse iperm; the outputs are then
 * unspecified.  Allocates one scratch block (about 8 bytes per entry plus the
 * sort's temporaries) and frees it; returns after the work on `stream` has
 * finished. */
ilu_status ilu_permute_device(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                              const int32_t *perm, const int32_t *iperm, int32_t *out_row_ptr,
                              int32_t *out_col_idx, int32_t *out_src, int32_t *diag_pos, hipStream_t stream);

/* Transposed structure on the device (the transposed views the adjoint's
 * solves run on, Sec. VI): t_row_ptr / t_col_idx is the CSR of the pattern's
 * transpose with columns ascending, t_map[q] the input entry that transposed
 * entry q came from, t_diag[j] the position of column j in transposed row j (-1
 * if absent).  Device arrays, caller-owned: row_ptr and t_row_ptr (n + 1),
 * col_idx, t_col_idx and t_map (nnz), t_diag (n).  ILU_ERR_CSR for an invalid
 * pattern (outputs then unspecified).  Allocates one scratch block (about 8
 * bytes per row and per entry plus the sort's temporaries) and frees it;
 * returns after the work on `stream` has finished. */
ilu_status ilu_transpose_device(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                int32_t *t_row_ptr, int32_t *t_col_idx, int32_t *t_map, int32_t *t_diag,
                                hipStream_t stream);

/* Row and entry offsets of matrix i in a batched handle (host arrays of count+1). */
ilu_status ilu_batch_offsets(ilu_handle h, int64_t *row_off, int64_t *nnz_off);

ilu_status ilu_get_info(ilu_handle h, ilu_info *out);

/* Copies the schedule and structure to host arrays; any pointer may be NULL.
 * Sizes: level_ptr n_levels+1, perm n, lu_row_ptr n+1, lu_col_idx nnz_lu,
 * diag_pos n, ulevel_ptr n_ulevels+1, ulevel_rows n, fill_lev nnz_lu,
 * lu_src nnz_lu (input entry of each factor entry, -1 for fill / inserted
 * diagonal), b_row_ptr n+1, b_col_idx nnz_b. */
ilu_status ilu_copy_schedule(ilu_handle h, int32_t *level_ptr, int32_t *perm, int32_t *lu_row_ptr,
                             int32_t *lu_col_idx, int32_t *diag_pos, int32_t *ulevel_ptr,
                             int32_t *ulevel_rows, int8_t *fill_lev, int32_t *lu_src,
                             int32_t *b_row_ptr, int32_t *b_col_idx);

/* Copies the tiles of one solve direction (dir 0: L, 1: U) to host arrays; any
 * pointer may be NULL.  Tiles are numbered in a topological order of that
 * direction's dependency graph; tile t holds positions [tile_ptr[t],
 * tile_ptr[t+1]) of tile_row (rows in the level ordering sorted by local level
 * inside the tile, -1 for padding that aligns each local level to 16 positions).
 * sci (nnz_lu entries, shared by both directions) encodes each off-diagonal
 * factor entry (r, c) by the LDS slot of c in r's tile of the direction that
 * reads it: the slots of a tile are its rows in position order, then its imports
 * (the distinct columns read from other tiles, in order of first use); diagonal
 * entries hold -1.
 * Sizes: tile_ptr n_tiles+1 (n_utiles+1 for dir 1), tile_row tile_ptr[last]. */
ilu_status ilu_copy_tiles(ilu_handle h, int32_t dir, int32_t *tile_ptr, int32_t *tile_row, int32_t *sci);

/* Copies the lower stage ("tail") of one solve direction (dir 0: L, 1: U; see
 * ilu_analyze_opts.tail_min_rows) to host arrays; any pointer may be NULL.
 * sizes[4] = {first tail level (-1: none), first tail position, steps, record
 * words}.  hdr (4 * (steps + 1)): per step its record offset, nrows | nlanes << 8
 * | log2(largest lane group) << 16 | flags << 24 (1: adds the previous step's
 * partial sum, 2: finishes its rows), entries, 0.  rec: per step, 4 words per row
 * (row in the level ordering, ring slot, input-ordering row, diagonal entry), one
 * word per lane (row in the step | log2 of its lane group << 8 | group leader <<
 * 16), then per entry (entry (lane, j) at j * nlanes + lane) its factor entry (-1:
 * none) and the source of its dependency value (a ring slot below 2048, 2048 + row
 * for the published buffer, -1: none).  For inspection and tests. */
ilu_status ilu_copy_tail(ilu_handle h, int32_t dir, int32_t *sizes, int32_t *hdr, int32_t *rec);

/* Copies the factor's lower stage (Sec. III-B, Even-Rows: the forward tail's rows
 * factored in level-ordered steps by one workgroup; used by ilu_factor for plain
 * ILU(k) at k = k_max when a tail is set) to host arrays; any pointer may be NULL.
 * sizes[10] = {first tail level (-1: no plan), first tail position, steps, umax
 * (longest U part of a tail row), ring rows, staging depth q, row records, L-entry
 * sources, match bytes, lane-map bytes}.  hdr (4 * (steps + 1)): per step its first
 * row record, rows, most L entries of a row, lane-map offset.  rows: 8 words per
 * record {row, first factor entry, len | K << 8 | log2 group << 16 | first lane <<
 * 24, ring base, first L-entry source, first match byte, 0, 0}.  lsrc: per L entry
 * the ring base of U(c) (>= 0) or -(diag(c) + 1) (read from the factor buffer).
 * match: per L entry e and entry t of the row (len bytes per e) the position of
 * entry t's column in U(c_e) (0 for t == e, 255 none).  lmap: 64 bytes per step,
 * each lane's row in the step (255: idle).  No plan when a tail row is longer than
 * 64 entries or has more than 16 L entries.  For inspection and tests. */
ilu_status ilu_copy_factor_tail(ilu_handle h, int32_t *sizes, int32_t *hdr, int32_t *rows, int32_t *lsrc,
                                uint8_t *match, uint8_t *lmap);

/* ---------------------------------------------------------------------------- */
/* Numeric factor (Sec. III, Fig. 1).                                            */
/* ---------------------------------------------------------------------------- */

/* flags of ilu_factor */
enum {
    ILU_CAST_F32 = 1,             /* also store an FP32 copy (round to nearest even) */
    ILU_CAST_BF16 = 2,            /* also store a BF16 copy (FP64 -> FP32 -> BF16, each RNE) */
    ILU_FACTOR_MODIFIED = 0x100   /* modified ILU (named as an option in Sec. I and Sec. III) */
};

/* ILU(k, tau) with 0 <= k <= k_max on the analysed pattern.  a_val: device, the
 * values of A in the input entry order (length nnz_a).  Entries with fill level
 * above k are absent; with tau > 0, a multiplier l_rc with |l_rc| < tau_r after
 * its division, and a U entry with |u_rj| < tau_r at the end of its row, are
 * dropped (set to 0 and marked), where tau_r = tau * ||A(row,:)||_2; the
 * diagonal is never dropped.  The FP64 factor is kept; flags ILU_CAST_F32 /
 * ILU_CAST_BF16 also store rounded copies for ILU_PREC_F32/BF16 applies.
 * ILU_FACTOR_MODIFIED: whatever row r loses is added to u_rr when it is lost --
 * an update l_rc * u_cj whose target (r, j) is not a kept entry is subtracted
 * from u_rr, a dropped multiplier adds back its value before the division, a
 * dropped U entry adds back its value (ascending column) -- so the row sums of
 * L*U equal those of A.  The tiled factor covers the modified form too; with
 * k < k_max it runs sync-free (or level launches).
 * Also loads the values of the permuted copy of A used by ilu_spmv.
 * Synchronises `stream` to read the status word.  info may be NULL.
 * Errors: ILU_ERR_STATE, ILU_ERR_ARG (k > k_max, tau < 0 or NaN, unknown flag
 * bits), ILU_ERR_ZERO_PIVOT, ILU_ERR_NONFINITE (first failing row in level
 * order), ILU_ERR_TIMEOUT, ILU_ERR_HIP. */
ilu_status ilu_factor(ilu_handle h, const double *a_val, int32_t k, double tau, int32_t flags,
                      ilu_factor_info *info, hipStream_t stream);

/* Device pointer to the factor values in factor order (L strictly lower with unit
 * diagonal implied, U upper with diagonal), of the given precision; owned by h. */
ilu_status ilu_factor_values(ilu_handle h, int32_t prec, const void **dev_ptr);

/* Copies FP64 factor values and the per-entry state (0 kept, 1 dropped by tau,
 * 2 absent: fill level above k) to host arrays of nnz_lu (either may be NULL). */
ilu_status ilu_copy_factor(ilu_handle h, double *lu_val, int8_t *state);

/* Copies the stored factor of precision prec (ILU_PREC_F32: float, ILU_PREC_BF16:
 * uint16 bit patterns, ILU_PREC_F64: double) to a host array of nnz_lu. */
ilu_status ilu_copy_factor_prec(ilu_handle h, int32_t prec, void *host);

/* ---------------------------------------------------------------------------- */
/* Apply, spmv (Sec. VI; Sec. I).                                                */
/* ---------------------------------------------------------------------------- */

/* x = M^{-1} b = P^T U^{-1} L^{-1} P b, or U^{-1} L^{-1} b with ILU_PERMUTED_SPACE.
 * b, x: device, [n][ld] (ld >= nrhs >= 1), vec_prec ILU_PREC_F64 (double) or
 * ILU_PREC_F32 (float).  fac_prec selects the stored factor: F64 computes in
 * FP64; F32/BF16 compute in FP32 (b rounded to FP32, x rounded to vec_prec).
 * x may alias b.  Asynchronous.  Errors: ILU_ERR_STATE (no factor / cast),
 * ILU_ERR_ARG, ILU_ERR_UNSUPPORTED (a user tile size whose tiles do not fit LDS).
 * A dependency wait that expires on the device (ILU_ERR_TIMEOUT) cannot be
 * returned by this asynchronous call: its outputs hold NaNs, the next call on the
 * handle re-arms the intermediates, and ilu_get_status (or the Krylov driver
 * that made the call) reports ILU_ERR_TIMEOUT. */
ilu_status ilu_apply(ilu_handle h, const void *b, void *x, int32_t nrhs, int64_t ld,
                     int32_t fac_prec, int32_t vec_prec, int32_t flags, hipStream_t stream);

/* Synchronises `stream` and reports whether an apply on h (ilu_apply,
 * ilu_apply_ex, ilu_apply_adjoint, graph replays) has timed out since the last
 * query: ILU_ERR_TIMEOUT (after re-arming the handle's intermediates and clearing
 * the record), else ILU_OK. */
ilu_status ilu_get_status(ilu_handle h, hipStream_t stream);

/* ilu_apply for callers that cannot allocate device memory during the call (code
 * under graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results (bit for bit), with the published intermediates y and z
 * ([n][nrhs] each, of the accumulate type: 8 bytes per element for F64 factors, 4
 * for F32/BF16) in a static device workspace of 64 MiB that the library holds on
 * every device it runs on until the process ends, instead of the buffers
 * ilu_apply allocates on first use.  Calls no hipMalloc/hipFree.  The workspace is
 * shared by every call on a device: calls that overlap on one device (any
 * handle, any stream) race; it is re-armed at the start of each call.  The
 * sync-free schedule needs the task list a first ilu_apply of the handle built
 * (ILU_ERR_STATE otherwise); the tiled and level schedules need nothing.
 * Errors: as ilu_apply, and ILU_ERR_ARG when 2 * n * nrhs * element size exceeds
 * 64 MiB (n * nrhs above 4,194,304 with F64 factors, 8,388,608 with F32/BF16). */
ilu_status ilu_apply_noalloc(ilu_handle h, const void *b, void *x, int32_t nrhs, int64_t ld,
                             int32_t fac_prec, int32_t vec_prec, int32_t flags, hipStream_t stream);

/* FP64 apply with explicit factor values and the forward intermediate:
 * lu_val (device, nnz_lu, may be NULL = the handle's factor), y_out (device,
 * [n][ld] in the level ordering, may be NULL) receives y = L^{-1} P b. */
ilu_status ilu_apply_ex(ilu_handle h, const double *lu_val, const double *b, double *x,
                        double *y_out, int32_t nrhs, int64_t ld, int32_t flags, hipStream_t stream);

/* Adjoint of ilu_apply_ex for a loss l with gx = dl/dx (original ordering):
 *   w  = U^{-T} P gx,  b' = L^{-T} w,  gb = P^T b'            (transposed solves)
 *   glu[p] = -sum_s w_{r,s} x_{perm[c],s}  for U entries (r, c), c >= r
 *   glu[p] = -sum_s b'_{r,s} y_{c,s}       for L entries (r, c), c < r
 * x (original ordering) and y (level ordering) are the outputs of the forward
 * call.  gb and glu (nnz_lu, factor order, summed over RHS) may be NULL.
 * All device, FP64, [n][ld].  Asynchronous. */
ilu_status ilu_apply_adjoint(ilu_handle h, const double *lu_val, const double *gx, const double *x,
                             const double *y, double *gb, double *glu, int32_t nrhs, int64_t ld,
                             hipStream_t stream);

/* A graph holding one captured ilu_apply with fixed arguments (its sync-free
 * launches and counter resets), replayed with ilu_graph_launch on any stream.
 * Each replay leaves the handle ready for the next one, so replays may be
 * interleaved with ordinary calls on the same handle (not concurrently).  The
 * graph borrows b and x (device) and the handle; destroy it before either.
 * The factor values it reads are the handle's current ones at replay time. */
typedef struct ilu_graph_s *ilu_graph;
ilu_status ilu_apply_graph_create(ilu_handle h, const void *b, void *x, int32_t nrhs, int64_t ld,
                                  int32_t fac_prec, int32_t vec_prec, int32_t flags, ilu_graph *out);
ilu_status ilu_graph_launch(ilu_graph g, hipStream_t stream);
ilu_status ilu_graph_destroy(ilu_graph g);

/* y = alpha * A x + beta * y with the values loaded by ilu_factor (or
 * ilu_set_values); FP64, device [n][ld].  With ILU_PERMUTED_SPACE, x and y are
 * in the level ordering and the product is with P A P^T. */
ilu_status ilu_spmv(ilu_handle h, double alpha, const double *x, double beta, double *y,
                    int32_t nrhs, int64_t ld, int32_t flags, hipStream_t stream);

/* Loads A's values (device, input order) for ilu_spmv without factoring. */
ilu_status ilu_set_values(ilu_handle h, const double *a_val, hipStream_t stream);

/* ---------------------------------------------------------------------------- */
/* Krylov drivers (the consumers of Sec. I-II).                                  */
/* ---------------------------------------------------------------------------- */

/* Preconditioned CG from x0 = 0 on one right-hand side, FP64 vectors, apply in
 * fac_prec; stops when the recursive residual norm / ||b|| <= rtol, then checks
 * the true residual (restarting the recurrence from it if it misses).
 * b, x device [n] (original ordering unless ILU_PERMUTED_SPACE).  Synchronous.
 * info may be NULL.  Returns ILU_OK, ILU_ERR_NOCONV or ILU_ERR_BREAKDOWN, or
 * ILU_ERR_TIMEOUT when an apply inside it timed out (checked at every scalar
 * readback). */
ilu_status ilu_solve_pcg(ilu_handle h, const double *b, double *x, double rtol, int32_t maxit,
                         int32_t fac_prec, int32_t flags, ilu_solve_info *info, hipStream_t stream);

/* Right-preconditioned flexible GMRES(restart) with modified Gram-Schmidt and
 * Givens rotations, x0 = 0; a cycle ends at |g_{j+1}| / ||b|| <= rtol, happy
 * breakdown or `restart` steps; the true residual decides whether to restart.
 * maxit bounds the total Arnoldi steps.  Synchronous.  ILU_ERR_TIMEOUT as for
 * ilu_solve_pcg. */
ilu_status ilu_solve_gmres(ilu_handle h, const double *b, double *x, double rtol, int32_t restart,
                           int32_t maxit, int32_t fac_prec, int32_t flags, ilu_solve_info *info,
                           hipStream_t stream);

/* ---------------------------------------------------------------------------- */
/* Scheduling and tuning.                                                         */
/* ---------------------------------------------------------------------------- */

/* Chooses the launch scheme of the factor and of the solves (ILU_SCHED_*) and the
 * lanes per row (0 = automatic from the longest row; else 4, 8, 16, 32 or 64;
 * factor lanes must cover the longest factor row).  The tiled factor runs ILU(k,
 * tau) and modified ILU(k, tau) with k = k_max and rows of at most 32 entries;
 * otherwise the call runs the sync-free factor.  A solve direction whose rows have
 * more than 32 dependencies runs sync-free under the tiled schedule.  Factor rows
 * longer than 64 entries (up to 4096) run with one wave per row and the row in
 * LDS, whatever the lanes; longer rows give ILU_ERR_UNSUPPORTED. */
ilu_status ilu_set_schedule(ilu_handle h, int32_t factor_sched, int32_t solve_sched,
                            int32_t lanes_factor, int32_t lanes_solve);
ilu_status ilu_get_schedule(ilu_handle h, int32_t *factor_sched, int32_t *solve_sched,
                            int32_t *lanes_factor, int32_t *lanes_solve);

/* Named tuning knobs.  Settable: "poll_sleep" (0..64, pause steps of about 64
 * clocks between polls of a value that is still pending), "tile_rows" (16..65536,
 * rebuilds the tiles of the tiled solves on the host and uploads them;
 * synchronous), "tile_lattice" (1, the default, or 0; rebuilds the tiles like
 * "tile_rows"): a matrix recognised as a 2D or 3D structured grid in natural order
 * (every factor entry joins rows at most 3 apart on each grid axis, the extents read
 * off the index offsets) is tiled in boxes of a basis of grid functionals that no
 * dependency decreases, taken in wavefront order -- cubes for ILU(0) on a 7-point
 * grid, sheared boxes once ILU(1) fill joins (x+1, y-1); 0, or any other matrix:
 * greedy growth; same results either way; read back, 1 means the current tiles are
 * boxes, "factor_tile_rows" (0, the default, or 16..65536; rebuilds the tiled
 * factor's tiles only): rows per tile of the tiled factor; the default shrinks
 * the solves' size by halves until a tile carries at most 8192 multiply-subtracts
 * of updates (ILU(0) on a 7-point grid: 512 rows; ILU(1) there: 128 rows); halved further
 * while the tile image does not fit LDS; read back, the size in use (0: no tiled
 * factor), "factor_staged" (1, the default: the sync-free and level factors
 * gather a row's dependency rows into LDS when they fit; 0: each dependency row
 * is read from global memory when its turn comes; same results).  Readable as well:
 * "nstreams" (task streams = XCDs found), "factor_tcap" (LDS entries staged per
 * factor row), "factor_tiled" (1 if the tiled factor can run on this handle:
 * rows of at most 32 entries and tiles that fit LDS).  "tail_min_rows" (0 or
 * 1..65536: rebuilds the lower stage of both solve directions as with the
 * analysis option of that name; synchronous).  "solve_blocks_per_cu" (0..8, default
 * 2: at most that many tiles of a tiled solve resident per compute unit, 0: as many
 * as LDS and waves allow; fewer tiles in flight contend less for the compute
 * unit's issue slots and LDS, which shortens each tile's level-to-level step;
 * same results).  "factor_lower_stage" (0, the default, or 1): with a tail set,
 * ilu_factor of plain ILU(k) at k = k_max runs the rows before the tail sync-free
 * and streams the tail's rows through one workgroup (ilu_copy_factor_tail); same
 * bits; readable, with "factor_lower_planned" (read only: 1 when the current tail
 * has such a plan).  "spmv_nz" (0 or 1; readable as 1 only when in use): the spmv
 * of a matrix with rows longer than 64 entries (one right-hand side, no empty
 * row) in nnz-balanced waves -- 16 consecutive entries per lane, row segments
 * added across lanes by a segmented scan and across waves by a second kernel, in a
 * fixed order -- instead of a lane group per row and one wave per long row; on by
 * default when a row exceeds 4096 entries.  "spmv_lanes" (1, 4, 8, 16, 32 or 64;
 * readable): lanes per row of the spmv's row pass; 1 takes one row per lane with
 * its entries loaded eight at a time, all in flight together (the default for rows
 * averaging at most 8 entries), otherwise a lane group per row with a butterfly sum
 * (default: half the mean row length rounded up to a power of two, at least 4);
 * same products, summed in another order.  "force_abort" (set only;
 * failure-path tests): 1 raises the device abort flag now, as an apply that timed
 * out and was not yet reported leaves it; 2 raises it inside the next apply, after
 * that apply's guard, so its kernels leave through their bounded waits (outputs
 * NaN, ilu_get_status then reports ILU_ERR_TIMEOUT).  Unknown keys give
 * ILU_ERR_ARG. */
ilu_status ilu_set_tuning(ilu_handle h, const char *key, int64_t value);
ilu_status ilu_get_tuning(ilu_handle h, const char *key, int64_t *value);

/* Times the candidate schedules of the FP64 apply and, when a_val (device values
 * in input order) is given, of the factor on this handle's matrix, and keeps the
 * fastest: level launches and sync-free launches with 1x and 2x the lanes per row
 * the rows need, and tiled launches at tile sizes 128, 256, 512 and 1024 rows (and
 * the current size).  The tile size is the level-merge threshold (a tile merges
 * consecutive levels of up to that many rows into one workgroup); the apply chooses
 * the tiling, and the tiled factor then has its own tile size timed
 * ("factor_tile_rows": its default and 64 .. 1024 rows).  The factor is re-run with the last call's k,
 * tau and flags, so the handle keeps the same factor (every schedule gives the same
 * bits).  The apply also tries the lower stage (tail_min_rows 64, or the handle's
 * own value) and keeps it if faster; with that tail in place and a plan for it, the
 * factor's lower stage ("factor_lower_stage") is timed against the chosen factor
 * schedule.  The spmv's row pass is timed at 1, 4, 8, 16, 32 and 64 lanes per row
 * ("spmv_lanes"); when the matrix has rows longer than 64 entries and no empty
 * row, its nnz-balanced pass is timed as well ("spmv_nz"); the fastest is kept.
 * Requires a factor.  Synchronous.  results (may be NULL) receives up to `cap`
 * rows of {stage (0 factor, 1 apply, 2 spmv), sched (10: lower stage; 11: tiled
 * factor at its own tile size; 20 spmv by rows, 21 spmv nnz-balanced), lanes or
 * tile rows (tiled, 11) or tail_min_rows (lower stage) or spmv lanes (20),
 * microseconds} as doubles; *n_results the row count. */
ilu_status ilu_tune(ilu_handle h, const double *a_val, int32_t reps, double *results, int32_t cap,
                    int32_t *n_results, hipStream_t stream);

/* ---------------------------------------------------------------------------- */
/* Kernel timing.                                                                 */
/* ---------------------------------------------------------------------------- */

/* Stages whose kernels are timed. */
enum {
    ILU_STAGE_FACTOR = 0,     /* the numeric factor kernel(s) */
    ILU_STAGE_FORWARD = 1,    /* forward triangular-solve kernel(s) (L, or U^T in the adjoint) */
    ILU_STAGE_BACKWARD = 2,   /* backward triangular-solve kernel(s) (U, or L^T in the adjoint) */
    ILU_STAGE_SPMV = 3,       /* spmv kernel */
    ILU_STAGE_FACTOR_CALL = 4,/* everything one ilu_factor call launches: guard, status reset, row
                                 thresholds, arming, the factor kernel(s), drop fix-up, the spmv
                                 value gather and the casts (not the status readback) */
    ILU_STAGE_APPLY_CALL = 5, /* everything one apply (or adjoint solve pair) launches: guard and
                                 both triangular solves */
    ILU_STAGE_COUNT = 6
};

/* While enabled, every stage launch on this handle is bracketed by a pair of HIP
 * events recorded on the launch's own stream (pool of `capacity` pairs; launches
 * beyond it are not timed); the *_CALL stages bracket whole calls around them.  ilu_profile_read synchronises the events, adds the
 * elapsed times per stage into ms[ILU_STAGE_COUNT] (milliseconds) and
 * launches[ILU_STAGE_COUNT], and clears the record.  Either output may be NULL. */
ilu_status ilu_profile_enable(ilu_handle h, int32_t enable, int32_t capacity);
ilu_status ilu_profile_read(ilu_handle h, double *ms, int64_t *launches);

/* ---------------------------------------------------------------------------- */
/* Calibration.                                                                   */
/* ---------------------------------------------------------------------------- */

/* Measures the floors of the current device (allocates and frees two buffers of
 * `bytes`, 0 = 2 GiB; synchronous): results[0] stream-read GB/s, [1] copy GB/s
 * (read + write bytes), [2] one published-value hop in ns between two blocks on
 * one XCD, [3] the same across XCDs (-1 if a bounded wait expired), [4] cost of
 * an empty kernel launch in us.  Up to `cap` values are written. */
ilu_status ilu_calibrate(int64_t bytes, double *results, int32_t cap);

/* ---------------------------------------------------------------------------- */
/* Lifetime and diagnostics.                                                      */
/* ---------------------------------------------------------------------------- */

ilu_status ilu_destroy(ilu_handle h);
const char *ilu_version(void);
const char *ilu_status_str(ilu_status s);
/* Copies the calling thread's last error message (NUL-terminated) into buf. */
ilu_status ilu_last_error(char *buf, int32_t len);

#ifdef __cplusplus
}
#endif

#endif /* JAVELIN_H */
