// Host-side analysis of the incomplete-LU hot path: intake, fill pattern, level
// schedule, permuted structure.  Plain C++ (no HIP); the result is uploaded by the
// C-ABI layer.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "javelin.h"

namespace jv {

struct HostAnalysis {
    int32_t n = 0;
    int64_t nnz_in = 0;
    int32_t k_max = 0;
    int32_t pattern = ILU_PATTERN_LOWER_SYM;
    std::vector<int32_t> in_rp;        // input row pointers (row norms for the tau test)

    // level schedule of the forward direction (factor and L solve)
    int32_t n_levels = 0;
    std::vector<int32_t> level_ptr;    // [n_levels + 1], rows of level l are [ptr[l], ptr[l+1])
    std::vector<int32_t> perm;         // level ordering -> input ordering
    std::vector<int32_t> iperm;        // input ordering -> level ordering
    std::vector<int32_t> order;        // preordering applied before the analysis (empty: none)

    // factor structure P S P^T in level order
    std::vector<int32_t> lu_rp, lu_ci, diag, lu_src;
    std::vector<int8_t> flev;          // fill level of each factor entry
    int32_t max_row_lu = 0;
    int32_t max_lower_lu = 0;          // longest strictly-lower part of a row
    int32_t max_upper_lu = 0;          // longest strictly-upper part of a row

    // permuted copy of A (inserted diagonals as explicit zeros)
    std::vector<int32_t> b_rp, b_ci, b_src;
    int32_t max_row_b = 0;

    // backward (U solve) schedule
    int32_t n_ulevels = 0;
    std::vector<int32_t> ulevel_ptr, ulevel_rows;

    // transposed factor structure for the adjoint: row j of (LU)^T holds column j
    std::vector<int32_t> t_rp, t_ci, t_map, t_diag;   // t_map: entry of (LU)^T -> entry of LU
    int32_t n_tlevels = 0, n_tulevels = 0;            // levels of U^T (forward) and L^T (backward)
    std::vector<int32_t> tlevel_ptr, tlevel_rows, tulevel_ptr, tulevel_rows;
};

// Tiles of one triangular-solve direction (dir 0: L, columns < r; dir 1: U,
// columns > r).  A tile is a set of rows that one workgroup solves with its
// values held in LDS; tiles are numbered in a topological order of the
// direction's dependency graph (every dependency of a row lies in an earlier tile
// or in the same tile).  Inside a tile, rows are sorted by local level (longest
// path over dependencies inside the tile) and every local level is padded with -1
// to a multiple of `unit` positions, so no run of `unit` consecutive positions
// mixes two local levels.
//
// LDS slots of a tile: its real rows in position order (0 .. rows-1), then its
// imports (the distinct dependencies that lie in other tiles).  Every
// off-diagonal entry of the direction is encoded by the slot of its column.
struct TileSet {
    int32_t cap = 0;                   // rows per tile requested (last tile may be smaller)
    int32_t unit = 0;                  // positions per wave chunk
    int32_t ntiles = 0;
    int32_t max_rows = 0;              // most rows in one tile
    int32_t max_slots = 0;             // most rows + imports in one tile
    int32_t max_pos = 0;               // most positions (rows + padding) in one tile
    int32_t max_imps = 0;              // most imports of one tile
    int32_t kmax = 0;                  // longest dependency list of a row
    std::vector<int32_t> ptr;          // [ntiles + 1] padded positions
    std::vector<int32_t> row;          // row (level ordering) at each position, -1 for padding
    std::vector<int32_t> rows_ptr;     // [ntiles + 1] offsets of each tile's rows in slot order
    std::vector<int32_t> rows;         // rows of each tile in slot order
    std::vector<int32_t> imp_ptr;      // [ntiles + 1] offsets of each tile's imports
    std::vector<int32_t> imp;          // imported rows (slot rows + i holds imp[imp_ptr[t] + i])
};

// Builds both directions' tiles and the solve column encoding: for every factor
// entry p = (r, c) with c != r, sci[p] = LDS slot of c in r's tile of the
// direction that reads the entry; diagonal entries get -1.  A direction whose
// rows have at most short_row dependencies is padded to chunks of 64 positions
// (one lane per row), otherwise to chunks of 16 (four lanes per row).  With
// `lattice`, a matrix recognised as a structured grid in natural order gets box
// tiles (returns the grid's dimension, 2 or 3), any other the greedy growth
// (returns 0).
int build_tiles(const HostAnalysis &H, int32_t cap, int32_t short_row, bool lattice, TileSet *fwd, TileSet *bwd,
                std::vector<int32_t> *sci);

// Forward tiles only (a tiling of its own for the factor when the solves' tiles
// are too large for its LDS image).
void build_forward_tiles(const HostAnalysis &H, int32_t cap, int32_t short_row, bool lattice, TileSet *fwd);

// Lower stage ("tail") of one triangular-solve direction: the longest suffix of
// its level order whose levels hold fewer than min_rows rows, cut into steps (rows
// of one level solved together by one wave; a row with more than 64 * kTailJ
// dependencies gets consecutive steps of its own whose partial sums carry over).
constexpr int kTailJ = 2;        // dependencies per lane
constexpr int kTailQ = 24;       // steps staged ahead (LDS buffers)
constexpr int kTailW = 2048;     // ring of recent results (power of two; at least 64 steps of 32 rows,
                                 // so that values not in the ring are kTailQ or more steps old)
constexpr int kTailRows = 32;    // most rows in one step
constexpr int kTailCarryIn = 1;  // step flag: add the previous step's partial sum
constexpr int kTailEmit = 2;     // step flag: the step finishes its rows
struct TailPlan {
    int32_t level0 = -1;         // first tail level (-1: no tail)
    int32_t pos0 = 0;            // first tail position in the direction's order
    int32_t nsteps = 0;
    int32_t max_rows = 0, max_lanes = 0;
    // 4 per step (+ a sentinel): record offset in `rec`,
    // nrows | nlanes << 8 | log2(largest lane group) << 16 | flags << 24, entries, 0
    std::vector<int32_t> hdr;
    // per step (starting at a multiple of 4 words): per row 4 words (row in the
    // level ordering, its ring slot, its input-ordering row, its diagonal entry),
    // lanes (row in the step | log2 group << 8 | leader << 16) [nlanes], then per entry
    // (lane-major, entry (lane, j) at j * nlanes + lane) the factor entry [nent]
    // (-1: none) and the source of the dependency value [nent]: a ring slot
    // (< kTailW; no row written since holds the same slot), kTailW + row (read
    // from the published buffer), or -1 (none)
    std::vector<int32_t> rec;
};
// dir 0: forward (L), 1: backward (U).  No tail when min_rows <= 0 or the suffix
// has fewer than min_levels levels.
void build_tail(const HostAnalysis &H, int dir, int32_t min_rows, int32_t min_levels, TailPlan *T);

// Lower stage of the numeric factor (plain ILU(k) at k = k_max): the rows of the
// forward solve's tail, cut into steps of rows of one level; a row gets an aligned
// group of 2^g >= its length lanes, lane t holding entry t.  Per row: its record
// {row, first factor entry, len | K << 8 | g << 16 | first lane << 24, ring base}
// and {first L-entry source, first match byte, 0, 0}; per L entry e the source of
// U(c_e): its ring base (>= 0: c_e's U part is in the LDS ring of recent rows)
// or -(diag(c_e) + 1) (read from the factor buffer); per L entry e and entry t of
// the row (e-major, len bytes per e) the position of entry t's column in U(c_e)
// (0 for t == e, the pivot; 255 none).  Per step: {first row record, rows, most L
// entries of a row, lane map offset}; the lane map gives each of the 64 lanes its
// row in the step (255: idle).  The ring holds kFTailRing values: ring_rows
// slots of umax entries, a row's slot at (row mod ring_rows).  A U part read
// from the ring was written at most ring_rows rows (in level order) before the
// step's last row; the stagers work q steps ahead, and every source fewer than q
// steps old is in the ring.
constexpr int kFTailK = 16;      // most L entries of a tail row
constexpr int kFTailQ = 6;       // most steps staged ahead
constexpr int kFTailRing = 8192; // ring entries (FP64)
struct FactorTailPlan {
    int32_t level0 = -1, pos0 = 0, nsteps = 0;
    int32_t umax = 0, ring_rows = 0, q = 0;
    std::vector<int32_t> hdr;     // 4 per step
    std::vector<int32_t> rows;    // 8 per row record
    std::vector<int32_t> lsrc;    // per L entry
    std::vector<uint8_t> match;   // per L entry and row entry
    std::vector<uint8_t> lmap;    // 64 per step
};
// false (no plan) when the forward solve has no tail, a tail row is longer than 64
// entries or has more than kFTailK L entries, or no staging depth of at least 2
// steps keeps every recent source in the ring
bool build_factor_tail(const HostAnalysis &H, const TailPlan &fwd, FactorTailPlan *T);

// Data of the tiled factor on the forward tiles.  LDS of a tile: the value area
// (the tile's rows' entries in slot order, then the U parts -- diagonal first -- of
// its imports) and one ready flag per tile row and per import.  Per tile row:
// meta (row, first entry, end entry, diagonal entry; the row is stored as ~row
// when its L entries never update one another, so that its multipliers are
// independent) and (value-area offset, offset of its first L entry among the
// tile's L entries).  Per L entry
// (r, c) in tile order: the value-area location of U(c)'s diagonal, the ready
// flag of c, and for each lane t < lanes the index j >= 1 in U(c) of the column
// of entry t of row r (-1 if that column is not in U(c)).  Per import: the factor
// entry of its diagonal, the length of its U part, its value-area offset.
struct FactorTiles {
    int32_t lanes = 0;                 // lanes per row (>= longest row)
    int32_t max_vals = 0;              // largest value area (entries)
    int32_t max_lents = 0;             // most L entries in one tile
    std::vector<int32_t> meta;         // 4 per tile row (slot order, tiles concatenated)
    std::vector<int32_t> off;          // 2 per tile row: value-area offset, L-entry offset
    std::vector<int32_t> lptr;         // [ntiles + 1] offsets of each tile's L entries
    std::vector<int32_t> dloc, dflag;  // per L entry
    std::vector<int8_t> match;         // lanes per L entry
    std::vector<uint32_t> cmask;       // per L entry (r, c): bit j set for each position j >= 1 of U(c)
                                       // whose update goes to u_rr in modified ILU (column r, or a
                                       // column that row r does not hold)
    std::vector<int32_t> imp;          // 4 per import: diagonal entry, U length, value-area offset, 0
    // What one tile stages, in one piece: per tile kFactorHdr words of header (see
    // FactorHdr), its tables as one 16-byte aligned blob in the order and layout
    // they take in LDS, and the input entry of each of its rows' value slots (-1:
    // fill).  lds_need[tau + 2 * modified]: bytes of LDS the largest tile needs.
    std::vector<int32_t> hdr;
    std::vector<int32_t> blob;         // 16-byte units (4 words each)
    std::vector<int32_t> vsrc;
    size_t lds_need[4] = {0, 0, 0, 0};
};

// Header words of a factor tile: blob offset and size (16-byte units), rows,
// imports, L entries, positions; byte offsets in the blob of the L-entry, match,
// import and position-slot tables (the row table at 0); first value-source
// entry, row value slots, all value slots (imports included), first L entry.
// Blob tables: per row int4 (row, complemented when its L entries are
// independent; first factor entry; value-area offset | length << 16 | L
// entries << 24; first L entry of the tile's L table), per L entry the LDS
// location of its U row | that row's ready slot << 16, per L entry and lane the
// lane's column position in that U row (0: none), per import int4 (diagonal
// entry, U length, value-area offset, 0), per position the row slot (-1: padding).
enum FactorHdr {
    kFhBlob, kFhBlobSize, kFhRows, kFhImps, kFhLents, kFhPos, kFhLent, kFhMatch, kFhImp, kFhPs,
    kFhVsrc, kFhRowVals, kFhVals, kFhL0, kFactorHdr = 16
};

// Builds the tiled-factor data from the forward tiles; lanes = power of two >= the
// longest factor row (the caller checks it is at most 16).
void build_factor_tiles(const HostAnalysis &H, const TileSet &fwd, int32_t lanes, FactorTiles *F);

// Returns ILU_OK or an error status with a message in *err.  ordering:
// ILU_ORDER_NATURAL (A as given) or ILU_ORDER_RCM (A preordered by reverse
// Cuthill-McKee; perm and the entry maps then refer to the input ordering).
ilu_status analyze_host(int32_t n, const int32_t *rp, const int32_t *ci, int64_t nnz, int32_t k_max,
                        int32_t pattern, int32_t ordering, HostAnalysis *out, std::string *err);

// Reverse Cuthill-McKee order of the graph of A + A^T: order[i] = input vertex i'.
std::vector<int32_t> rcm_order(int32_t n, const int32_t *rp, const int32_t *ci);

}  // namespace jv
