// Tiles of the triangular solves (host).
//
// The sync-free solve pays one global-memory hop (publish, then a poll on
// another compute unit) for every dependency on its critical path.  Grouping rows
// into tiles that one workgroup solves lets the dependencies inside a tile go
// through LDS instead.  Two ways of forming tiles:
//
// - Lattice boxes.  When the matrix is a 2D or 3D structured grid in natural
//   order (every factor entry joins rows whose grid coordinates differ by at most
//   kLatR per axis, the extents read off the index offsets), each direction's
//   dependency vectors are taken in grid coordinates and a unimodular basis of
//   small integer functionals is chosen that no dependency decreases.  Tiles are
//   the boxes of that basis (sides of powers of two, `cap` lattice points), so a
//   dependency between two tiles never goes from a later box coordinate to an
//   earlier one, and tiles are ordered by the sum of their box coordinates (a
//   wavefront order).  For ILU(0) on a 7-point grid the basis is the axes and the
//   tiles are cubes; the fill of ILU(1) adds dependencies such as (x+1, y-1) that
//   make axis-aligned cubes depend on each other in cycles, and the basis becomes
//   the sheared one (z, y+z, x+y+z).
// - Greedy growth, for every other matrix: Kahn's algorithm on the direction's
//   dependency graph, the next row placed being the ready row with the most
//   dependencies already in the open tile (ties: lower level, then lower index),
//   or, when no ready row touches the open tile, the ready row of lowest level.  A
//   tile closes at `cap` rows.
//
// Either way tile order is topological, which is what the kernels' start-ordered
// tile claims need to be free of deadlock.
#include <algorithm>
#include <array>
#include <climits>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <queue>
#include <set>
#include <tuple>
#include <vector>

#include "par.h"

#include "analysis.h"

namespace jv {

namespace {

// Structured-grid view of the input ordering: row i sits at x = i mod e0,
// y = (i / e0) mod e1, z = i / (e0 e1) (dim 2: y = i / e0, z = 0).
struct Lattice {
    int dim = 0;
    int64_t e0 = 0, e1 = 1;
};

constexpr int kLatR = 3;           // largest per-axis coordinate difference of a factor entry
constexpr int kLatMaxOffsets = 48; // more distinct index offsets in L: not a grid
constexpr int kLatF = 2;           // basis functionals take coefficients in [-kLatF, kLatF]

inline void lat_coords(const Lattice &L, int64_t i, int64_t c[3]) {
    c[0] = i % L.e0;
    if (L.dim == 2) {
        c[1] = i / L.e0;
        c[2] = 0;
    } else {
        c[1] = (i / L.e0) % L.e1;
        c[2] = i / (L.e0 * L.e1);
    }
}

// every offset is a + b e0 + c e0 e1 with |a|, |b|, |c| <= kLatR
bool lat_offsets_fit(const std::vector<int64_t> &D, int dim, int64_t e0, int64_t e01) {
    for (int64_t o : D) {
        bool ok = false;
        for (int c = dim == 3 ? -kLatR : 0; c <= (dim == 3 ? kLatR : 0) && !ok; ++c)
            for (int b = -kLatR; b <= kLatR && !ok; ++b) {
                const int64_t a = o - b * e0 - c * e01;
                ok = a >= -kLatR && a <= kLatR;
            }
        if (!ok) return false;
    }
    return true;
}

// Every off-diagonal factor entry joins rows at most kLatR apart on each axis.
bool lat_valid(const HostAnalysis &H, const Lattice &L) {
    for (int32_t q = 0; q < H.n; ++q) {
        int64_t a[3], b[3];
        lat_coords(L, H.perm[q], a);
        for (int32_t p = H.lu_rp[q]; p < H.lu_rp[q + 1]; ++p) {
            lat_coords(L, H.perm[H.lu_ci[p]], b);
            for (int k = 0; k < 3; ++k)
                if (a[k] - b[k] > kLatR || b[k] - a[k] > kLatR) return false;
        }
    }
    return true;
}

// Grid extents from the distinct index offsets of L's entries (input ordering):
// the x extent is an offset give or take kLatR, the xy extent likewise a large
// offset minus small multiples of the x extent.  Every extent must exceed
// 2 kLatR + 1, so that a dependency wrapping around an axis cannot pass the
// check.  Returns false when no candidate fits every entry.
bool detect_lattice(const HostAnalysis &H, Lattice *out) {
    const int64_t n = H.n;
    std::vector<int64_t> D;
    for (int32_t q = 0; q < H.n; ++q) {
        const int64_t r = H.perm[q];
        for (int32_t p = H.lu_rp[q]; p < H.diag[q]; ++p) {
            const int64_t o = r - H.perm[H.lu_ci[p]];
            if (o <= 0) return false;   // not in natural order
            if (std::find(D.begin(), D.end(), o) == D.end()) {
                if ((int)D.size() == kLatMaxOffsets) return false;
                D.push_back(o);
            }
        }
    }
    if (D.empty()) return false;
    std::sort(D.begin(), D.end());
    const int64_t emin = 2 * kLatR + 2;
    std::set<std::pair<int64_t, int64_t>> tried;
    for (int dim = 3; dim >= 2; --dim)
        for (int64_t o : D)
            for (int d0 = -kLatR; d0 <= kLatR; ++d0) {
                const int64_t e0 = o + d0;
                if (e0 < emin) continue;
                for (int64_t o2 : dim == 3 ? D : std::vector<int64_t>{0})
                    for (int b = dim == 3 ? -kLatR : 0; b <= (dim == 3 ? kLatR : 0); ++b)
                        for (int a = dim == 3 ? -kLatR : 0; a <= (dim == 3 ? kLatR : 0); ++a) {
                            const int64_t e01 = dim == 3 ? o2 - b * e0 - a : n;
                            if (e01 % e0 != 0 || e01 / e0 < emin || n % e01 != 0 || n / e01 < (dim == 3 ? emin : 1))
                                continue;
                            if (dim == 2 && n / e0 < emin) continue;
                            const std::pair<int64_t, int64_t> key{e0, dim == 3 ? e01 : 0};
                            if (!tried.insert(key).second) continue;
                            if (!lat_offsets_fit(D, dim, e0, e01)) continue;
                            Lattice L;
                            L.dim = dim;
                            L.e0 = e0;
                            L.e1 = dim == 3 ? e01 / e0 : n / e0;
                            if (lat_valid(H, L)) {
                                *out = L;
                                return true;
                            }
                        }
            }
    return false;
}

int64_t gcd64(int64_t a, int64_t b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Box tiles of one direction on a lattice.  Fills tile_of and order (rows by
// tile, in a topological order of the direction inside each tile); returns the
// tile count, or 0 when no basis of small functionals fits the dependencies.
int32_t lattice_tiles(const HostAnalysis &H, const Lattice &L, int dir, int32_t cap, const std::vector<int32_t> &lev,
                      std::vector<int32_t> &tile_of, std::vector<int32_t> &order) {
    const int32_t n = H.n;
    const int dim = L.dim;
    // dependency vectors (row minus dependency, grid coordinates)
    std::vector<std::array<int64_t, 3>> V;
    for (int32_t q = 0; q < n; ++q) {
        int64_t a[3], b[3];
        lat_coords(L, H.perm[q], a);
        const int32_t p0 = dir == 0 ? H.lu_rp[q] : H.diag[q] + 1, p1 = dir == 0 ? H.diag[q] : H.lu_rp[q + 1];
        for (int32_t p = p0; p < p1; ++p) {
            lat_coords(L, H.perm[H.lu_ci[p]], b);
            const std::array<int64_t, 3> u{a[0] - b[0], a[1] - b[1], a[2] - b[2]};
            if (std::find(V.begin(), V.end(), u) == V.end()) V.push_back(u);
        }
    }
    // admissible functionals: primitive, no dependency decreases them; cheapest first
    std::vector<std::array<int64_t, 3>> F;
    const int hi2 = dim == 3 ? kLatF : 0;
    for (int f2 = -hi2; f2 <= hi2; ++f2)
        for (int f1 = -kLatF; f1 <= kLatF; ++f1)
            for (int f0 = -kLatF; f0 <= kLatF; ++f0) {
                if (gcd64(gcd64(f0, f1), f2) != 1) continue;
                bool ok = true;
                for (const auto &u : V) ok = ok && f0 * u[0] + f1 * u[1] + f2 * u[2] >= 0;
                if (ok) F.push_back({f0, f1, f2});
            }
    auto cost = [](const std::array<int64_t, 3> &f) { return std::abs(f[0]) + std::abs(f[1]) + std::abs(f[2]); };
    std::stable_sort(F.begin(), F.end(), [&](const auto &x, const auto &y) { return cost(x) < cost(y); });
    int best[3] = {-1, -1, -1};
    int64_t best_cost = -1;
    const int nf = (int)F.size();
    for (int i = 0; i < nf; ++i)
        for (int j = i + 1; j < nf; ++j) {
            if (dim == 2) {
                const int64_t det = F[i][0] * F[j][1] - F[i][1] * F[j][0];
                const int64_t c = cost(F[i]) + cost(F[j]);
                if ((det == 1 || det == -1) && (best_cost < 0 || c < best_cost)) {
                    best_cost = c;
                    best[0] = i;
                    best[1] = j;
                }
                continue;
            }
            for (int k = j + 1; k < nf; ++k) {
                const auto &x = F[i], &y = F[j], &z = F[k];
                const int64_t det = x[0] * (y[1] * z[2] - y[2] * z[1]) - x[1] * (y[0] * z[2] - y[2] * z[0]) +
                                    x[2] * (y[0] * z[1] - y[1] * z[0]);
                const int64_t c = cost(x) + cost(y) + cost(z);
                if ((det == 1 || det == -1) && (best_cost < 0 || c < best_cost)) {
                    best_cost = c;
                    best[0] = i;
                    best[1] = j;
                    best[2] = k;
                }
            }
        }
    if (best_cost < 0) return 0;
    // box sides: powers of two, as even as possible, product at most cap
    int64_t side[3] = {1, 1, 1}, prod = 1;
    for (int i = 0; prod * 2 <= cap; ++i) {
        side[i % dim] *= 2;
        prod *= 2;
    }
    // box coordinates of every row
    std::vector<int64_t> g((size_t)n * dim);
    int64_t gmin[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
    for (int32_t q = 0; q < n; ++q) {
        int64_t a[3];
        lat_coords(L, H.perm[q], a);
        for (int i = 0; i < dim; ++i) {
            const auto &f = F[best[i]];
            const int64_t v = f[0] * a[0] + f[1] * a[1] + f[2] * a[2];
            g[(size_t)q * dim + i] = v;
            gmin[i] = std::min(gmin[i], v);
        }
    }
    int64_t nb[3] = {1, 1, 1};
    for (int32_t q = 0; q < n; ++q)
        for (int i = 0; i < dim; ++i) {
            int64_t &v = g[(size_t)q * dim + i];
            v = (v - gmin[i]) / side[i];
            nb[i] = std::max(nb[i], v + 1);
        }
    // wavefront order of boxes: sum of box coordinates, then the coordinates
    std::vector<int64_t> key(n);
    for (int32_t q = 0; q < n; ++q) {
        int64_t s = 0, k = 0;
        for (int i = 0; i < dim; ++i) {
            s += g[(size_t)q * dim + i];
            k = k * nb[i] + g[(size_t)q * dim + i];
        }
        key[q] = s * nb[0] * nb[1] * nb[2] + k;
    }
    std::vector<int64_t> keys(key);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    for (int32_t q = 0; q < n; ++q)
        tile_of[q] = (int32_t)(std::lower_bound(keys.begin(), keys.end(), key[q]) - keys.begin());
    order.resize(n);
    for (int32_t q = 0; q < n; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return tile_of[x] != tile_of[y] ? tile_of[x] < tile_of[y] : lev[x] < lev[y];
    });
    return (int32_t)keys.size();
}

// Greedy growth (see the file comment).  Fills tile_of and order (placement
// order, topological) and returns the tile count.
int32_t greedy_tiles(const HostAnalysis &H, int dir, int32_t cap, const std::vector<int32_t> &lev,
                     std::vector<int32_t> &tile_of, std::vector<int32_t> &order) {
    const int32_t n = H.n;
    const std::vector<int32_t> &rp = H.lu_rp, &ci = H.lu_ci, &dg = H.diag;
    auto dbeg = [&](int32_t r) { return dir == 0 ? rp[r] : dg[r] + 1; };
    auto dend = [&](int32_t r) { return dir == 0 ? dg[r] : rp[r + 1]; };
    // successor lists
    std::vector<int32_t> sp(n + 1, 0), indeg(n, 0);
    for (int32_t r = 0; r < n; ++r) {
        indeg[r] = dend(r) - dbeg(r);
        for (int32_t p = dbeg(r); p < dend(r); ++p) ++sp[ci[p] + 1];
    }
    for (int32_t i = 0; i < n; ++i) sp[i + 1] += sp[i];
    std::vector<int32_t> sv(sp[n]), fill(sp.begin(), sp.end() - 1);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t p = dbeg(r); p < dend(r); ++p) sv[fill[ci[p]]++] = r;

    using Seed = std::pair<int32_t, int32_t>;                       // (level, row), smallest first
    std::priority_queue<Seed, std::vector<Seed>, std::greater<Seed>> seed;
    using Hot = std::tuple<int32_t, int32_t, int32_t>;              // (score, -level, -row), largest first
    std::priority_queue<Hot> hot;
    std::vector<int32_t> score(n, 0), touched;
    std::vector<char> placed(n, 0);
    order.clear();
    order.reserve(n);
    for (int32_t r = 0; r < n; ++r)
        if (indeg[r] == 0) seed.push({lev[r], r});
    int32_t cur = 0, size = 0;
    while ((int32_t)order.size() < n) {
        int32_t r = -1;
        while (!hot.empty()) {
            const int32_t x = -std::get<2>(hot.top());
            hot.pop();
            if (!placed[x]) {
                r = x;
                break;
            }
        }
        while (r < 0) {   // the graph is acyclic, so an unplaced ready row exists
            const int32_t x = seed.top().second;
            seed.pop();
            if (!placed[x]) r = x;
        }
        placed[r] = 1;
        tile_of[r] = cur;
        order.push_back(r);
        ++size;
        for (int32_t q = sp[r]; q < sp[r + 1]; ++q) {
            const int32_t s = sv[q];
            if (score[s]++ == 0) touched.push_back(s);
            if (--indeg[s] == 0) {
                seed.push({lev[s], s});
                hot.push({score[s], -lev[s], -s});
            }
        }
        if (size == cap) {
            ++cur;
            size = 0;
            for (int32_t s : touched) score[s] = 0;
            touched.clear();
            hot = std::priority_queue<Hot>();
        }
    }
    return cur + (size > 0 ? 1 : 0);
}

void tiles_one(const HostAnalysis &H, int dir, int32_t cap, int32_t short_row, const Lattice *lat, TileSet *T,
               std::vector<int32_t> *sci) {
    const int32_t n = H.n;
    const std::vector<int32_t> &rp = H.lu_rp, &ci = H.lu_ci, &dg = H.diag;
    auto dbeg = [&](int32_t r) { return dir == 0 ? rp[r] : dg[r] + 1; };
    auto dend = [&](int32_t r) { return dir == 0 ? dg[r] : rp[r + 1]; };

    // level of every row in this direction
    std::vector<int32_t> lev(n, 0);
    if (dir == 0) {
        for (int32_t l = 0; l < H.n_levels; ++l)
            for (int32_t q = H.level_ptr[l]; q < H.level_ptr[l + 1]; ++q) lev[q] = l;
    } else {
        for (int32_t l = 0; l < H.n_ulevels; ++l)
            for (int32_t q = H.ulevel_ptr[l]; q < H.ulevel_ptr[l + 1]; ++q) lev[H.ulevel_rows[q]] = l;
    }
    std::vector<int32_t> tile_of(n, -1), order;
    int32_t ntiles = lat ? lattice_tiles(H, *lat, dir, cap, lev, tile_of, order) : 0;
    if (ntiles == 0) ntiles = greedy_tiles(H, dir, cap, lev, tile_of, order);

    // local levels (placement order is topological)
    std::vector<int32_t> llev(n, 0);
    for (int32_t r : order)
        for (int32_t p = dbeg(r); p < dend(r); ++p) {
            const int32_t c = ci[p];
            if (tile_of[c] == tile_of[r]) llev[r] = std::max(llev[r], llev[c] + 1);
        }
    // per tile: rows by local level (stable in placement order), each level padded;
    // slots: rows in position order, then the tile's imports
    T->kmax = 0;
    for (int32_t r = 0; r < n; ++r) T->kmax = std::max(T->kmax, dend(r) - dbeg(r));
    const int32_t unit = T->kmax <= short_row ? 64 : 16;
    T->cap = cap;
    T->unit = unit;
    T->ntiles = ntiles;
    T->max_rows = T->max_slots = T->max_pos = T->max_imps = 0;
    T->ptr.assign(1, 0);
    T->row.clear();
    T->rows_ptr.assign(1, 0);
    T->rows.clear();
    T->imp_ptr.assign(1, 0);
    T->imp.clear();
    std::vector<int32_t> slot(n, -1), imp_slot(n, -1);
    size_t a = 0;
    for (int32_t t = 0; t < ntiles; ++t) {
        size_t b = a;
        while (b < order.size() && tile_of[order[b]] == t) ++b;
        std::vector<int32_t> rows(order.begin() + a, order.begin() + b);
        std::stable_sort(rows.begin(), rows.end(), [&](int32_t x, int32_t y) { return llev[x] < llev[y]; });
        const size_t base = T->row.size();
        int32_t nslot = 0;
        for (size_t i = 0; i < rows.size();) {
            size_t j = i;
            while (j < rows.size() && llev[rows[j]] == llev[rows[i]]) ++j;
            for (size_t k = i; k < j; ++k) {
                slot[rows[k]] = nslot++;
                T->row.push_back(rows[k]);
                T->rows.push_back(rows[k]);
            }
            while ((T->row.size() - base) % unit) T->row.push_back(-1);
            i = j;
        }
        // imports, in order of first use
        const size_t ibase = T->imp.size();
        for (int32_t r : rows)
            for (int32_t p = dbeg(r); p < dend(r); ++p) {
                const int32_t c = ci[p];
                if (tile_of[c] != t && imp_slot[c] < 0) {
                    imp_slot[c] = nslot + (int32_t)(T->imp.size() - ibase);
                    T->imp.push_back(c);
                }
            }
        for (int32_t r : rows)
            for (int32_t p = dbeg(r); p < dend(r); ++p) {
                const int32_t c = ci[p];
                (*sci)[p] = tile_of[c] == t ? slot[c] : imp_slot[c];
            }
        for (size_t i = ibase; i < T->imp.size(); ++i) imp_slot[T->imp[i]] = -1;
        T->ptr.push_back((int32_t)T->row.size());
        T->rows_ptr.push_back((int32_t)T->rows.size());
        T->imp_ptr.push_back((int32_t)T->imp.size());
        T->max_rows = std::max<int32_t>(T->max_rows, nslot);
        T->max_slots = std::max<int32_t>(T->max_slots, nslot + (int32_t)(T->imp.size() - ibase));
        T->max_pos = std::max<int32_t>(T->max_pos, (int32_t)(T->row.size() - base));
        T->max_imps = std::max<int32_t>(T->max_imps, (int32_t)(T->imp.size() - ibase));
        a = b;
    }
}

}  // namespace

int build_tiles(const HostAnalysis &H, int32_t cap, int32_t short_row, bool lattice, TileSet *fwd, TileSet *bwd,
                std::vector<int32_t> *sci) {
    sci->assign(H.lu_ci.size(), -1);
    Lattice L;
    const bool lat = lattice && detect_lattice(H, &L);
    // the directions write disjoint entries of sci (lower and upper parts of each
    // row): built side by side
    run_pair([&] { tiles_one(H, 0, cap, short_row, lat ? &L : nullptr, fwd, sci); },
             [&] { tiles_one(H, 1, cap, short_row, lat ? &L : nullptr, bwd, sci); });
    return lat ? L.dim : 0;
}

void build_forward_tiles(const HostAnalysis &H, int32_t cap, int32_t short_row, bool lattice, TileSet *fwd) {
    std::vector<int32_t> sci(H.lu_ci.size(), -1);
    Lattice L;
    const bool lat = lattice && detect_lattice(H, &L);
    tiles_one(H, 0, cap, short_row, lat ? &L : nullptr, fwd, &sci);
}

namespace {

size_t a16(size_t b) { return (b + 15) & ~(size_t)15; }

// Tile t's header, blob and value sources (its tables are the last ones appended
// to F's per-entry arrays).  F holds the tiles from tb on, whose first row
// position is rb (its per-row and per-tile arrays are indexed from there).  A
// tile whose offsets do not fit the packed fields makes the whole set unusable
// (lds_need beyond any LDS).
void append_tile_blob(const HostAnalysis &H, const TileSet &T, int32_t t, int32_t lanes, int32_t tb, int32_t rb,
                      FactorTiles *F) {
    const int32_t r0 = T.rows_ptr[t], nrows = T.rows_ptr[t + 1] - r0;
    const int32_t l0 = F->lptr[t - tb], nl = F->lptr[t - tb + 1] - l0;
    const int32_t i0 = T.imp_ptr[t], nimp = T.imp_ptr[t + 1] - i0;
    const int32_t p0 = T.ptr[t], npos = T.ptr[t + 1] - p0;
    size_t o = 0;
    const size_t o_rows = o;
    o = a16(o + (size_t)nrows * 16);
    const size_t o_lent = o;
    o = a16(o + (size_t)nl * 4);
    const size_t o_match = o;
    o = a16(o + (size_t)nl * lanes);
    const size_t o_imp = o;
    o = a16(o + (size_t)nimp * 16);
    const size_t o_ps = o;
    o = a16(o + (size_t)npos * 2);
    std::vector<unsigned char> b(o, 0);
    bool packs = nrows + nimp <= 65536;
    int32_t *rw = reinterpret_cast<int32_t *>(b.data() + o_rows);
    for (int32_t k = 0; k < nrows; ++k) {
        const int32_t *m = F->meta.data() + 4 * (size_t)(r0 - rb + k), *of = F->off.data() + 2 * (size_t)(r0 - rb + k);
        const int32_t len = m[2] - m[1], K = m[3] - m[1];
        packs = packs && of[0] < 65536 && len < 256 && K < 256;
        rw[4 * k] = m[0];
        rw[4 * k + 1] = m[1];
        rw[4 * k + 2] = of[0] | len << 16 | K << 24;
        rw[4 * k + 3] = of[1];
    }
    uint32_t *le = reinterpret_cast<uint32_t *>(b.data() + o_lent);
    for (int32_t k = 0; k < nl; ++k) {
        const int32_t dl = F->dloc[l0 + k], df = F->dflag[l0 + k];
        packs = packs && dl < 65536;
        le[k] = (uint32_t)dl | (uint32_t)df << 16;
    }
    std::memcpy(b.data() + o_match, F->match.data() + (size_t)l0 * lanes, (size_t)nl * lanes);
    const size_t fi0 = F->imp.size() - 4 * (size_t)nimp;   // this tile's imports: the last appended
    std::memcpy(b.data() + o_imp, F->imp.data() + fi0, (size_t)nimp * 16);
    int16_t *ps = reinterpret_cast<int16_t *>(b.data() + o_ps);
    for (int32_t q = 0, k = 0; q < npos; ++q) ps[q] = (int16_t)(T.row[p0 + q] >= 0 ? k++ : -1);
    // value sources of the rows, in value-area order
    const int32_t vbase = (int32_t)F->vsrc.size();
    for (int32_t q = r0; q < r0 + nrows; ++q) {
        const int32_t r = T.rows[q];
        for (int32_t p = H.lu_rp[r]; p < H.lu_rp[r + 1]; ++p) F->vsrc.push_back(H.lu_src[p]);
    }
    const int32_t nvr = (int32_t)F->vsrc.size() - vbase;
    int32_t nvals = nvr;
    for (int32_t i = 0; i < nimp; ++i) nvals = std::max(nvals, F->imp[fi0 + 4 * i + 2] + F->imp[fi0 + 4 * i + 1]);
    packs = packs && nvals <= 65536;
    const int32_t boff = (int32_t)(F->blob.size() / 4);
    F->blob.resize(F->blob.size() + o / 4);
    std::memcpy(F->blob.data() + 4 * (size_t)boff, b.data(), o);
    int32_t h[kFactorHdr] = {boff, (int32_t)(o / 16), nrows, nimp, nl, npos, (int32_t)o_lent, (int32_t)o_match,
                             (int32_t)o_imp, (int32_t)o_ps, vbase, nvr, nvals, l0};
    F->hdr.insert(F->hdr.end(), h, h + kFactorHdr);
    // LDS: values, ready words, the blob, then the thresholds and masks if used
    const size_t base = a16((size_t)nvals * 8) + a16((size_t)(nrows + nimp) * 8) + o;
    for (int v = 0; v < 4; ++v) {
        const size_t need = packs ? base + ((v & 1) ? (size_t)nrows * 8 : 0) + ((v & 2) ? (size_t)nl * 4 : 0)
                                  : SIZE_MAX;
        F->lds_need[v] = std::max(F->lds_need[v], need);
    }
}

// Tiles [tb, te) into F, indexed from tile tb and its first row position.
void build_factor_range(const HostAnalysis &H, const TileSet &T, int32_t lanes, int32_t tb, int32_t te,
                        FactorTiles *F) {
    const std::vector<int32_t> &rp = H.lu_rp, &ci = H.lu_ci, &dg = H.diag;
    const int32_t rb = T.rows_ptr[tb];
    F->lanes = lanes;
    F->max_vals = F->max_lents = 0;
    F->hdr.clear();
    F->blob.clear();
    F->vsrc.clear();
    for (size_t &x : F->lds_need) x = 0;
    F->meta.clear();
    F->off.clear();
    F->lptr.assign(1, 0);
    F->dloc.clear();
    F->dflag.clear();
    F->match.clear();
    F->cmask.clear();
    F->imp.clear();
    std::vector<int32_t> slot_of(H.n, -1), imp_of(H.n, -1), iloc(H.n, -1);
    for (int32_t t = tb; t < te; ++t) {
        const int32_t r0 = T.rows_ptr[t], r1 = T.rows_ptr[t + 1];
        const int32_t nrows = r1 - r0;
        // value area: rows in slot order, then imports' U parts
        int32_t va = 0, la = 0;
        for (int32_t q = r0; q < r1; ++q) {
            const int32_t r = T.rows[q];
            slot_of[r] = q - r0;
            F->meta.insert(F->meta.end(), {r, rp[r], rp[r + 1], dg[r]});
            F->off.insert(F->off.end(), {va, la});
            va += rp[r + 1] - rp[r];
            la += dg[r] - rp[r];
        }
        for (int32_t i = T.imp_ptr[t]; i < T.imp_ptr[t + 1]; ++i) {
            const int32_t c = T.imp[i];
            imp_of[c] = i - T.imp_ptr[t];
            iloc[c] = va;
            F->imp.insert(F->imp.end(), {dg[c], rp[c + 1] - dg[c], va, 0});
            va += rp[c + 1] - dg[c];
        }
        F->max_vals = std::max(F->max_vals, va);
        F->max_lents = std::max(F->max_lents, la);
        // L entries
        for (int32_t q = r0; q < r1; ++q) {
            const int32_t r = T.rows[q];
            const size_t lfirst = F->dloc.size();
            for (int32_t p = rp[r]; p < dg[r]; ++p) {
                const int32_t c = ci[p];
                if (slot_of[c] >= 0) {
                    F->dloc.push_back(F->off[2 * (r0 - rb + slot_of[c])] + (dg[c] - rp[c]));
                    F->dflag.push_back(slot_of[c]);
                } else {
                    F->dloc.push_back(iloc[c]);
                    F->dflag.push_back(nrows + imp_of[c]);
                }
                // U(c) columns, diagonal first; both rows are sorted: merge
                for (int32_t l = 0; l < lanes; ++l) {
                    int8_t m = -1;
                    const int32_t pe = rp[r] + l;
                    if (pe < rp[r + 1]) {
                        const int32_t col = ci[pe];
                        const int32_t *b = ci.data() + dg[c] + 1, *e = ci.data() + rp[c + 1];
                        const int32_t *f = std::lower_bound(b, e, col);
                        if (f != e && *f == col) m = (int8_t)(f - (ci.data() + dg[c]));
                    }
                    F->match.push_back(m);
                }
                uint32_t cm = 0;
                for (int32_t j = 1; j < rp[c + 1] - dg[c]; ++j) {
                    const int32_t col = ci[dg[c] + j];
                    if (col == r || !std::binary_search(ci.data() + rp[r], ci.data() + rp[r + 1], col))
                        cm |= 1u << j;
                }
                F->cmask.push_back(cm);
            }
            // a row whose L entries never update one another (no L entry's column
            // lies in U(c) of an earlier L entry c) has independent multipliers:
            // its row id is stored complemented to say so
            const int32_t nl = dg[r] - rp[r];
            bool flat = true;
            for (int32_t e1 = 0; e1 < nl && flat; ++e1)
                for (int32_t e2 = e1 + 1; e2 < nl; ++e2)
                    if (F->match[(lfirst + e1) * lanes + e2] > 0) {
                        flat = false;
                        break;
                    }
            if (flat) F->meta[4 * (size_t)(q - rb)] = ~r;
        }
        F->lptr.push_back((int32_t)F->dloc.size());
        append_tile_blob(H, T, t, lanes, tb, rb, F);
        for (int32_t q = r0; q < r1; ++q) slot_of[T.rows[q]] = -1;
        for (int32_t i = T.imp_ptr[t]; i < T.imp_ptr[t + 1]; ++i) {
            imp_of[T.imp[i]] = -1;
            iloc[T.imp[i]] = -1;
        }
    }
}

}  // namespace

// Ranges of tiles are built side by side, each into a part of its own, and the
// parts concatenated: the tables a tile stages are tile-local, so only the
// global offsets (a tile's blob, value sources and first L entry, and the L
// pointers) move by what the earlier parts hold.
void build_factor_tiles(const HostAnalysis &H, const TileSet &T, int32_t lanes, FactorTiles *F) {
    std::vector<FactorTiles> part(host_threads());
    const int nparts = parallel_chunks(T.ntiles, 64, [&](int c, int64_t lo, int64_t hi) {
        build_factor_range(H, T, lanes, (int32_t)lo, (int32_t)hi, &part[c]);
    });
    if (nparts == 1) {
        *F = std::move(part[0]);
        return;
    }
    FactorTiles &out = *F;
    out = FactorTiles();
    out.lanes = lanes;
    out.lptr.assign(1, 0);
    for (int c = 0; c < nparts; ++c) {
        FactorTiles &P = part[c];
        const int32_t loff = out.lptr.back(), voff = (int32_t)out.vsrc.size(), boff = (int32_t)(out.blob.size() / 4);
        out.max_vals = std::max(out.max_vals, P.max_vals);
        out.max_lents = std::max(out.max_lents, P.max_lents);
        for (int v = 0; v < 4; ++v) out.lds_need[v] = std::max(out.lds_need[v], P.lds_need[v]);
        for (size_t k = 1; k < P.lptr.size(); ++k) out.lptr.push_back(P.lptr[k] + loff);
        for (size_t h = 0; h < P.hdr.size(); h += kFactorHdr) {
            P.hdr[h + kFhBlob] += boff;
            P.hdr[h + kFhVsrc] += voff;
            P.hdr[h + kFhL0] += loff;
        }
        auto cat = [](auto &dst, auto &src) {
            dst.insert(dst.end(), src.begin(), src.end());
            std::vector<typename std::decay_t<decltype(src)>::value_type>().swap(src);
        };
        cat(out.meta, P.meta);
        cat(out.off, P.off);
        cat(out.dloc, P.dloc);
        cat(out.dflag, P.dflag);
        cat(out.match, P.match);
        cat(out.cmask, P.cmask);
        cat(out.imp, P.imp);
        cat(out.hdr, P.hdr);
        cat(out.blob, P.blob);
        cat(out.vsrc, P.vsrc);
    }
}

}  // namespace jv
