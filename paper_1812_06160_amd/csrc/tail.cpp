// Lower stage of the triangular solves (host plan).
//
// Sec. III-B ("Lower Stage", Fig. 7) moves the rows that level scheduling cannot
// keep busy -- the narrow levels at the end of the level order -- into a second
// stage that a few workers take in order.  Here the lower stage ("tail") of a
// solve direction is the longest suffix of its level order whose levels all hold
// fewer than `min_rows` rows; every dependency of a tail row lies in an earlier
// level, so the suffix is closed under "depends on a tail row".  One workgroup
// streams the tail: a compute wave walks it level by level while stager waves
// fetch what each step needs ahead of it.  Rows of the upper stage are finished
// before the tail starts (the paper's rows-in-parallel part: their values are
// simply read), tail values that were computed a few steps earlier are read from
// a ring in LDS, older ones from the published buffer.
//
// A step is a group of rows of one level that the compute wave solves at once:
// row k gets an aligned group of G_k lanes (G_k a power of two with G_k * kTailJ
// >= its dependencies) and the groups are packed in descending size into the 64
// lanes; the row's dependencies go to its lanes, kTailJ per lane, and the group's
// partial sums are added by a butterfly over the group.  A row with more
// dependencies than one wave holds is split over consecutive steps of its own,
// whose partial sums carry from one step to the next (the segmented-rows idea of
// Sec. III-B applied to one long row).
#include <algorithm>
#include <vector>

#include "analysis.h"

namespace jv {

namespace {

int log2_ceil(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

void build_tail(const HostAnalysis &H, int dir, int32_t min_rows, int32_t min_levels, TailPlan *T) {
    *T = TailPlan();
    if (min_rows <= 0) return;
    const int32_t n = H.n;
    const std::vector<int32_t> &lp = dir == 0 ? H.level_ptr : H.ulevel_ptr;
    const int32_t nl = (int32_t)lp.size() - 1;
    int32_t t = nl;
    while (t > 0 && lp[t] - lp[t - 1] < min_rows) --t;
    if (nl - t < std::max(1, min_levels)) return;
    T->level0 = t;
    T->pos0 = lp[t];
    auto row_at = [&](int32_t q) { return dir == 0 ? q : H.ulevel_rows[q]; };
    std::vector<int32_t> pos_of;   // backward: row -> position in the U order
    if (dir == 1) {
        pos_of.assign(n, 0);
        for (int32_t q = 0; q < n; ++q) pos_of[H.ulevel_rows[q]] = q;
    }
    auto pos = [&](int32_t r) { return dir == 0 ? r : pos_of[r]; };
    auto dbeg = [&](int32_t r) { return dir == 0 ? H.lu_rp[r] : H.diag[r] + 1; };
    auto dend = [&](int32_t r) { return dir == 0 ? H.diag[r] : H.lu_rp[r + 1]; };
    constexpr int W = kTailW, J = kTailJ;
    constexpr int kMaxEnt = 64 * J;

    // steps: (rows, per-row lane group) of one level; long rows alone, in chunks
    struct Item {
        int32_t r, g;      // row, log2 of its lane group
        int32_t b, e;      // its dependencies [b, e) within the row's entries (a chunk)
        int32_t flags;     // kTailCarryIn, kTailEmit
    };
    std::vector<std::vector<Item>> steps;
    std::vector<int32_t> step_level;   // the level each step belongs to
    std::vector<int32_t> step_of(n - T->pos0, -1);   // tail position -> its (emitting) step
    for (int32_t l = t; l < nl; ++l) {
        std::vector<Item> shortr;
        for (int32_t q = lp[l]; q < lp[l + 1]; ++q) {
            const int32_t r = row_at(q), len = dend(r) - dbeg(r);
            if (len > kMaxEnt) {
                for (int32_t c0 = 0; c0 < len; c0 += kMaxEnt) {
                    Item it{r, 6, c0, std::min(len, c0 + kMaxEnt), 0};
                    if (c0 > 0) it.flags |= kTailCarryIn;
                    if (c0 + kMaxEnt >= len) it.flags |= kTailEmit;
                    steps.push_back({it});
                    step_level.push_back(l);
                }
                step_of[q - T->pos0] = (int32_t)steps.size() - 1;
            } else {
                shortr.push_back({r, log2_ceil(std::max(1, (len + J - 1) / J)), 0, len, kTailEmit});
            }
        }
        std::stable_sort(shortr.begin(), shortr.end(), [](const Item &a, const Item &b) { return a.g > b.g; });
        std::vector<Item> cur;
        int lanes = 0;
        for (const Item &it : shortr) {
            if (lanes + (1 << it.g) > 64 || (int)cur.size() == kTailRows) {
                steps.push_back(cur);
                step_level.push_back(l);
                cur.clear();
                lanes = 0;
            }
            cur.push_back(it);
            lanes += 1 << it.g;
            step_of[pos(it.r) - T->pos0] = (int32_t)steps.size();
        }
        if (!cur.empty()) {
            steps.push_back(cur);
            step_level.push_back(l);
        }
    }
    T->nsteps = (int32_t)steps.size();
    // the positions of each step's level: steps follow the level order, so the
    // steps after the one that wrote a dependency (up to the step that reads it)
    // write positions between the start of the dependency's level and the end of
    // the reader's previous step's level; when that range is shorter than the
    // ring, no other position has taken the dependency's ring slot
    std::vector<int32_t> lstart(T->nsteps), lend(T->nsteps);
    for (int32_t s = 0; s < T->nsteps; ++s) {
        lstart[s] = lp[step_level[s]];
        lend[s] = lp[step_level[s] + 1];
    }
    T->hdr.reserve((size_t)T->nsteps * 4);
    for (int32_t s = 0; s < T->nsteps; ++s) {
        const std::vector<Item> &S = steps[s];
        const int32_t nrows = (int32_t)S.size();
        int32_t nlanes = 0, gmax = 0;
        for (const Item &it : S) {
            nlanes += 1 << it.g;
            gmax = std::max(gmax, it.g);
        }
        const int32_t nent = nlanes * J;
        const int32_t flags = S.size() == 1 ? S[0].flags : kTailEmit;
        while (T->rec.size() % 4) T->rec.push_back(0);   // rows are read as int4
        T->hdr.push_back((int32_t)T->rec.size());
        T->hdr.push_back(nrows | nlanes << 8 | gmax << 16 | flags << 24);
        T->hdr.push_back(nent);
        T->hdr.push_back(0);
        T->max_rows = std::max(T->max_rows, nrows);
        T->max_lanes = std::max(T->max_lanes, nlanes);
        for (const Item &it : S) {
            T->rec.push_back(it.r);
            T->rec.push_back(pos(it.r) & (W - 1));
            T->rec.push_back(H.perm[it.r]);
            T->rec.push_back(H.diag[it.r]);
        }
        // lanes: row index in the step, log2 of its group, group leader
        std::vector<int32_t> lane(nlanes, 0), start(nrows, 0);
        for (int32_t k = 0, l0 = 0; k < nrows; ++k) {
            start[k] = l0;
            for (int32_t i = 0; i < (1 << S[k].g); ++i) lane[l0 + i] = k | S[k].g << 8 | (i == 0 ? 1 << 16 : 0);
            l0 += 1 << S[k].g;
        }
        T->rec.insert(T->rec.end(), lane.begin(), lane.end());
        // entries, lane-major: entry (lane, j) at j * nlanes + lane
        std::vector<int32_t> ep(nent, -1), ec(nent, -1);
        for (int32_t k = 0; k < nrows; ++k) {
            const Item &it = S[k];
            const int32_t G = 1 << it.g, r = it.r;
            for (int32_t i = it.b; i < it.e; ++i) {
                const int32_t ii = i - it.b, p = dbeg(r) + i, c = H.lu_ci[p];
                const int32_t e = (ii / G) * nlanes + start[k] + ii % G;
                ep[e] = p;
                const int32_t pc = pos(c);
                int32_t code = W + c;   // read from the published buffer
                if (pc >= T->pos0) {
                    const int32_t sd = step_of[pc - T->pos0];
                    if (sd < s && lend[s - 1] - lstart[sd] <= W) code = pc & (W - 1);
                }
                ec[e] = code;
            }
        }
        T->rec.insert(T->rec.end(), ep.begin(), ep.end());
        T->rec.insert(T->rec.end(), ec.begin(), ec.end());
    }
    T->hdr.push_back((int32_t)T->rec.size());
    T->hdr.push_back(0);
    T->hdr.push_back(0);
    T->hdr.push_back(0);
}


// The factor's lower stage (Sec. III-B, Even-Rows and Fig. 7): the tail rows are
// factored in level order, a step at a time.  For its L entries e ascending a
// row divides entry e by the pivot of column c_e and every later entry whose
// column lies in U(c_e) subtracts multiplier * u -- the serial up-looking
// algorithm's operations in its order (Sec. III, Fig. 1), hence its bits; the
// entries with c_e before the tail (already final, ER's rows-in-parallel part)
// and the corner's (c_e in the tail) come in that same column order.
bool build_factor_tail(const HostAnalysis &H, const TailPlan &fwd, FactorTailPlan *T) {
    *T = FactorTailPlan();
    if (fwd.nsteps == 0 || fwd.level0 < 0) return false;
    const int32_t n = H.n, pos0 = fwd.pos0, t0 = fwd.level0;
    const int32_t nl = (int32_t)H.level_ptr.size() - 1;
    int32_t umax = 1;
    for (int32_t r = pos0; r < n; ++r) {
        const int32_t len = H.lu_rp[r + 1] - H.lu_rp[r], K = H.diag[r] - H.lu_rp[r];
        if (len > 64 || K > kFTailK) return false;
        umax = std::max(umax, H.lu_rp[r + 1] - H.diag[r]);
    }
    int32_t W = 1;
    while (2 * W * umax <= kFTailRing) W *= 2;
    // steps: rows of one level, groups of 2^g >= len lanes packed largest first
    struct Step {
        int32_t level;
        std::vector<std::pair<int32_t, int32_t>> rows;   // (row, g)
    };
    std::vector<Step> steps;
    std::vector<int32_t> step_of(n - pos0, -1);
    for (int32_t l = t0; l < nl; ++l) {
        std::vector<std::pair<int32_t, int32_t>> rs;
        for (int32_t r = H.level_ptr[l]; r < H.level_ptr[l + 1]; ++r) {
            const int32_t len = H.lu_rp[r + 1] - H.lu_rp[r];
            int32_t g = 0;
            while ((1 << g) < len) ++g;
            rs.push_back({r, g});
        }
        std::stable_sort(rs.begin(), rs.end(), [](const auto &a, const auto &b) { return a.second > b.second; });
        Step cur{l, {}};
        int32_t lanes = 0;
        for (const auto &rg : rs) {
            if (lanes + (1 << rg.second) > 64) {
                steps.push_back(cur);
                cur = Step{l, {}};
                lanes = 0;
            }
            cur.rows.push_back(rg);
            lanes += 1 << rg.second;
            step_of[rg.first - pos0] = (int32_t)steps.size();
        }
        if (!cur.rows.empty()) steps.push_back(cur);
    }
    const int32_t ns = (int32_t)steps.size();
    // Ring rule: c's slot is intact when read at step s if no row written from c's
    // step through s holds the same slot: the levels of those steps span at most W
    // rows (rows are numbered in level order).  Staging depth q: the largest <=
    // kFTailQ for which every source at most q steps old passes.
    auto span_ok = [&](int32_t sd, int32_t s) {
        return H.level_ptr[steps[s].level + 1] - H.level_ptr[steps[sd].level] <= W;
    };
    int32_t q = kFTailQ;
    for (int32_t s = 0; s < ns && q >= 2; ++s) {
        for (const auto &rg : steps[s].rows) {
            const int32_t r = rg.first;
            for (int32_t p = H.lu_rp[r]; p < H.diag[r]; ++p) {
                const int32_t c = H.lu_ci[p];
                if (c < pos0) continue;
                const int32_t sd = step_of[c - pos0];
                while (q >= 2 && s - sd < q && !span_ok(sd, s)) --q;
            }
        }
    }
    if (q < 2) return false;
    T->level0 = t0;
    T->pos0 = pos0;
    T->nsteps = ns;
    T->umax = umax;
    T->ring_rows = W;
    T->q = q;
    for (int32_t s = 0; s < ns; ++s) {
        const Step &S = steps[s];
        int32_t kmax = 0;
        for (const auto &rg : S.rows) kmax = std::max(kmax, H.diag[rg.first] - H.lu_rp[rg.first]);
        T->hdr.insert(T->hdr.end(), {(int32_t)(T->rows.size() / 8), (int32_t)S.rows.size(), kmax,
                                     (int32_t)T->lmap.size()});
        std::vector<uint8_t> lm(64, 255);
        int32_t lane0 = 0;
        for (int32_t k = 0; k < (int32_t)S.rows.size(); ++k) {
            const int32_t r = S.rows[k].first, g = S.rows[k].second;
            const int32_t len = H.lu_rp[r + 1] - H.lu_rp[r], K = H.diag[r] - H.lu_rp[r];
            for (int32_t t = 0; t < (1 << g); ++t) lm[lane0 + t] = (uint8_t)k;
            T->rows.insert(T->rows.end(), {r, H.lu_rp[r], len | K << 8 | g << 16 | lane0 << 24,
                                           (r & (W - 1)) * umax, (int32_t)T->lsrc.size(), (int32_t)T->match.size(),
                                           0, 0});
            for (int32_t e = 0; e < K; ++e) {
                const int32_t c = H.lu_ci[H.lu_rp[r] + e];
                bool ring = false;
                if (c >= pos0) {
                    const int32_t sd = step_of[c - pos0];
                    ring = s - sd < q || span_ok(sd, s);
                }
                T->lsrc.push_back(ring ? (c & (W - 1)) * umax : -(H.diag[c] + 1));
                // positions in U(c) of the row's entries t > e (both rows sorted)
                const int32_t *ub = H.lu_ci.data() + H.diag[c], *ue = H.lu_ci.data() + H.lu_rp[c + 1];
                for (int32_t t = 0; t < len; ++t) {
                    uint8_t j = 255;
                    if (t == e) {
                        j = 0;
                    } else if (t > e) {
                        const int32_t col = H.lu_ci[H.lu_rp[r] + t];
                        const int32_t *f = std::lower_bound(ub, ue, col);
                        if (f != ue && *f == col) j = (uint8_t)(f - ub);
                    }
                    T->match.push_back(j);
                }
            }
            lane0 += 1 << g;
        }
        T->lmap.insert(T->lmap.end(), lm.begin(), lm.end());
    }
    T->hdr.insert(T->hdr.end(), {(int32_t)(T->rows.size() / 8), 0, 0, (int32_t)T->lmap.size()});
    return true;
}

}  // namespace jv
