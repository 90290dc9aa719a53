// Host analysis: CSR intake, ILU(k) fill pattern, level sets, level-order
// permutation, permuted factor structure, solve schedules.
//
// Level sets follow the paper's definition directly (Sec. II): rows with no
// incoming dependency form a level, they are removed, and the step repeats.  The
// peeling is a Kahn-style frontier sweep over the dependency graph of lower(S)
// or lower(S + S^T) (Sec. III); rows of a level keep their input order, so the
// permutation is the stable sort by level.
#include "analysis.h"
#include "par.h"

#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>

namespace jv {

namespace {

// Peels a DAG given as successor lists.  indeg counts incoming edges with
// multiplicity.  Returns the number of levels; `order` lists rows level by level,
// ascending inside a level; `ptr` delimits the levels.  Returns -1 on a cycle.
int32_t peel(int32_t n, const std::vector<int64_t> &sp, const std::vector<int32_t> &succ,
             std::vector<int32_t> indeg, std::vector<int32_t> &order, std::vector<int32_t> &ptr,
             std::vector<int32_t> *level_of) {
    order.clear();
    order.reserve(n);
    ptr.assign(1, 0);
    std::vector<int32_t> frontier, next;
    for (int32_t i = 0; i < n; ++i)
        if (indeg[i] == 0) frontier.push_back(i);
    int32_t nlev = 0;
    while (!frontier.empty()) {
        std::sort(frontier.begin(), frontier.end());
        for (int32_t i : frontier) {
            order.push_back(i);
            if (level_of) (*level_of)[i] = nlev;
        }
        ptr.push_back((int32_t)order.size());
        next.clear();
        for (int32_t i : frontier)
            for (int64_t e = sp[i]; e < sp[i + 1]; ++e)
                if (--indeg[succ[e]] == 0) next.push_back(succ[e]);
        frontier.swap(next);
        ++nlev;
    }
    if ((int32_t)order.size() != n) return -1;
    return nlev;
}

// Successor lists of the triangular dependencies of a CSR pattern: with
// lower == true, row i depends on every column j < i of its row (edge j -> i);
// otherwise on every column j > i (edge j -> i, solved from the bottom).
void triangular_deps(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, bool lower,
                     std::vector<int64_t> &sp, std::vector<int32_t> &succ, std::vector<int32_t> &indeg) {
    sp.assign((size_t)n + 1, 0);
    indeg.assign(n, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t j = ci[p];
            if (lower ? (j < i) : (j > i)) {
                sp[j + 1]++;
                indeg[i]++;
            }
        }
    for (int32_t i = 0; i < n; ++i) sp[i + 1] += sp[i];
    succ.assign((size_t)sp[n], 0);
    std::vector<int64_t> fill(sp.begin(), sp.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t j = ci[p];
            if (lower ? (j < i) : (j > i)) succ[fill[j]++] = i;
        }
}

}  // namespace

// Arguments and CSR intake: monotone row pointers, sorted unique in-range columns.
static ilu_status check_input(int32_t n, const int32_t *rp, const int32_t *ci, int64_t nnz, int32_t k_max,
                              int32_t pattern, std::string *err) {
    if (n <= 0 || !rp || !ci) { *err = "analyze: n <= 0 or NULL array"; return ILU_ERR_ARG; }
    if (k_max < 0 || k_max > 100) { *err = "analyze: k_max must be in [0, 100]"; return ILU_ERR_ARG; }
    if (pattern != ILU_PATTERN_LOWER_SYM && pattern != ILU_PATTERN_LOWER_A) {
        *err = "analyze: unknown dependency pattern";
        return ILU_ERR_ARG;
    }
    if (nnz < 0 || nnz >= ((int64_t)1 << 31) - (int64_t)n) {
        *err = "analyze: nnz must be below 2^31";
        return ILU_ERR_UNSUPPORTED;
    }
    // ---- intake: monotone row pointers, sorted unique in-range columns ----
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) { *err = "analyze: row_ptr[0] != 0 or row_ptr[n] != nnz"; return ILU_ERR_CSR; }
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) { *err = "analyze: row_ptr decreases at row " + std::to_string(i); return ILU_ERR_CSR; }
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) { *err = "analyze: column out of range in row " + std::to_string(i); return ILU_ERR_CSR; }
            if (p > rp[i] && ci[p] <= ci[p - 1]) { *err = "analyze: columns unsorted or duplicated in row " + std::to_string(i); return ILU_ERR_CSR; }
        }
    }
    return ILU_OK;
}

static void transpose_and_schedules(HostAnalysis &H);

static ilu_status analyze_natural(int32_t n, const int32_t *rp, const int32_t *ci, int64_t nnz, int32_t k_max,
                                  int32_t pattern, HostAnalysis *out, std::string *err) {
    if (!out) { *err = "analyze: NULL output"; return ILU_ERR_ARG; }
    ilu_status st0 = check_input(n, rp, ci, nnz, k_max, pattern, err);
    if (st0 != ILU_OK) return st0;
    HostAnalysis &H = *out;
    H = HostAnalysis();
    H.n = n;
    H.nnz_in = nnz;
    H.k_max = k_max;
    H.pattern = pattern;
    H.in_rp.assign(rp, rp + n + 1);

    // ---- canonical pattern: the diagonal is always stored (no pivoting, Sec. III) ----
    std::vector<int32_t> crp((size_t)n + 1), cci, csrc;
    cci.reserve((size_t)nnz + n);
    csrc.reserve((size_t)nnz + n);
    crp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        bool placed = std::binary_search(ci + rp[i], ci + rp[i + 1], i);
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (!placed && ci[p] > i) { cci.push_back(i); csrc.push_back(-1); placed = true; }
            cci.push_back(ci[p]);
            csrc.push_back(p);
        }
        if (!placed) { cci.push_back(i); csrc.push_back(-1); }
        crp[i + 1] = (int32_t)cci.size();
    }

    // ---- fill pattern S by level of fill, in the input ordering (Sec. III) ----
    // Row i starts from A's row at level 0.  Earlier columns k are taken in
    // ascending order from a min-heap; each contributes level(i,k) + level(k,j) + 1
    // to every later column j of row k, admitted when it does not exceed k_max.
    std::vector<int32_t> srp((size_t)n + 1), sci, ssrc;
    std::vector<int8_t> slev;
    if (k_max == 0) {
        srp = crp;
        sci = cci;
        ssrc = csrc;
        slev.assign(sci.size(), 0);
    } else {
        sci.reserve(cci.size() * 2);
        ssrc.reserve(cci.size() * 2);
        slev.reserve(cci.size() * 2);
        std::vector<int32_t> lvl(n), stamp(n, -1), srcj(n), touched;
        std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> heap;
        srp[0] = 0;
        for (int32_t i = 0; i < n; ++i) {
            touched.clear();
            for (int32_t p = crp[i]; p < crp[i + 1]; ++p) {
                int32_t j = cci[p];
                stamp[j] = i;
                lvl[j] = 0;
                srcj[j] = csrc[p];
                touched.push_back(j);
                if (j < i) heap.push(j);
            }
            while (!heap.empty()) {
                int32_t k = heap.top();
                heap.pop();
                int32_t lk = lvl[k];
                for (int32_t q = srp[k]; q < srp[k + 1]; ++q) {
                    int32_t j = sci[q];
                    if (j <= k) continue;
                    int32_t nl = lk + slev[q] + 1;
                    if (nl > k_max) continue;
                    if (stamp[j] != i) {
                        stamp[j] = i;
                        lvl[j] = nl;
                        srcj[j] = -1;
                        touched.push_back(j);
                        if (j < i) heap.push(j);
                    } else if (nl < lvl[j]) {
                        lvl[j] = nl;
                    }
                }
            }
            std::sort(touched.begin(), touched.end());
            for (int32_t j : touched) {
                sci.push_back(j);
                slev.push_back((int8_t)lvl[j]);
                ssrc.push_back(srcj[j]);
            }
            if (sci.size() >= ((size_t)1 << 31)) { *err = "analyze: fill pattern exceeds 2^31 entries"; return ILU_ERR_UNSUPPORTED; }
            srp[i + 1] = (int32_t)sci.size();
        }
    }

    // ---- level sets by peeling (Sec. II): dependencies of lower(S) or lower(S+S^T) ----
    {
        std::vector<int64_t> sp((size_t)n + 1, 0);
        std::vector<int32_t> indeg(n, 0);
        const bool sym = pattern == ILU_PATTERN_LOWER_SYM;
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = srp[i]; p < srp[i + 1]; ++p) {
                int32_t j = sci[p];
                if (j < i) { sp[j + 1]++; indeg[i]++; }
                else if (j > i && sym) { sp[i + 1]++; indeg[j]++; }
            }
        for (int32_t i = 0; i < n; ++i) sp[i + 1] += sp[i];
        std::vector<int32_t> succ((size_t)sp[n]);
        std::vector<int64_t> fill(sp.begin(), sp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = srp[i]; p < srp[i + 1]; ++p) {
                int32_t j = sci[p];
                if (j < i) succ[fill[j]++] = i;
                else if (j > i && sym) succ[fill[i]++] = j;
            }
        H.n_levels = peel(n, sp, succ, indeg, H.perm, H.level_ptr, nullptr);
        if (H.n_levels < 0) { *err = "analyze: dependency cycle (internal error)"; return ILU_ERR_ARG; }
    }
    H.iperm.assign(n, 0);
    for (int32_t r = 0; r < n; ++r) H.iperm[H.perm[r]] = r;

    // ---- permuted structures: rows in level order, columns renamed and sorted ----
    auto permute_rows = [&](const std::vector<int32_t> &xrp, const std::vector<int32_t> &xci,
                            const std::vector<int32_t> &xsrc, const std::vector<int8_t> *xlev,
                            std::vector<int32_t> &orp, std::vector<int32_t> &oci, std::vector<int32_t> &osrc,
                            std::vector<int8_t> *olev, std::vector<int32_t> *odiag, int32_t &maxrow) {
        orp.assign((size_t)n + 1, 0);
        for (int32_t r = 0; r < n; ++r) {
            int32_t i = H.perm[r];
            orp[r + 1] = orp[r] + (xrp[i + 1] - xrp[i]);
        }
        oci.resize(orp[n]);
        osrc.resize(orp[n]);
        if (olev) olev->resize(orp[n]);
        if (odiag) odiag->assign(n, -1);
        // rows write disjoint ranges: chunks of rows run on their own threads
        std::vector<int32_t> cmax(host_threads(), 0);
        parallel_chunks(n, 1 << 14, [&](int c, int64_t lo, int64_t hi) {
            std::vector<std::pair<int32_t, int32_t>> tmp;
            int32_t m = 0;
            for (int32_t r = (int32_t)lo; r < (int32_t)hi; ++r) {
                int32_t i = H.perm[r];
                tmp.clear();
                for (int32_t p = xrp[i]; p < xrp[i + 1]; ++p) tmp.emplace_back(H.iperm[xci[p]], p);
                std::sort(tmp.begin(), tmp.end());
                int32_t o = orp[r];
                m = std::max(m, (int32_t)tmp.size());
                for (size_t t = 0; t < tmp.size(); ++t) {
                    oci[o + t] = tmp[t].first;
                    osrc[o + t] = xsrc[tmp[t].second];
                    if (olev) (*olev)[o + t] = (*xlev)[tmp[t].second];
                    if (odiag && tmp[t].first == r) (*odiag)[r] = o + (int32_t)t;
                }
            }
            cmax[c] = m;
        });
        maxrow = *std::max_element(cmax.begin(), cmax.end());
    };
    permute_rows(srp, sci, ssrc, &slev, H.lu_rp, H.lu_ci, H.lu_src, &H.flev, &H.diag, H.max_row_lu);
    for (int32_t r = 0; r < n; ++r) {
        H.max_lower_lu = std::max(H.max_lower_lu, H.diag[r] - H.lu_rp[r]);
        H.max_upper_lu = std::max(H.max_upper_lu, H.lu_rp[r + 1] - H.diag[r] - 1);
    }
    permute_rows(crp, cci, csrc, nullptr, H.b_rp, H.b_ci, H.b_src, nullptr, nullptr, H.max_row_b);

    // The check of the level schedule with the backward schedule, and the
    // transposed structure with its two schedules, read only the factor
    // structure and write disjoint fields: the two groups run side by side.
    bool level_ok = true;
    run_pair(
        [&] {
            // every strictly lower factor entry must point to an earlier level (the
            // schedule is valid); checked once here because the kernels rely on it
            std::vector<int32_t> lvl_of(n);
            for (int32_t l = 0; l < H.n_levels; ++l)
                for (int32_t r = H.level_ptr[l]; r < H.level_ptr[l + 1]; ++r) lvl_of[r] = l;
            for (int32_t r = 0; r < n && level_ok; ++r)
                for (int32_t p = H.lu_rp[r]; p < H.diag[r]; ++p)
                    if (lvl_of[H.lu_ci[p]] >= lvl_of[r]) { level_ok = false; break; }
            // ---- backward schedule: peel the upper dependencies from the last rows ----
            std::vector<int64_t> sp;
            std::vector<int32_t> succ, indeg;
            triangular_deps(n, H.lu_rp, H.lu_ci, false, sp, succ, indeg);
            H.n_ulevels = peel(n, sp, succ, indeg, H.ulevel_rows, H.ulevel_ptr, nullptr);
        },
        [&] { transpose_and_schedules(H); });
    if (!level_ok) { *err = "analyze: invalid level schedule (internal error)"; return ILU_ERR_ARG; }
    if (H.n_ulevels < 0) { *err = "analyze: upper schedule cycle (internal error)"; return ILU_ERR_ARG; }
    if (H.n_tlevels < 0 || H.n_tulevels < 0) { *err = "analyze: transposed schedule cycle (internal error)"; return ILU_ERR_ARG; }
    return ILU_OK;
}

// ---- transposed factor structure and its schedules (adjoint) ----
static void transpose_and_schedules(HostAnalysis &H) {
    const int32_t n = H.n;
    {
        const int64_t nz = H.lu_rp[n];
        H.t_rp.assign((size_t)n + 1, 0);
        for (int64_t p = 0; p < nz; ++p) H.t_rp[H.lu_ci[p] + 1]++;
        for (int32_t j = 0; j < n; ++j) H.t_rp[j + 1] += H.t_rp[j];
        H.t_ci.resize(nz);
        H.t_map.resize(nz);
        H.t_diag.assign(n, -1);
        std::vector<int32_t> fill(H.t_rp.begin(), H.t_rp.end() - 1);
        for (int32_t i = 0; i < n; ++i)          // rows ascending: columns of (LU)^T come out sorted
            for (int32_t p = H.lu_rp[i]; p < H.lu_rp[i + 1]; ++p) {
                int32_t j = H.lu_ci[p];
                int32_t o = fill[j]++;
                H.t_ci[o] = i;
                H.t_map[o] = p;
                if (i == j) H.t_diag[j] = o;
            }
        run_pair(
            [&] {
                std::vector<int64_t> sp;
                std::vector<int32_t> succ, indeg;
                triangular_deps(n, H.t_rp, H.t_ci, true, sp, succ, indeg);
                H.n_tlevels = peel(n, sp, succ, indeg, H.tlevel_rows, H.tlevel_ptr, nullptr);
            },
            [&] {
                std::vector<int64_t> sp;
                std::vector<int32_t> succ, indeg;
                triangular_deps(n, H.t_rp, H.t_ci, false, sp, succ, indeg);
                H.n_tulevels = peel(n, sp, succ, indeg, H.tulevel_rows, H.tulevel_ptr, nullptr);
            });
    }
}


// Reverse Cuthill-McKee order of the graph of A + A^T (diagonal ignored), the
// preordering that Sec. VII sets against nested dissection.  Components in order
// of their smallest vertex; each starts from a pseudo-peripheral vertex found by
// the George-Liu search seeded with the component's vertex of least (degree,
// index); the Cuthill-McKee sweep queues each vertex's unvisited neighbours by
// (degree, index); the concatenated sweep is reversed.  order[i] = input vertex
// that becomes vertex i.
std::vector<int32_t> rcm_order(int32_t n, const int32_t *rp, const int32_t *ci) {
    // symmetric adjacency: each vertex's neighbours in both directions, sorted and
    // de-duplicated per vertex (vertices in chunks on threads)
    std::vector<int64_t> bp((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) {
                bp[i + 1]++;
                bp[ci[p] + 1]++;
            }
    for (int32_t i = 0; i < n; ++i) bp[i + 1] += bp[i];
    std::vector<int32_t> buf((size_t)bp[n]);
    {
        std::vector<int64_t> cur(bp.begin(), bp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
                if (ci[p] != i) {
                    buf[cur[i]++] = ci[p];
                    buf[cur[ci[p]]++] = i;
                }
    }
    std::vector<int32_t> len(n);
    parallel_chunks(n, 1 << 14, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            int32_t *b = buf.data() + bp[i], *e = buf.data() + bp[i + 1];
            std::sort(b, e);
            len[i] = (int32_t)(std::unique(b, e) - b);
        }
    });
    std::vector<int32_t> gp((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) gp[i + 1] = gp[i] + len[i];
    std::vector<int32_t> gj((size_t)gp[n]);
    parallel_chunks(n, 1 << 14, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) std::copy(buf.data() + bp[i], buf.data() + bp[i] + len[i], gj.data() + gp[i]);
    });
    std::vector<int32_t>().swap(buf);
    auto deg = [&](int32_t v) { return gp[v + 1] - gp[v]; };
    auto before = [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; };

    // breadth-first level structure: returns its depth; `bfs` holds the reached
    // vertices in visit order and `last` the start of the deepest level
    std::vector<int32_t> seen(n, -1), bfs;
    bfs.reserve(n);
    int32_t epoch = 0;
    auto levels = [&](int32_t root, size_t &last) {
        ++epoch;
        bfs.clear();
        bfs.push_back(root);
        seen[root] = epoch;
        size_t level_begin = 0, level_end = 1;
        int32_t depth = 0;
        while (true) {
            for (size_t k = level_begin; k < level_end; ++k)
                for (int32_t e = gp[bfs[k]]; e < gp[bfs[k] + 1]; ++e)
                    if (seen[gj[e]] != epoch) {
                        seen[gj[e]] = epoch;
                        bfs.push_back(gj[e]);
                    }
            if (bfs.size() == level_end) break;
            level_begin = level_end;
            level_end = bfs.size();
            ++depth;
        }
        last = level_begin;
        return depth;
    };

    std::vector<char> placed(n, 0);
    std::vector<int32_t> sweep;
    sweep.reserve(n);
    std::vector<int32_t> kids;
    for (int32_t v = 0; v < n; ++v) {
        if (placed[v]) continue;
        size_t last = 0;
        levels(v, last);
        int32_t start = *std::min_element(bfs.begin(), bfs.end(), before);
        int32_t depth = levels(start, last);
        while (true) {
            const int32_t x = *std::min_element(bfs.begin() + (std::ptrdiff_t)last, bfs.end(), before);
            size_t xlast = 0;
            const int32_t dx = levels(x, xlast);
            if (dx <= depth) break;
            start = x;
            depth = dx;
            last = xlast;
        }
        size_t head = sweep.size();
        sweep.push_back(start);
        placed[start] = 1;
        while (head < sweep.size()) {
            const int32_t u = sweep[head++];
            kids.clear();
            for (int32_t e = gp[u]; e < gp[u + 1]; ++e)
                if (!placed[gj[e]]) {
                    placed[gj[e]] = 1;
                    kids.push_back(gj[e]);
                }
            std::sort(kids.begin(), kids.end(), before);
            sweep.insert(sweep.end(), kids.begin(), kids.end());
        }
    }
    std::reverse(sweep.begin(), sweep.end());
    return sweep;
}

ilu_status analyze_host(int32_t n, const int32_t *rp, const int32_t *ci, int64_t nnz, int32_t k_max,
                        int32_t pattern, int32_t ordering, HostAnalysis *out, std::string *err) {
    if (ordering == ILU_ORDER_NATURAL) return analyze_natural(n, rp, ci, nnz, k_max, pattern, out, err);
    if (ordering != ILU_ORDER_RCM) {
        *err = "analyze: unknown ordering";
        return ILU_ERR_ARG;
    }
    // validate A as given, then analyse Q A Q^T and compose the maps back
    ilu_status st = check_input(n, rp, ci, nnz, k_max, pattern, err);
    if (st != ILU_OK) return st;
    if (!out) { *err = "analyze: NULL output"; return ILU_ERR_ARG; }
    const std::vector<int32_t> q = rcm_order(n, rp, ci);
    std::vector<int32_t> iq(n);
    for (int32_t i = 0; i < n; ++i) iq[q[i]] = i;
    std::vector<int32_t> qrp((size_t)n + 1, 0), qci((size_t)nnz), qsrc((size_t)nnz);
    for (int32_t i = 0; i < n; ++i) qrp[i + 1] = qrp[i] + (rp[q[i] + 1] - rp[q[i]]);
    parallel_chunks(n, 1 << 14, [&](int, int64_t lo, int64_t hi) {
        std::vector<std::pair<int32_t, int32_t>> row;
        for (int32_t i = (int32_t)lo; i < (int32_t)hi; ++i) {
            const int32_t o = q[i];
            row.clear();
            for (int32_t p = rp[o]; p < rp[o + 1]; ++p) row.emplace_back(iq[ci[p]], p);
            std::sort(row.begin(), row.end());
            for (size_t k = 0; k < row.size(); ++k) {
                qci[qrp[i] + k] = row[k].first;
                qsrc[qrp[i] + k] = row[k].second;
            }
        }
    });
    st = analyze_natural(n, qrp.data(), qci.data(), nnz, k_max, pattern, out, err);
    if (st != ILU_OK) return st;
    HostAnalysis &H = *out;
    for (auto &s : H.lu_src)
        if (s >= 0) s = qsrc[s];
    for (auto &s : H.b_src)
        if (s >= 0) s = qsrc[s];
    for (int32_t r = 0; r < n; ++r) H.perm[r] = q[H.perm[r]];
    for (int32_t r = 0; r < n; ++r) H.iperm[H.perm[r]] = r;
    H.in_rp.assign(rp, rp + n + 1);   // tau row norms: input rows, input entry order
    H.order = q;
    return ILU_OK;
}

}  // namespace jv
