// Autotuner: times the launch schemes of the factor and of the FP64 apply on the
// handle's own matrix and keeps the fastest.  The candidates are one launch per
// level and one persistent sync-free launch (each with 1x and 2x the lanes per
// row the longest row needs), and the tiled launch at tile sizes of 128, 256,
// 512 and 1024 rows (and the handle's own size).  The tile size is this design's
// level-merge threshold: a tile merges consecutive levels of up to that many rows
// into one workgroup whose dependencies go through LDS.  The apply also tries the
// lower stage (narrow levels at the end of each direction streamed by one
// workgroup, levels of fewer than 64 rows or the handle's own threshold).  The
// apply -- called many times per factor -- picks the tiling; the tiled factor then
// has its own tile size timed (its default, by update work per row, and 64 to 1024
// rows) before its scheme is picked.  Every
// schedule computes the same bits (the factor reproduces the serial up-looking
// order on all of them), so re-running the caller's factor -- same k, tau and
// flags -- leaves the handle with the factor it had.  The spmv's lanes per row
// are timed too, and with long rows its nnz-balanced pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "device.h"
#include "handle.h"
#include "javelin.h"

using namespace jv;

namespace {

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" ilu_status ilu_tune(ilu_handle h, const double *a_val, int32_t reps, double *results, int32_t cap,
                               int32_t *n_results, hipStream_t s) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_tune: NULL handle");
    if (h->host_only) return fail(ILU_ERR_STATE, "ilu_tune: host-only analysis");
    if (!h->factored) return fail(ILU_ERR_STATE, "ilu_tune: requires a factor");
    if (reps < 1) reps = 3;
    const HostAnalysis &H = h->H;
    const int32_t save_fs = h->sched_factor, save_ss = h->sched_solve;
    const int32_t save_lf = h->lanes_factor, save_ls = h->lanes_solve;
    const int32_t save_tr = h->tile_rows;
    const int32_t save_fr = h->factor_rows;
    // the caller's factor: same k, tau and flags (casts, modified form)
    const int32_t k = h->k_used;
    const double tau = h->tau_used;
    const int32_t fflags = h->flags_used;
    std::vector<double> rows;
    Timer T;
    auto time_it = [&](auto &&fn, double *us) -> ilu_status {
        ilu_status st = fn();   // warm-up (also builds task lists)
        if (st != ILU_OK) return st;
        hipError_t e0 = hipEventRecord(T.a, s);
        for (int r = 0; r < reps; ++r)
            if ((st = fn()) != ILU_OK) return st;
        if (e0 == hipSuccess) e0 = hipEventRecord(T.b, s);
        if (e0 == hipSuccess) e0 = hipEventSynchronize(T.b);
        float ms = 0.f;
        if (e0 == hipSuccess) e0 = hipEventElapsedTime(&ms, T.a, T.b);
        if (e0 != hipSuccess) return hip_fail(e0, "ilu_tune: timing");
        *us = 1e3 * ms / reps;
        return ILU_OK;
    };
    const int32_t save_tail = h->tail_min_rows;
    auto restore = [&](ilu_status st) {
        if (h->tail_min_rows != save_tail) (void)h->make_tail(save_tail);
        h->sched_factor = save_fs;
        h->sched_solve = save_ss;
        h->lanes_factor = save_lf;
        h->lanes_solve = save_ls;
        if (h->factor_rows != save_fr) {
            h->factor_rows = save_fr;
            if (h->tile_rows == save_tr) (void)h->make_factor_tiles();
        }
        if (h->tile_rows != save_tr) (void)h->make_tiles(save_tr, false);
        return st;
    };
    auto factor = [&]() { return ilu_factor(h, a_val, k, tau, fflags, nullptr, s); };
    DevBuf buf;
    hipError_t e = hipMalloc(&buf.p, (size_t)H.n * 16);
    if (e != hipSuccess) return hip_fail(e, "ilu_tune: buffers");
    double *b = (double *)buf.p, *x = b + H.n;
    if ((e = launch_fill_u64((uint64_t *)b, 0x3FF0000000000000ull, H.n, s)) != hipSuccess)   // b = 1
        return hip_fail(e, "ilu_tune: fill");
    auto apply = [&]() { return ilu_apply(h, b, x, 1, 1, ILU_PREC_F64, ILU_PREC_F64, ILU_PERMUTED_SPACE, s); };

    // ---- tiled: tile sizes (the level-merge threshold), apply and factor ----
    // (without a lower stage; it is a candidate of its own below)
    const int32_t tail_in = h->tail_min_rows;
    if (tail_in != 0) {
        ilu_status st = h->make_tail(0);
        if (st != ILU_OK) return restore(st);
    }
    std::vector<int32_t> sizes = {128, 256, 512, 1024};
    if (std::find(sizes.begin(), sizes.end(), save_tr) == sizes.end()) sizes.push_back(save_tr);
    struct TileRes {
        int32_t rows;
        double apply_us, factor_us;
    };
    std::vector<TileRes> tres;
    for (int32_t tr : sizes) {
        if (tr > std::max<int32_t>(H.n, 16) && tr != save_tr) continue;
        ilu_status st = h->make_tiles(tr, false);
        if (st != ILU_OK) return restore(st);
        TileRes r{tr, -1.0, -1.0};
        h->sched_solve = ILU_SCHED_TILED;
        st = time_it(apply, &r.apply_us);
        if (st == ILU_ERR_UNSUPPORTED) r.apply_us = -1.0;   // tiles beyond LDS
        else if (st != ILU_OK) return restore(st);
        if (a_val && h->ftiles_ok && k == H.k_max) {
            h->sched_factor = ILU_SCHED_TILED;
            st = time_it(factor, &r.factor_us);
            if (st != ILU_OK) return restore(st);
        }
        if (r.apply_us >= 0) rows.insert(rows.end(), {1.0, (double)ILU_SCHED_TILED, (double)tr, r.apply_us});
        if (r.factor_us >= 0) rows.insert(rows.end(), {0.0, (double)ILU_SCHED_TILED, (double)tr, r.factor_us});
        tres.push_back(r);
    }
    h->sched_factor = save_fs;
    // ---- level and sync-free applies, lanes per row (without a lower stage) ----
    double best_apply = 1e300;
    int best_ss = save_ss, best_ls = save_ls;
    int32_t best_tr = save_tr;
    for (const TileRes &r : tres)
        if (r.apply_us >= 0 && r.apply_us < best_apply) {
            best_apply = r.apply_us;
            best_ss = ILU_SCHED_TILED;
            best_tr = r.rows;
        }
    for (int sched = ILU_SCHED_LEVEL; sched <= ILU_SCHED_SYNCFREE; ++sched)
        for (int lanes = 4; lanes <= 64; lanes *= 2) {
            h->sched_solve = sched;
            h->lanes_solve = lanes;
            double us = 0;
            ilu_status st = time_it(apply, &us);
            if (st != ILU_OK) return restore(st);
            rows.insert(rows.end(), {1.0, (double)sched, (double)lanes, us});
            if (us < best_apply) {
                best_apply = us;
                best_ss = sched;
                best_ls = lanes;
            }
        }
    h->sched_solve = best_ss;
    h->lanes_solve = best_ss == ILU_SCHED_TILED ? save_ls : best_ls;
    // the lower stage: narrow levels at the end of each direction streamed by one
    // workgroup (levels of fewer than 64 rows), next to the best schedule so far
    int32_t best_tail = 0;
    for (int32_t m : {tail_in > 0 ? tail_in : 64}) {
        ilu_status st = h->make_tail(m);
        if (st != ILU_OK) return restore(st);
        if (m > 0 && h->tail[0].nsteps == 0 && h->tail[1].nsteps == 0) continue;
        double us = 0;
        if ((st = time_it(apply, &us)) != ILU_OK) return restore(st);
        rows.insert(rows.end(), {1.0, 10.0, (double)m, us});
        if (us < best_apply) {
            best_apply = us;
            best_tail = m;
        }
    }
    if (h->tail_min_rows != best_tail) {
        ilu_status st = h->make_tail(best_tail);
        if (st != ILU_OK) return restore(st);
    }
    // the tiling of the chosen apply (or, when the apply is not tiled, the one the
    // tiled factor liked best)
    if (best_ss != ILU_SCHED_TILED) {
        double bf = 1e300;
        for (const TileRes &r : tres)
            if (r.factor_us >= 0 && r.factor_us < bf) {
                bf = r.factor_us;
                best_tr = r.rows;
            }
    }
    if (h->tile_rows != best_tr) {
        ilu_status st = h->make_tiles(best_tr, false);
        if (st != ILU_OK) return restore(st);
    }
    // ---- factor: tiled on the chosen tiling (its own tile size searched) vs
    // sync-free and level launches ----
    if (a_val) {
        double best = 1e300;
        int best_fs = save_fs, best_lf = save_lf;
        for (const TileRes &r : tres)
            if (r.rows == best_tr && r.factor_us >= 0) {
                best = r.factor_us;
                best_fs = ILU_SCHED_TILED;
            }
        if (best_fs == ILU_SCHED_TILED) {
            // the tiled factor's tile size: the default (by update work per row) and
            // 64 .. 1024 rows, each size timed once
            int32_t best_fr = h->factor_rows;
            std::vector<int32_t> seen;
            for (int32_t fr : {0, 64, 128, 256, 512, 1024}) {
                if (fr > std::max<int32_t>(H.n, 16)) continue;
                h->factor_rows = fr;
                ilu_status st = h->make_factor_tiles();
                if (st != ILU_OK) return restore(st);
                if (!h->ftiles_ok) continue;
                const int32_t used = h->ftset_own ? h->ftset.cap : h->tile_rows;
                if (std::find(seen.begin(), seen.end(), used) != seen.end()) continue;
                seen.push_back(used);
                h->sched_factor = ILU_SCHED_TILED;
                double us = 0;
                if ((st = time_it(factor, &us)) != ILU_OK) return restore(st);
                rows.insert(rows.end(), {0.0, 11.0, (double)used, us});
                if (us < best) {
                    best = us;
                    best_fr = fr;
                }
            }
            h->factor_rows = best_fr;
            ilu_status st = h->make_factor_tiles();
            if (st != ILU_OK) return restore(st);
        }
        const int lmin = std::max(4, std::min(save_lf, 64));
        for (int sched = ILU_SCHED_LEVEL; sched <= ILU_SCHED_SYNCFREE; ++sched)
            for (int lanes = lmin; lanes <= 64 && lanes <= 2 * lmin; lanes *= 2) {
                h->sched_factor = sched;
                h->lanes_factor = lanes;
                double us = 0;
                ilu_status st = time_it(factor, &us);
                if (st != ILU_OK) return restore(st);
                rows.insert(rows.end(), {0.0, (double)sched, (double)lanes, us});
                if (us < best) {
                    best = us;
                    best_fs = sched;
                    best_lf = lanes;
                }
            }
        h->sched_factor = best_fs;
        h->lanes_factor = best_fs == ILU_SCHED_TILED ? save_lf : best_lf;
        // the factor's lower stage, when the chosen tail has a plan for it
        const bool save_fl = h->factor_lower;
        h->factor_lower = false;
        if (h->ftail_ok && h->tail_min_rows > 0 && k == H.k_max && tau == 0.0 && !(fflags & ILU_FACTOR_MODIFIED)) {
            h->factor_lower = true;
            double us = 0;
            ilu_status st = time_it(factor, &us);
            if (st != ILU_OK) {
                h->factor_lower = save_fl;
                return restore(st);
            }
            rows.insert(rows.end(), {0.0, 10.0, (double)h->tail_min_rows, us});
            h->factor_lower = us < best;
        }
        // leave the caller's factor computed on the chosen schedule
        ilu_status st = factor();
        if (st != ILU_OK) return restore(st);
    }
    // ---- spmv: lanes per row of the row pass, then the nnz-balanced pass when built ----
    if (h->bvals) {
        auto spmv = [&]() { return ilu_spmv(h, 1.0, b, 0.0, x, 1, 1, ILU_PERMUTED_SPACE, s); };
        const bool save_nz = h->spmv_nz;
        const int32_t save_lsp = h->lanes_spmv;
        h->spmv_nz = false;
        double best = 1e300;
        int32_t best_l = save_lsp;
        for (int32_t lanes : {1, 4, 8, 16, 32, 64}) {
            h->lanes_spmv = lanes;
            double us = 0;
            ilu_status st = time_it(spmv, &us);
            if (st != ILU_OK) {
                h->spmv_nz = save_nz;
                h->lanes_spmv = save_lsp;
                return restore(st);
            }
            rows.insert(rows.end(), {2.0, 20.0, (double)lanes, us});
            if (us < best) {
                best = us;
                best_l = lanes;
            }
        }
        h->lanes_spmv = best_l;
        bool best_nz = false;
        if (h->nz_waves > 0) {
            h->spmv_nz = true;
            double us = 0;
            ilu_status st = time_it(spmv, &us);
            if (st != ILU_OK) {
                h->spmv_nz = save_nz;
                return restore(st);
            }
            rows.insert(rows.end(), {2.0, 21.0, 0.0, us});
            best_nz = us < best;
        }
        h->spmv_nz = best_nz;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ilu_tune: synchronize");
    const int nr = (int)(rows.size() / 4);
    if (n_results) *n_results = nr;
    if (results && cap > 0) std::memcpy(results, rows.data(), sizeof(double) * 4 * std::min(cap, nr));
    return ILU_OK;
}
