// Autotuner: times the launch schemes (one launch per level vs one persistent
// sync-free launch, and for the apply also the tiled launch) and the lanes per
// row of the factor and of the FP64 apply on the handle's own matrix, and keeps
// the fastest.  The factor is deterministic, so
// re-running it with the same values reproduces the same factor bits.
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

}  // namespace

extern "C" ilu_status ilu_tune(ilu_handle h, const double *a_val, int32_t reps, double *results, int32_t cap,
                               int32_t *n_results, hipStream_t s) {
    if (!h) return fail(ILU_ERR_ARG, "ilu_tune: NULL handle");
    if (!h->factored) return fail(ILU_ERR_STATE, "ilu_tune: requires a factor");
    if (reps < 1) reps = 3;
    const HostAnalysis &H = h->H;
    const int32_t save_fs = h->sched_factor, save_ss = h->sched_solve;
    const int32_t save_lf = h->lanes_factor, save_ls = h->lanes_solve;
    const int32_t k = h->k_used;
    const int32_t casts = (h->has32 ? 1 : 0) | (h->has16 ? 2 : 0);
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
    // ---- factor ----
    int best_fs = save_fs, best_lf = save_lf;
    if (a_val) {
        double best = 1e300;
        const int lmin = std::max(4, save_lf);
        for (int sched = ILU_SCHED_LEVEL; sched <= ILU_SCHED_SYNCFREE; ++sched)
            for (int lanes = lmin; lanes <= 64 && lanes <= 2 * lmin; lanes *= 2) {
                h->sched_factor = sched;
                h->lanes_factor = lanes;
                double us = 0;
                ilu_status st =
                    time_it([&]() { return ilu_factor(h, a_val, k, 0.0, casts, nullptr, s); }, &us);
                if (st != ILU_OK) {
                    h->sched_factor = save_fs;
                    h->lanes_factor = save_lf;
                    return st;
                }
                rows.insert(rows.end(), {0.0, (double)sched, (double)lanes, us});
                if (us < best) {
                    best = us;
                    best_fs = sched;
                    best_lf = lanes;
                }
            }
        h->sched_factor = best_fs;
        h->lanes_factor = best_lf;
        // leave a factor equal to the caller's (tau = 0 and the handle's k)
    }
    // ---- apply (FP64, one right-hand side, permuted space) ----
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, (size_t)H.n * 16);
    if (e != hipSuccess) return hip_fail(e, "ilu_tune: buffers");
    double *b = (double *)buf, *x = b + H.n;
    if ((e = launch_fill_u64((uint64_t *)b, 0x3FF0000000000000ull, H.n, s)) != hipSuccess) {   // b = 1
        (void)hipFree(buf);
        return hip_fail(e, "ilu_tune: fill");
    }
    double best = 1e300;
    int best_ss = save_ss, best_ls = save_ls;
    for (int sched = ILU_SCHED_LEVEL; sched <= ILU_SCHED_SYNCFREE; ++sched)
        for (int lanes = 4; lanes <= 64; lanes *= 2) {
            h->sched_solve = sched;
            h->lanes_solve = lanes;
            double us = 0;
            ilu_status st = time_it(
                [&]() { return ilu_apply(h, b, x, 1, 1, ILU_PREC_F64, ILU_PREC_F64, ILU_PERMUTED_SPACE, s); }, &us);
            if (st != ILU_OK) {
                (void)hipFree(buf);
                h->sched_solve = save_ss;
                h->lanes_solve = save_ls;
                return st;
            }
            rows.insert(rows.end(), {1.0, (double)sched, (double)lanes, us});
            if (us < best) {
                best = us;
                best_ss = sched;
                best_ls = lanes;
            }
        }
    {   // tiled (one candidate: the handle's current tiles); not every tiling fits
        h->sched_solve = ILU_SCHED_TILED;
        double us = 0;
        ilu_status st = time_it(
            [&]() { return ilu_apply(h, b, x, 1, 1, ILU_PREC_F64, ILU_PREC_F64, ILU_PERMUTED_SPACE, s); }, &us);
        if (st == ILU_OK) {
            rows.insert(rows.end(), {1.0, (double)ILU_SCHED_TILED, 0.0, us});
            if (us < best) {
                best = us;
                best_ss = ILU_SCHED_TILED;
                best_ls = save_ls;
            }
        } else if (st != ILU_ERR_UNSUPPORTED) {
            (void)hipFree(buf);
            h->sched_solve = save_ss;
            h->lanes_solve = save_ls;
            return st;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    h->sched_solve = best_ss;
    h->lanes_solve = best_ls;
    const int nr = (int)(rows.size() / 4);
    if (n_results) *n_results = nr;
    if (results && cap > 0) std::memcpy(results, rows.data(), sizeof(double) * 4 * std::min(cap, nr));
    return ILU_OK;
}
