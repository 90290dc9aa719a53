// Krylov drivers that consume the preconditioner: PCG and right-preconditioned
// flexible GMRES(m) (the iterative methods of the paper's Sec. I-II that rely on
// spmv and stri).  Both run in the level ordering (b is permuted once, x is
// permuted back at exit), so every apply and spmv inside the loop streams the
// permuted structures without index translation.  Vector work is FP64; the
// apply uses the requested factor precision.  Scalars stay on the device; the
// host reads back one small block per iteration for the convergence test.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "blas.h"
#include "device.h"
#include "handle.h"
#include "javelin.h"

using namespace jv;

namespace {

ilu_status ensure_kry(ilu_handle_s *h, size_t bytes, hipStream_t s) {
    if (h->kry_bytes >= bytes) return ILU_OK;
    if (h->d_kry) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(h->d_kry);
        allocs_erase(h, h->d_kry);
        h->d_kry = nullptr;
        h->kry_bytes = 0;
    }
    void *p;
    hipError_t e = h->alloc_bytes(&p, bytes);
    if (e != hipSuccess) return hip_fail(e, "krylov workspace");
    h->d_kry = (double *)p;
    h->kry_bytes = bytes;
    return ILU_OK;
}

const void *factor_ptr(ilu_handle_s *h, int prec) {
    if (prec == ILU_PREC_F64) return h->d_lu;
    if (prec == ILU_PREC_F32) return h->has32 ? h->d_lu32 : nullptr;
    if (prec == ILU_PREC_BF16) return h->has16 ? h->d_lu16 : nullptr;
    return nullptr;
}

struct Ctx {
    ilu_handle_s *h;
    int64_t n;
    int prec;
    hipStream_t s;
    double *scal;   // device scalar slots
    double *work;   // dot partials
};

// Pinned readback block: kPinScal scalars, then kPinCoef GMRES coefficients, then the
// info words.
constexpr int kPinScal = 64, kPinCoef = 64;
constexpr size_t kPinBytes = sizeof(double) * (kPinScal + kPinCoef) + sizeof(int32_t) * kInfoSlots;

ilu_status ensure_pin(ilu_handle_s *h) {
    if (!h->h_kry_pin) {
        void *p = nullptr;
        hipError_t e = hipHostMalloc(&p, kPinBytes, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "krylov pinned block");
        h->h_kry_pin = (double *)p;
    }
    if (!h->kry_ev) {
        hipError_t e = hipEventCreateWithFlags(&h->kry_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "krylov event");
    }
    return ILU_OK;
}

// Applies inside a driver skip the per-call guard: the driver runs it once at its
// start and checks the abort flag at every readback, so each apply starts clear.
ilu_status apply(Ctx &c, const double *in, double *out) {
    return run_solves(c.h, 0, factor_ptr(c.h, c.prec), c.prec, 0, in, out, nullptr, nullptr, 1, 1,
                      ILU_PERMUTED_SPACE, c.s, nullptr, false);
}

ilu_status spmv(Ctx &c, double alpha, const double *x, double beta, double *y) {
    return ilu_spmv(c.h, alpha, x, beta, y, 1, 1, ILU_PERMUTED_SPACE, c.s);
}

// A readback is posted and later awaited, so that work that does not depend on the
// scalars (the next preconditioner apply) is queued behind the copies before the host
// waits: the device never idles during the host's convergence test.  post_readback
// queues the copy of `count` device scalars and of the info words (the abort flag and
// the timeout count of the applies queued before it) into the pinned block and
// records the event; wait_readback waits for it, hands the scalars over, and stops
// the driver with ILU_ERR_TIMEOUT when an apply's wait expired, since the iterate is
// then meaningless.
ilu_status post_readback(Ctx &c, const double *dev, int count) {
    hipError_t e = hipMemcpyAsync(c.h->h_kry_pin, dev, sizeof(double) * count, hipMemcpyDeviceToHost, c.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c.h->h_kry_pin + kPinScal + kPinCoef, c.h->d_info, sizeof(int32_t) * kInfoSlots,
                           hipMemcpyDeviceToHost, c.s);
    if (e == hipSuccess) e = hipEventRecord(c.h->kry_ev, c.s);
    if (e != hipSuccess) return hip_fail(e, "krylov readback");
    return ILU_OK;
}

ilu_status wait_readback(Ctx &c, double *host, int count) {
    hipError_t e = hipEventSynchronize(c.h->kry_ev);
    if (e != hipSuccess) return hip_fail(e, "krylov readback");
    std::memcpy(host, c.h->h_kry_pin, sizeof(double) * count);
    int32_t w[kInfoSlots];
    std::memcpy(w, c.h->h_kry_pin + kPinScal + kPinCoef, sizeof(w));
    if (w[kInfoAbort] || w[kInfoTimeouts]) return c.h->take_timeout(c.s, "krylov");
    return ILU_OK;
}

ilu_status readback(Ctx &c, const double *dev, double *host, int count) {
    ilu_status st = post_readback(c, dev, count);
    return st == ILU_OK ? wait_readback(c, host, count) : st;
}

// Whether the step under test is likely not the last: its relative residual,
// extrapolated from the last two by one geometric step, is still above rtol.  A
// speculative apply queued on the last step is a whole apply spent for nothing,
// which costs more than the host wait it hides when applies are long.
bool likely_more(double rel0, double rel1, double rtol) {
    const double pred = rel0 > 0.0 ? rel1 * (rel1 / rel0) : rel1;
    return pred > rtol;
}

#define CHK(x)                          \
    do {                                \
        ilu_status st_ = (x);           \
        if (st_ != ILU_OK) return st_;  \
    } while (0)
#define HCHK(x, what)                                  \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

ilu_status check_common(ilu_handle_s *h, const double *b, double *x, double rtol, int prec, int flags) {
    if (!h) return fail(ILU_ERR_STATE, "solve: NULL handle");
    if (!h->factored || !h->bvals) return fail(ILU_ERR_STATE, "solve: no factor");
    if (!b || !x) return fail(ILU_ERR_ARG, "solve: NULL vector");
    if (!(rtol > 0.0)) return fail(ILU_ERR_ARG, "solve: rtol must be > 0");
    if (flags & ~ILU_PERMUTED_SPACE) return fail(ILU_ERR_ARG, "solve: unknown flags");
    if (!factor_ptr(h, prec)) return fail(ILU_ERR_STATE, "solve: factor precision not available");
    return ILU_OK;
}

}  // namespace

extern "C" ilu_status ilu_solve_pcg(ilu_handle h, const double *b, double *x, double rtol, int32_t maxit,
                                    int32_t fac_prec, int32_t flags, ilu_solve_info *info, hipStream_t s) {
    CHK(check_common(h, b, x, rtol, fac_prec, flags));
    const int64_t n = h->H.n;
    CHK(ensure_kry(h, sizeof(double) * (size_t)n * 6, s));
    CHK(ensure_pin(h));
    CHK(h->ensure_workspace(1, fac_prec == ILU_PREC_F64 ? 0 : 1, s) == hipSuccess ? ILU_OK : fail(ILU_ERR_HIP, "pcg workspace"));
    HCHK(h->guard(s), "pcg guard");
    double *bp = h->d_kry, *xp = bp + n, *r = xp + n, *z = r + n, *p = z + n, *q = p + n;
    Ctx c{h, n, fac_prec, s, h->d_dotwork + kDotParts, h->d_dotwork};
    double *S = c.scal;   // 0 bnorm^2, 1 and 2 r.z (the two alternate), 3 pq, 4 rr
    if (flags & ILU_PERMUTED_SPACE) HCHK(hipMemcpyAsync(bp, b, n * 8, hipMemcpyDeviceToDevice, s), "pcg copy");
    else HCHK(blas_permute(n, h->d_perm, b, bp, 0, s), "pcg permute");
    HCHK(hipMemsetAsync(xp, 0, n * 8, s), "pcg zero");
    HCHK(blas_dot(n, bp, bp, &S[0], c.work, s), "pcg dot");
    double hb[2];
    CHK(readback(c, &S[0], hb, 1));
    const double bnorm = std::sqrt(hb[0]);
    ilu_solve_info I{};
    I.status = ILU_ERR_NOCONV;
    I.relres = 1.0;
    I.true_relres = 1.0;
    if (bnorm == 0.0) {
        I.status = ILU_OK;
        I.relres = I.true_relres = 0.0;
    } else {
        HCHK(hipMemcpyAsync(r, bp, n * 8, hipMemcpyDeviceToDevice, s), "pcg copy");
        double rel0 = 1.0, rel1 = 1.0;   // the last two relative residuals
        for (;;) {
            bool converged = false;
            int cur = 1;   // slot of r.z for the current direction p
            CHK(apply(c, r, z));
            HCHK(hipMemcpyAsync(p, z, n * 8, hipMemcpyDeviceToDevice, s), "pcg copy");
            HCHK(blas_dot(n, r, z, &S[cur], c.work, s), "pcg dot");
            while (I.iters < maxit) {
                CHK(spmv(c, 1.0, p, 0.0, q));
                HCHK(blas_dot(n, p, q, &S[3], c.work, s), "pcg dot");
                HCHK(blas_pcg_xr_rr(n, &S[cur], &S[3], p, q, xp, r, &S[4], c.work, s), "pcg update");
                CHK(post_readback(c, &S[3], 2));
                // The next direction needs only device data: queue it before the host
                // wait, unless this step is likely the last.  When the test below stops
                // the loop, x and r are already final and the speculative z, p and r.z
                // are overwritten before any later use.
                const int nxt = 3 - cur;
                const bool spec = I.iters + 1 < maxit && likely_more(rel0, rel1, rtol);
                if (spec) {
                    CHK(apply(c, r, z));
                    HCHK(blas_dot(n, r, z, &S[nxt], c.work, s), "pcg dot");
                    HCHK(blas_xpby_dev(n, &S[nxt], &S[cur], z, p, s), "pcg p update");
                }
                CHK(wait_readback(c, hb, 2));
                ++I.iters;
                if (hb[0] == 0.0) {
                    I.status = ILU_ERR_BREAKDOWN;
                    break;
                }
                I.relres = std::sqrt(hb[1]) / bnorm;
                if (I.relres <= rtol) {
                    converged = true;
                    break;
                }
                rel0 = rel1;
                rel1 = I.relres;
                if (!spec && I.iters < maxit) {
                    CHK(apply(c, r, z));
                    HCHK(blas_dot(n, r, z, &S[nxt], c.work, s), "pcg dot");
                    HCHK(blas_xpby_dev(n, &S[nxt], &S[cur], z, p, s), "pcg p update");
                }
                cur = nxt;
            }
            // true residual
            HCHK(hipMemcpyAsync(r, bp, n * 8, hipMemcpyDeviceToDevice, s), "pcg copy");
            CHK(spmv(c, -1.0, xp, 1.0, r));
            HCHK(blas_dot(n, r, r, &S[4], c.work, s), "pcg dot");
            CHK(readback(c, &S[4], hb, 1));
            I.true_relres = std::sqrt(hb[0]) / bnorm;
            if (I.true_relres <= rtol) {
                I.status = ILU_OK;
                break;
            }
            if (!converged || I.iters >= maxit || I.status == ILU_ERR_BREAKDOWN) {
                if (I.status != ILU_ERR_BREAKDOWN) I.status = ILU_ERR_NOCONV;
                break;
            }
        }
    }
    if (flags & ILU_PERMUTED_SPACE) HCHK(hipMemcpyAsync(x, xp, n * 8, hipMemcpyDeviceToDevice, s), "pcg copy");
    else HCHK(blas_permute(n, h->d_perm, xp, x, 1, s), "pcg permute");
    HCHK(hipStreamSynchronize(s), "pcg sync");
    if (info) *info = I;
    if (I.status != ILU_OK)
        return fail(I.status, I.status == ILU_ERR_BREAKDOWN ? "pcg: breakdown (p.Ap == 0)" : "pcg: no convergence");
    return ILU_OK;
}

extern "C" ilu_status ilu_solve_gmres(ilu_handle h, const double *b, double *x, double rtol, int32_t restart,
                                      int32_t maxit, int32_t fac_prec, int32_t flags, ilu_solve_info *info,
                                      hipStream_t s) {
    CHK(check_common(h, b, x, rtol, fac_prec, flags));
    if (restart < 1 || restart > 60) return fail(ILU_ERR_ARG, "gmres: restart must be in [1, 60]");
    const int m = restart;
    const int64_t n = h->H.n;
    CHK(ensure_kry(h, sizeof(double) * (size_t)n * (size_t)(2 * m + 4), s));
    CHK(ensure_pin(h));
    CHK(h->ensure_workspace(1, fac_prec == ILU_PREC_F64 ? 0 : 1, s) == hipSuccess ? ILU_OK : fail(ILU_ERR_HIP, "gmres workspace"));
    HCHK(h->guard(s), "gmres guard");
    double *bp = h->d_kry, *xp = bp + n, *w = xp + n, *V = w + n, *Z = V + (size_t)n * (m + 1);
    Ctx c{h, n, fac_prec, s, h->d_dotwork + kDotParts, h->d_dotwork};
    double *S = c.scal;  // 0..m: current Hessenberg column, m+1: beta, m+2..: y coefficients (<= 30)
    if (m + 2 + m > kDotScalars) return fail(ILU_ERR_ARG, "gmres: restart too large for the scalar area");
    if (flags & ILU_PERMUTED_SPACE) HCHK(hipMemcpyAsync(bp, b, n * 8, hipMemcpyDeviceToDevice, s), "gmres copy");
    else HCHK(blas_permute(n, h->d_perm, b, bp, 0, s), "gmres permute");
    HCHK(hipMemsetAsync(xp, 0, n * 8, s), "gmres zero");
    HCHK(blas_dot(n, bp, bp, &S[m + 1], c.work, s, 1), "gmres norm");
    double hb[64];
    CHK(readback(c, &S[m + 1], hb, 1));
    const double bnorm = hb[0];
    ilu_solve_info I{};
    I.status = ILU_ERR_NOCONV;
    I.relres = I.true_relres = 1.0;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), yv(m);
    if (bnorm == 0.0) {
        I.status = ILU_OK;
        I.relres = I.true_relres = 0.0;
    } else {
        for (;;) {
            // r = b - A x, beta = ||r||
            HCHK(hipMemcpyAsync(w, bp, n * 8, hipMemcpyDeviceToDevice, s), "gmres copy");
            CHK(spmv(c, -1.0, xp, 1.0, w));
            HCHK(blas_dot(n, w, w, &S[m + 1], c.work, s, 1), "gmres norm");
            CHK(readback(c, &S[m + 1], hb, 1));
            const double beta = hb[0];
            I.true_relres = beta / bnorm;
            if (I.true_relres <= rtol) {
                I.status = ILU_OK;
                break;
            }
            if (I.iters >= maxit) break;
            HCHK(blas_scale_inv_dev(n, &S[m + 1], w, V, s), "gmres scale");
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int jend = -1;
            bool breakdown = false;
            bool queued = false;   // apply and spmv of step j already queued
            double rel0 = I.true_relres, rel1 = I.true_relres;   // the last two relative residuals
            for (int j = 0; j < m && I.iters < maxit; ++j) {
                double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
                if (!queued) {
                    CHK(apply(c, vj, zj));
                    CHK(spmv(c, 1.0, zj, 0.0, w));
                }
                // modified Gram-Schmidt: each step's update fused with the next
                // step's dot (the last one with the norm)
                HCHK(blas_dot(n, w, V, &S[0], c.work, s), "gmres dot");
                for (int i = 0; i <= j; ++i) {
                    double *vi = V + (size_t)i * n;
                    const bool last = i == j;
                    HCHK(blas_axpy_dot(n, &S[i], -1.0, vi, w, last ? w : vi + n, &S[i + 1], c.work, s, last ? 1 : 0),
                         "gmres orthogonalisation");
                }
                HCHK(blas_scale_inv_dev(n, &S[j + 1], w, V + (size_t)(j + 1) * n, s), "gmres scale");
                CHK(post_readback(c, S, j + 2));
                // The next Arnoldi step's apply and spmv need only v_{j+1}: queue them
                // before the host wait, unless this step is likely the last.  If the
                // test below ends the cycle, their results (z_{j+1} and w) are
                // overwritten before any later use.
                queued = j + 1 < m && I.iters + 1 < maxit && likely_more(rel0, rel1, rtol);
                if (queued) {
                    double *vn = V + (size_t)(j + 1) * n, *zn = Z + (size_t)(j + 1) * n;
                    CHK(apply(c, vn, zn));
                    CHK(spmv(c, 1.0, zn, 0.0, w));
                }
                CHK(wait_readback(c, hb, j + 2));
                for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = hb[i];
                for (int i = 0; i < j; ++i) {   // previous rotations
                    const double a = H[(size_t)i * m + j], cc = H[(size_t)(i + 1) * m + j];
                    const double t1 = cs[i] * a, t2 = sn[i] * cc, t3 = cs[i] * cc, t4 = sn[i] * a;
                    H[(size_t)i * m + j] = t1 + t2;
                    H[(size_t)(i + 1) * m + j] = t3 - t4;
                }
                const double a = H[(size_t)j * m + j], cc = H[(size_t)(j + 1) * m + j];
                const double aa = a * a, c2 = cc * cc;
                const double den = std::sqrt(aa + c2);
                cs[j] = a / den;
                sn[j] = cc / den;
                H[(size_t)j * m + j] = den;
                H[(size_t)(j + 1) * m + j] = 0.0;
                g[j + 1] = -(sn[j] * g[j]);
                g[j] = cs[j] * g[j];
                ++I.iters;
                jend = j;
                I.relres = std::fabs(g[j + 1]) / bnorm;
                breakdown = hb[j + 1] == 0.0;
                if (I.relres <= rtol || breakdown) break;
                rel0 = rel1;
                rel1 = I.relres;
            }
            if (jend < 0) break;
            for (int i = jend; i >= 0; --i) {
                double sum = g[i];
                for (int t = i + 1; t <= jend; ++t) {
                    const double u = H[(size_t)i * m + t] * yv[t];
                    sum = sum - u;
                }
                yv[i] = sum / H[(size_t)i * m + i];
            }
            // The coefficients go through the pinned block's own area, which no later
            // readback writes; the next readback's wait orders any reuse of it.
            double *coef = h->h_kry_pin + kPinScal;
            std::memcpy(coef, yv.data(), sizeof(double) * (jend + 1));
            HCHK(hipMemcpyAsync(&S[m + 2], coef, sizeof(double) * (jend + 1), hipMemcpyHostToDevice, s),
                 "gmres coefficients");
            HCHK(blas_combine(n, jend + 1, &S[m + 2], Z, n, xp, s), "gmres update");
        }
    }
    if (flags & ILU_PERMUTED_SPACE) HCHK(hipMemcpyAsync(x, xp, n * 8, hipMemcpyDeviceToDevice, s), "gmres copy");
    else HCHK(blas_permute(n, h->d_perm, xp, x, 1, s), "gmres permute");
    HCHK(hipStreamSynchronize(s), "gmres sync");
    if (info) *info = I;
    if (I.status != ILU_OK) return fail(I.status, "gmres: no convergence");
    return ILU_OK;
}
