// Vector kernels used by the Krylov drivers (blas.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace jv {

constexpr int kDotParts = 1024;   // fixed partial count: dot products are deterministic
constexpr int kDotScalars = 64;   // device scalar slots the drivers keep after the partials
// bytes of a dot work area: kDotParts partials, then kDotScalars scalar slots
constexpr size_t kDotWorkBytes = sizeof(double) * (kDotParts + kDotScalars);

// *out = x . y (or sqrt of it when sqrt_mode == 1); work is a dot work area
hipError_t blas_dot(int64_t n, const double *x, const double *y, double *out, double *work, hipStream_t s,
                    int sqrt_mode = 0);
// y += sign * *num * x, then *out = y . z of the updated y (z may be y; sqrt of it
// when sqrt_mode == 1), with the bits of the two calls it stands for (work: a dot
// work area)
hipError_t blas_axpy_dot(int64_t n, const double *num, double sign, const double *x, double *y, const double *z,
                         double *out, double *work, hipStream_t s, int sqrt_mode = 0);
// y = x + (*num / *den) * y
hipError_t blas_xpby_dev(int64_t n, const double *num, const double *den, const double *x, double *y,
                         hipStream_t s);
// alpha = *rz / *pq; x += alpha p; r -= alpha q; *rr = r . r of the new r, with
// the bits of blas_dot(r, r) (work: a dot work area)
hipError_t blas_pcg_xr_rr(int64_t n, const double *rz, const double *pq, const double *p, const double *q, double *x,
                          double *r, double *rr, double *work, hipStream_t s);
// y = x / *sc (no-op when *sc == 0)
hipError_t blas_scale_inv_dev(int64_t n, const double *sc, const double *x, double *y, hipStream_t s);
// y = a x + b y (b == 0: y = a x)
hipError_t blas_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
// x += sum_{j<k} c[j] Z[j]   (c on the device)
hipError_t blas_combine(int64_t n, int k, const double *c, const double *Z, int64_t ldz, double *x, hipStream_t s);
// inverse == 0: out[r] = in[perm[r]]; inverse == 1: out[perm[r]] = in[r]
hipError_t blas_permute(int64_t n, const int32_t *perm, const double *in, double *out, int inverse, hipStream_t s);

}  // namespace jv
