// Vector kernels of the Krylov drivers: deterministic two-stage dot products
// whose results stay in device memory, and updates whose scalars are read from
// device memory, so a modified Gram-Schmidt sweep needs no host round trip.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "blas.h"

namespace jv {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s = s + part[i];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kBlock) void k_dot_partial(int64_t n, const double *__restrict__ x,
                                                        const double *__restrict__ y, double *__restrict__ part) {
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double p = x[i] * y[i];
        acc = acc + p;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = sum(part); mode 1 stores sqrt of the sum instead
__global__ __launch_bounds__(kBlock) void k_dot_final(int nparts, const double *__restrict__ part, double *out,
                                                      int mode) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) acc = acc + part[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) *out = mode == 1 ? sqrt(s) : s;
}

// One modified Gram-Schmidt step fused with the next one's dot: y += (sign * *num)
// * x, then the partials of y . z for the updated y (z may be y itself), on the
// dot's grid, so k_dot_final gives the bits of a separate dot after the update
__global__ __launch_bounds__(kBlock) void k_axpy_dot(int64_t n, const double *num, double sign,
                                                     const double *__restrict__ x, double *y, const double *z,
                                                     double *__restrict__ part) {
    const double a = sign * *num;
    const bool self = z == y;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double t = a * x[i];
        const double yn = y[i] + t;
        y[i] = yn;
        const double p = yn * (self ? yn : z[i]);
        acc = acc + p;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// y = x + (num / den) * y
__global__ __launch_bounds__(kBlock) void k_xpby_dev(int64_t n, const double *num, const double *den,
                                                     const double *__restrict__ x, double *__restrict__ y) {
    const double b = *num / *den;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double t = b * y[i];
        y[i] = x[i] + t;
    }
}

// PCG step: alpha = rz / pq; x += alpha p; r -= alpha q; with the partials of
// r . r (the new r) on the dot's grid, so k_dot_final gives the bits of a separate
// dot of r with itself
__global__ __launch_bounds__(kBlock) void k_pcg_xr_rr(int64_t n, const double *rz, const double *pq,
                                                      const double *__restrict__ p, const double *__restrict__ q,
                                                      double *__restrict__ x, double *__restrict__ r,
                                                      double *__restrict__ part) {
    const double alpha = *rz / *pq;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double tp = alpha * p[i];
        x[i] = x[i] + tp;
        const double tq = alpha * q[i];
        const double rn = r[i] - tq;
        r[i] = rn;
        const double sq = rn * rn;
        acc = acc + sq;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// y = x * (1 / s) with s read from device memory; leaves y untouched if s == 0
__global__ __launch_bounds__(kBlock) void k_scale_inv_dev(int64_t n, const double *s, const double *__restrict__ x,
                                                          double *__restrict__ y) {
    const double d = *s;
    if (d == 0.0) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) y[i] = x[i] / d;
}

__global__ __launch_bounds__(kBlock) void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                                                  double *__restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double t1 = a * x[i];
        double v = t1;
        if (b != 0.0) {
            const double t2 = b * y[i];
            v = t1 + t2;
        }
        y[i] = v;
    }
}

// x += sum_i c[i] * Z[i] for i < k (columns of Z are n-vectors, stride ldz)
__global__ __launch_bounds__(kBlock) void k_combine(int64_t n, int k, const double *c, const double *__restrict__ Z,
                                                    int64_t ldz, double *__restrict__ x) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double v = x[i];
        for (int j = 0; j < k; ++j) {
            const double t = c[j] * Z[(int64_t)j * ldz + i];
            v = v + t;
        }
        x[i] = v;
    }
}

// out[r] = in[perm[r]] (gather into the level ordering) or out[perm[r]] = in[r]
__global__ __launch_bounds__(kBlock) void k_permute(int64_t n, const int32_t *__restrict__ perm,
                                                    const double *__restrict__ in, double *__restrict__ out,
                                                    int inverse) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += stride) {
        if (inverse) out[perm[r]] = in[r];
        else out[r] = in[perm[r]];
    }
}

int vec_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t blas_dot(int64_t n, const double *x, const double *y, double *out, double *work, hipStream_t s,
                    int sqrt_mode) {
    const int parts = kDotParts;
    hipLaunchKernelGGL(k_dot_partial, dim3(parts), dim3(kBlock), 0, s, n, x, y, work);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, s, parts, work, out, sqrt_mode);
    return hipGetLastError();
}

hipError_t blas_axpy_dot(int64_t n, const double *num, double sign, const double *x, double *y, const double *z,
                         double *out, double *work, hipStream_t s, int sqrt_mode) {
    hipLaunchKernelGGL(k_axpy_dot, dim3(kDotParts), dim3(kBlock), 0, s, n, num, sign, x, y, z, work);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, s, kDotParts, work, out, sqrt_mode);
    return hipGetLastError();
}

hipError_t blas_xpby_dev(int64_t n, const double *num, const double *den, const double *x, double *y,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_xpby_dev, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, num, den, x, y);
    return hipGetLastError();
}

hipError_t blas_pcg_xr_rr(int64_t n, const double *rz, const double *pq, const double *p, const double *q, double *x,
                          double *r, double *rr, double *work, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_xr_rr, dim3(kDotParts), dim3(kBlock), 0, s, n, rz, pq, p, q, x, r, work);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, s, kDotParts, work, rr, 0);
    return hipGetLastError();
}

hipError_t blas_scale_inv_dev(int64_t n, const double *sc, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_inv_dev, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, sc, x, y);
    return hipGetLastError();
}

hipError_t blas_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t blas_combine(int64_t n, int k, const double *c, const double *Z, int64_t ldz, double *x, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, k, c, Z, ldz, x);
    return hipGetLastError();
}

hipError_t blas_permute(int64_t n, const int32_t *perm, const double *in, double *out, int inverse, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, perm, in, out, inverse);
    return hipGetLastError();
}

}  // namespace jv
