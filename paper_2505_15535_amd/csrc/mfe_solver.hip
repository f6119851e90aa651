// Vector kernels of the Newton-CG solver (Sec. 2.2-2.3): fused CG updates
// and deterministic two-pass FP64 dot products.

#include <hip/hip_runtime.h>

#include "mfe_kernels.hpp"

namespace mfe {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    // wavefront reduction, then across the 4 wavefronts of the block
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
    return s;
}

// partials[b] = sum a*b, partials[nb + b] = sum c*d over block b's grid-stride range
__global__ __launch_bounds__(kRedThreads) void dot2_partial_kernel(const double* __restrict__ a,
                                                                   const double* __restrict__ b,
                                                                   const double* __restrict__ c,
                                                                   const double* __restrict__ d, int64_t n,
                                                                   double* __restrict__ partials) {
    __shared__ double sh[kRedThreads / 64];
    double s0 = 0.0, s1 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        s0 = fma(a[i], b[i], s0);
        if (c) s1 = fma(c[i], d[i], s1);
    }
    const double t0 = block_sum(s0, sh);
    const double t1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = t0;
        partials[gridDim.x + blockIdx.x] = t1;
    }
}

// out[0..1] = sums of the two partial arrays (fixed order: deterministic)
__global__ __launch_bounds__(kRedThreads) void reduce2_kernel(const double* __restrict__ partials, int nb,
                                                              double* __restrict__ out) {
    __shared__ double sh[kRedThreads / 64];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        s0 += partials[i];
        s1 += partials[nb + i];
    }
    const double t0 = block_sum(s0, sh);
    const double t1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        out[0] = t0;
        out[1] = t1;
    }
}

// out[0] = sum of x (single workgroup, fixed order)
__global__ __launch_bounds__(kRedThreads) void sum_kernel(const double* __restrict__ x, int64_t n,
                                                          double* __restrict__ out) {
    __shared__ double sh[kRedThreads / 64];
    double s0 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s0 += x[i];
    const double t0 = block_sum(s0, sh);
    if (threadIdx.x == 0) out[0] = t0;
}

// x += alpha p; r -= alpha Ap; z = dinv .* r (z = r without dinv); partial (r.r, r.z)
__device__ __forceinline__ void cg_update_body(double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                                               const double* __restrict__ p, const double* __restrict__ Ap,
                                               const double* __restrict__ dinv, double alpha, int64_t n,
                                               double* __restrict__ partials) {
    __shared__ double sh[kRedThreads / 64];
    double s0 = 0.0, s1 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, Ap[i], r[i]);
        r[i] = ri;
        const double zi = dinv ? dinv[i] * ri : ri;
        z[i] = zi;
        s0 = fma(ri, ri, s0);
        s1 = fma(ri, zi, s1);
    }
    const double t0 = block_sum(s0, sh);
    const double t1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = t0;
        partials[gridDim.x + blockIdx.x] = t1;
    }
}

__global__ __launch_bounds__(kRedThreads) void cg_update_kernel(double* __restrict__ x, double* __restrict__ r,
                                                                double* __restrict__ z, const double* __restrict__ p,
                                                                const double* __restrict__ Ap,
                                                                const double* __restrict__ dinv, double alpha,
                                                                int64_t n, double* __restrict__ partials) {
    cg_update_body(x, r, z, p, Ap, dinv, alpha, n, partials);
}

// The same with alpha = rz / pAp read from device memory, and alpha = 0
// (nothing changes) unless both are positive.
__global__ __launch_bounds__(kRedThreads) void cg_update_dev_kernel(double* __restrict__ x, double* __restrict__ r,
                                                                    double* __restrict__ z,
                                                                    const double* __restrict__ p,
                                                                    const double* __restrict__ Ap,
                                                                    const double* __restrict__ dinv,
                                                                    const double* __restrict__ rz,
                                                                    const double* __restrict__ pAp, int64_t n,
                                                                    double* __restrict__ partials) {
    const double a = rz[0], b = pAp[0];
    cg_update_body(x, r, z, p, Ap, dinv, (a > 0.0 && b > 0.0) ? a / b : 0.0, n, partials);
}

// p = z + beta p with beta = rz_new / rz_old read from device memory (0
// unless rz_old > 0)
__global__ void p_update_dev_kernel(const double* __restrict__ z, const double* __restrict__ rz_new,
                                    const double* __restrict__ rz_old, double* __restrict__ p, int64_t n) {
    const double o = rz_old[0];
    const double beta = o > 0.0 ? rz_new[0] / o : 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = fma(1.0, z[i], beta * p[i]);
}

// x += (nd[0] / nd[1]) y when both are positive and the ratio is finite
__global__ void axpy_ratio_kernel(const double* __restrict__ nd, const double* __restrict__ y, double* __restrict__ x,
                                  int64_t n) {
    const double num = nd[0], den = nd[1];
    double a = (num > 0.0 && den > 0.0) ? num / den : 0.0;
    if (!isfinite(a)) a = 0.0;
    if (a == 0.0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = fma(a, y[i], x[i]);
}

// y = a x + b y
// dst[idx[i]] = src[i]: compact values (one per listed index) into a full vector
__global__ void scatter_indexed_kernel(const int64_t* __restrict__ idx, int64_t n, const double* __restrict__ src,
                                       double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[i];
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = fma(a, x[i], b * y[i]);
}

// y = s * x (elementwise product with s, or copy when s is null) times scale
__global__ void scale_mul_kernel(double scale, const double* __restrict__ s, const double* __restrict__ x,
                                 double* __restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = scale * (s ? s[i] * x[i] : x[i]);
}

// d = 1 / d, or 1 / |d| with `absolute`; entries that are not positive
// (after the absolute value) and finite set *bad
__global__ void invert_kernel(double* __restrict__ d, int64_t n, int* __restrict__ bad, bool absolute) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = absolute ? fabs(d[i]) : d[i];
        if (!(v > 0.0) || !(v < 1e300)) atomicOr(bad, 1);
        d[i] = 1.0 / v;
    }
}

// partials[j * nb + b] = sum over block b of z . Y[j] (Y: m rows of n), j < m <= kMaxDirs
__global__ __launch_bounds__(kRedThreads) void multidot_kernel(const double* __restrict__ z,
                                                               const double* __restrict__ Y, int m, int64_t n,
                                                               double* __restrict__ partials) {
    __shared__ double sh[kRedThreads / 64];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int j = 0; j < m; ++j) {
        const double* y = Y + (int64_t)j * n;
        double acc = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc = fma(z[i], y[i], acc);
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) partials[(int64_t)j * gridDim.x + blockIdx.x] = t;
    }
}

// out[j] = sum of partials[j * nb .. j * nb + nb) (fixed order)
__global__ __launch_bounds__(kRedThreads) void reduce_rows_kernel(const double* __restrict__ partials, int nb, int m,
                                                                  double* __restrict__ out) {
    __shared__ double sh[kRedThreads / 64];
    for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[(int64_t)j * nb + i];
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) out[j] = t;
    }
}

// p = z - sum_j c[j] P[j]
__global__ void multi_axpy_kernel(const double* __restrict__ z, const double* __restrict__ P, DirCoeffs c, int m,
                                  int64_t n, double* __restrict__ p) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double v = z[i];
        for (int j = 0; j < m; ++j) v = fma(-c.c[j], P[(int64_t)j * n + i], v);
        p[i] = v;
    }
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + kRedThreads - 1) / kRedThreads;
    return (unsigned)(b > kDotBlocks ? kDotBlocks : (b < 1 ? 1 : b));
}

hipError_t launch_dot2(const double* a, const double* b, const double* c, const double* d, int64_t n,
                       double* partials, double* out, hipStream_t s) {
    const unsigned nb = grid_for(n);
    hipLaunchKernelGGL(dot2_partial_kernel, dim3(nb), dim3(kRedThreads), 0, s, a, b, c, d, n, partials);
    hipLaunchKernelGGL(reduce2_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_cg_update(double* x, double* r, double* z, const double* p, const double* Ap, const double* dinv,
                            double alpha, int64_t n, double* partials, double* out, hipStream_t s) {
    const unsigned nb = grid_for(n);
    hipLaunchKernelGGL(cg_update_kernel, dim3(nb), dim3(kRedThreads), 0, s, x, r, z, p, Ap, dinv, alpha, n,
                       partials);
    hipLaunchKernelGGL(reduce2_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_cg_update_dev(double* x, double* r, double* z, const double* p, const double* Ap,
                                const double* dinv, const double* rz, const double* pAp, int64_t n, double* partials,
                                double* out, hipStream_t s) {
    const unsigned nb = grid_for(n);
    hipLaunchKernelGGL(cg_update_dev_kernel, dim3(nb), dim3(kRedThreads), 0, s, x, r, z, p, Ap, dinv, rz, pAp, n,
                       partials);
    hipLaunchKernelGGL(reduce2_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_p_update_dev(const double* z, const double* rz_new, const double* rz_old, double* p, int64_t n,
                               hipStream_t s) {
    hipLaunchKernelGGL(p_update_dev_kernel, dim3(grid_for(n)), dim3(kRedThreads), 0, s, z, rz_new, rz_old, p, n);
    return hipGetLastError();
}

hipError_t launch_multidot(const double* z, const double* Y, int m, int64_t n, double* partials, double* out,
                           hipStream_t s) {
    const unsigned nb = grid_for(n) > 256 ? 256 : grid_for(n);  // m * nb partials fit the 2 kDotBlocks scratch
    hipLaunchKernelGGL(multidot_kernel, dim3(nb), dim3(kRedThreads), 0, s, z, Y, m, n, partials);
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, (int)nb, m, out);
    return hipGetLastError();
}

hipError_t launch_multi_axpy(const double* z, const double* P, const DirCoeffs& c, int m, int64_t n, double* p,
                             hipStream_t s) {
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n)), dim3(kRedThreads), 0, s, z, P, c, m, n, p);
    return hipGetLastError();
}

hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kRedThreads), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t launch_axpy_ratio(const double* nd, const double* y, double* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpy_ratio_kernel, dim3(grid_for(n)), dim3(kRedThreads), 0, s, nd, y, x, n);
    return hipGetLastError();
}

hipError_t launch_scatter_indexed(const int64_t* idx, int64_t n, const double* src, double* dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_indexed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx, n, src, dst);
    return hipGetLastError();
}
hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(kRedThreads), 0, s, a, x, b, y, n);
    return hipGetLastError();
}

hipError_t launch_scale_mul(double scale, const double* sc, const double* x, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(scale_mul_kernel, dim3(grid_for(n)), dim3(kRedThreads), 0, s, scale, sc, x, y, n);
    return hipGetLastError();
}

hipError_t launch_invert(double* d, int64_t n, int* bad, hipStream_t s, bool absolute) {
    hipLaunchKernelGGL(invert_kernel, dim3(grid_for(n)), dim3(kRedThreads), 0, s, d, n, bad, absolute);
    return hipGetLastError();
}

}  // namespace mfe
