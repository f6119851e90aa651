// Kernels of the geometric multigrid preconditioner (Sec. 2.3): grid
// transfers between nested Q_p boxes as tensor products of 1D matrices
// (prolongation, restriction, interpolation of the linearisation point to the
// coarser level), the Chebyshev-Jacobi smoother update, the precision
// conversions of the mixed-precision V-cycle and the direct solve on a small
// coarsest level.  FP64 and FP32 instances.

#include <hip/hip_runtime.h>

#include "mfe_kernels.hpp"

namespace mfe {

// out = M_axis in, where M (rows x cols, CSR) acts along `axis` of nodal
// arrays [nz][ny][nx][3]; the other two extents are shared by in and out.
// Fused forms for the V-cycle (f.dinv: the level's inverse diagonal, 0 at
// constrained dofs):
//   f.b != null:  in is read as the free-dof residual (dinv != 0) ? b - in : 0
//   f.x != null:  x[t] += (dinv[t] != 0) ? result : 0 and f.clear[t] = 0
//                 (out is not written)
template <typename T>
struct AxisFuse {
    const T* b = nullptr;
    const T* dinv = nullptr;
    T* x = nullptr;
    T* clear = nullptr;
};

template <typename T>
__global__ void axis_csr_kernel(const int* __restrict__ rowptr, const int* __restrict__ colidx,
                                const T* __restrict__ vals, int axis, int nx_out, int ny_out, int nz_out,
                                int nx_in, int ny_in, const T* __restrict__ in, T* __restrict__ out,
                                AxisFuse<T> f) {
    const int64_t n = (int64_t)nx_out * ny_out * nz_out * 3;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const int c = (int)(t % 3);
        int64_t r = t / 3;
        const int i = (int)(r % nx_out);
        r /= nx_out;
        const int j = (int)(r % ny_out);
        const int k = (int)(r / ny_out);
        const int row = axis == 0 ? i : (axis == 1 ? j : k);
        T s = 0;
        for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) {
            const int col = colidx[e];
            const int ii = axis == 0 ? col : i, jj = axis == 1 ? col : j, kk = axis == 2 ? col : k;
            const int64_t q = 3 * (ii + (int64_t)nx_in * (jj + (int64_t)ny_in * kk)) + c;
            T v = in[q];
            if (f.b) v = f.dinv[q] != T(0) ? f.b[q] - v : T(0);
            s = fma(vals[e], v, s);
        }
        if (f.x) {
            if (f.dinv[t] != T(0)) f.x[t] += s;
            f.clear[t] = T(0);
        } else {
            out[t] = s;
        }
    }
}

// Chebyshev step with the residual formed on the fly:
//   d = c1 d + c2 dinv .* (b - Ax);  x += d (x = d when x_init);  Ax = 0
// (Ax null: residual b; c1 = 0: d is not read).  Clearing Ax leaves the
// buffer ready for the next operator application, which accumulates.
template <typename T>
__global__ void cheb_kernel(T* __restrict__ d, T* __restrict__ x, const T* __restrict__ b, T* __restrict__ Ax,
                            const T* __restrict__ dinv, T c1, T c2, int64_t n, bool x_init) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        T r = b[i];
        if (Ax) {
            r -= Ax[i];
            Ax[i] = T(0);
        }
        const T step = c2 * dinv[i] * r;
        const T di = c1 == T(0) ? step : fma(c1, d[i], step);
        d[i] = di;
        x[i] = x_init ? di : x[i] + di;
    }
}

// x += y;  y = 0
template <typename T>
__global__ void add_clear_kernel(T* __restrict__ x, T* __restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        x[i] += y[i];
        y[i] = T(0);
    }
}

// y = x (plain copy)
template <typename T>
__global__ void copy_kernel(const T* __restrict__ x, T* __restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = x[i];
}

// y = a x + b y
template <typename T>
__global__ void axpby_t_kernel(T a, const T* __restrict__ x, T b, T* __restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = fma(a, x[i], b * y[i]);
}

template <typename S, typename D>
__global__ void convert_kernel(const S* __restrict__ src, D* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (D)src[i];
}

static unsigned grid_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

template <typename T>
static hipError_t axis_csr_t(const int* rowptr, const int* colidx, const T* vals, int axis, int nx_out, int ny_out,
                             int nz_out, int nx_in, int ny_in, const T* in, T* out, const T* rb, const T* dinv,
                             T* x, T* clear, hipStream_t s) {
    const int64_t n = (int64_t)nx_out * ny_out * nz_out * 3;
    AxisFuse<T> f;
    f.b = rb;
    f.dinv = dinv;
    f.x = x;
    f.clear = clear;
    hipLaunchKernelGGL(axis_csr_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, rowptr, colidx, vals, axis, nx_out,
                       ny_out, nz_out, nx_in, ny_in, in, out, f);
    return hipGetLastError();
}
hipError_t launch_axis_csr(const int* rowptr, const int* colidx, const double* vals, int axis, int nx_out,
                           int ny_out, int nz_out, int nx_in, int ny_in, const double* in, double* out,
                           hipStream_t s, const double* rb, const double* dinv, double* x, double* clear) {
    return axis_csr_t(rowptr, colidx, vals, axis, nx_out, ny_out, nz_out, nx_in, ny_in, in, out, rb, dinv, x, clear,
                      s);
}
hipError_t launch_axis_csr(const int* rowptr, const int* colidx, const float* vals, int axis, int nx_out,
                           int ny_out, int nz_out, int nx_in, int ny_in, const float* in, float* out,
                           hipStream_t s, const float* rb, const float* dinv, float* x, float* clear) {
    return axis_csr_t(rowptr, colidx, vals, axis, nx_out, ny_out, nz_out, nx_in, ny_in, in, out, rb, dinv, x, clear,
                      s);
}

template <typename T>
static hipError_t cheb_t(T* d, T* x, const T* b, T* Ax, const T* dinv, T c1, T c2, int64_t n, bool x_init,
                         hipStream_t s) {
    hipLaunchKernelGGL(cheb_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, d, x, b, Ax, dinv, c1, c2, n, x_init);
    return hipGetLastError();
}
hipError_t launch_cheb(double* d, double* x, const double* b, double* Ax, const double* dinv, double c1,
                       double c2, int64_t n, hipStream_t s, bool x_init) {
    return cheb_t(d, x, b, Ax, dinv, c1, c2, n, x_init, s);
}
hipError_t launch_cheb(float* d, float* x, const float* b, float* Ax, const float* dinv, float c1, float c2,
                       int64_t n, hipStream_t s, bool x_init) {
    return cheb_t(d, x, b, Ax, dinv, c1, c2, n, x_init, s);
}

template <typename T>
static hipError_t add_clear_t(T* x, T* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(add_clear_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}
hipError_t launch_add_clear(double* x, double* y, int64_t n, hipStream_t s) { return add_clear_t(x, y, n, s); }
hipError_t launch_add_clear(float* x, float* y, int64_t n, hipStream_t s) { return add_clear_t(x, y, n, s); }

template <typename T>
static hipError_t copy_t(const T* x, T* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}
hipError_t launch_copy(const double* x, double* y, int64_t n, hipStream_t s) { return copy_t(x, y, n, s); }
hipError_t launch_copy(const float* x, float* y, int64_t n, hipStream_t s) { return copy_t(x, y, n, s); }

hipError_t launch_axpby(float a, const float* x, float b, float* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_t_kernel<float>, dim3(grid_of(n)), dim3(256), 0, s, a, x, b, y, n);
    return hipGetLastError();
}

hipError_t launch_convert(const double* src, float* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(grid_of(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}
hipError_t launch_convert(const float* src, double* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(grid_of(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Direct solve on the coarsest level: the inverse of its tangent on the free
// dofs (nf <= kDenseMax) is formed once per linearisation point and applied
// as one matrix-vector product per V-cycle.
// ---------------------------------------------------------------------------
constexpr int kSweepThreads = 1024;                          // 16 wavefronts
constexpr int kSweepWaves = kSweepThreads / 64;
constexpr int kSweepNB = (kDenseMax + 7) / 8;                 // 8 x 8 blocks per row
constexpr int kSweepBlocks = kSweepNB * (kSweepNB + 1) / 2;   // blocks of the lower triangle
constexpr int kSweepPer = (kSweepBlocks + kSweepWaves - 1) / kSweepWaves;  // blocks per wavefront

// One workgroup.  The free block of A is inverted in place by the symmetric
// sweep operator (Goodnight 1979): for each pivot k, with c = column k and
// d = c_k,
//   a_ij -= c_i c_j / d (i, j != k),  a_ik = c_i / d (i != k),  a_kk = -1 / d,
// which leaves -A^-1 once every pivot is swept; every pivot is positive
// exactly when A is positive definite.  The lower triangle is split into 8 x 8
// blocks (diagonal blocks kept whole), dealt round-robin to the wavefronts;
// lane l holds entry (8 bi + l / 8, 8 bj + l % 8) of each of its blocks in a
// register.  Per pivot only column k passes through LDS, and a wavefront's
// reads of it touch 8 distinct addresses.  Ainv (nf x nf, row-major) = A^-1.
__global__ __launch_bounds__(kSweepThreads) void sweep_inverse_kernel(const double* __restrict__ A, int n,
                                                                      const int* __restrict__ free_idx, int nf,
                                                                      double* __restrict__ Ainv,
                                                                      int* __restrict__ fail) {
    __shared__ double sCol[kSweepNB * 8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nb = (nf + 7) / 8, nblocks = nb * (nb + 1) / 2;
    double v[kSweepPer];
    int ij[kSweepPer];  // i << 16 | j of the entry held, or -1
#pragma unroll
    for (int m = 0; m < kSweepPer; ++m) {
        const int blk = wave + kSweepWaves * m;
        v[m] = 0.0;
        ij[m] = -1;
        if (blk < nblocks) {
            int bi = (int)((sqrt(8.0 * (double)blk + 1.0) - 1.0) * 0.5);
            while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
            while (bi * (bi + 1) / 2 > blk) --bi;
            const int bj = blk - bi * (bi + 1) / 2;
            const int i = 8 * bi + (lane >> 3), j = 8 * bj + (lane & 7);
            if (i < nf && j < nf) {
                ij[m] = i << 16 | j;
                v[m] = A[(int64_t)free_idx[i] * n + free_idx[j]];
            }
        }
    }
    bool bad = false;
    for (int k = 0; k < nf; ++k) {
        // column k: the entries (i, k) held, and by symmetry (k, j) of the
        // blocks left of the diagonal block of row k
#pragma unroll
        for (int m = 0; m < kSweepPer; ++m) {
            const int e = ij[m];
            if (e < 0) continue;
            const int i = e >> 16, j = e & 0xffff;
            if (j == k) sCol[i] = v[m];
            else if (i == k && (j >> 3) < (k >> 3)) sCol[j] = v[m];
        }
        __syncthreads();
        const double d = sCol[k];  // the same value in every thread
        if (!(d > 0.0) || !isfinite(d)) {
            bad = true;
            break;
        }
        const double rd = 1.0 / d;
#pragma unroll
        for (int m = 0; m < kSweepPer; ++m) {
            const int e = ij[m];
            if (e < 0) continue;
            const int i = e >> 16, j = e & 0xffff;
            const double ci = sCol[i], cj = sCol[j];
            if (i != k && j != k) v[m] -= ci * cj * rd;
            else if (i == k && j == k) v[m] = -rd;
            else v[m] = (i == k ? cj : ci) * rd;
        }
        __syncthreads();
    }
    if (bad) {
        if (threadIdx.x == 0) *fail = 1;
        return;
    }
#pragma unroll
    for (int m = 0; m < kSweepPer; ++m) {
        const int e = ij[m];
        if (e < 0) continue;
        const int i = e >> 16, j = e & 0xffff;
        Ainv[(int64_t)i * nf + j] = -v[m];
        if ((i >> 3) != (j >> 3)) Ainv[(int64_t)j * nf + i] = -v[m];
    }
    if (threadIdx.x == 0) *fail = 0;
}

// x[r] = sum_j Ainv[pos[r]][j] b[free_idx[j]] for a free dof r, 0 for a
// constrained one (pos[r] < 0): one wavefront per dof
template <typename T>
__global__ __launch_bounds__(256) void dense_matvec_kernel(const T* __restrict__ Ainv, const int* __restrict__ pos,
                                                           const int* __restrict__ free_idx, int nf,
                                                           const T* __restrict__ b, T* __restrict__ x, int n) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;  // whole wavefronts
    const int fi = pos[row];
    if (fi < 0) {
        if (lane == 0) x[row] = T(0);
        return;
    }
    T s = T(0);
    for (int j = lane; j < nf; j += 64) s += Ainv[(int64_t)fi * nf + j] * b[free_idx[j]];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) x[row] = s;
}

hipError_t launch_sweep_inverse(const double* A, int n, const int* free_idx, int nf, double* Ainv, int* fail,
                                hipStream_t s) {
    if (nf <= 0 || nf > kDenseMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sweep_inverse_kernel, dim3(1), dim3(kSweepThreads), 0, s, A, n, free_idx, nf, Ainv, fail);
    return hipGetLastError();
}

template <typename T>
static hipError_t dense_matvec_t(const T* Ainv, const int* pos, const int* free_idx, int nf, const T* b, T* x, int n,
                                 hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dense_matvec_kernel<T>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, Ainv, pos, free_idx,
                       nf, b, x, n);
    return hipGetLastError();
}
hipError_t launch_dense_matvec(const double* Ainv, const int* pos, const int* free_idx, int nf, const double* b,
                               double* x, int n, hipStream_t s) {
    return dense_matvec_t(Ainv, pos, free_idx, nf, b, x, n, s);
}
hipError_t launch_dense_matvec(const float* Ainv, const int* pos, const int* free_idx, int nf, const float* b,
                               float* x, int n, hipStream_t s) {
    return dense_matvec_t(Ainv, pos, free_idx, nf, b, x, n, s);
}

}  // namespace mfe
