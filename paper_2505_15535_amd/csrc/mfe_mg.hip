// Kernels of the geometric multigrid preconditioner (Sec. 2.3): grid
// transfers between nested Q_p boxes as tensor products of 1D matrices
// (prolongation, restriction, interpolation of the linearisation point to the
// coarser level), the Chebyshev-Jacobi smoother update and the precision
// conversions of the mixed-precision V-cycle.  FP64 and FP32 instances.

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

}  // namespace mfe
