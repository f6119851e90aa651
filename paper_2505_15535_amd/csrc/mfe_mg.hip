// Kernels of the geometric multigrid preconditioner (Sec. 2.3): grid
// transfers between nested Q_p boxes as tensor products of 1D matrices
// (prolongation, restriction, interpolation of the linearisation point to the
// coarser level), and the Chebyshev-Jacobi smoother update.

#include <hip/hip_runtime.h>

#include "mfe_kernels.hpp"

namespace mfe {

// out = M_axis in, where M (rows x cols, CSR) acts along `axis` of nodal
// arrays [nz][ny][nx][3]; the other two extents are shared by in and out.
__global__ void axis_csr_kernel(const int* __restrict__ rowptr, const int* __restrict__ colidx,
                                const double* __restrict__ vals, int axis, int nx_out, int ny_out, int nz_out,
                                int nx_in, int ny_in, const double* __restrict__ in, double* __restrict__ out) {
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
        double s = 0.0;
        for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) {
            const int col = colidx[e];
            const int ii = axis == 0 ? col : i, jj = axis == 1 ? col : j, kk = axis == 2 ? col : k;
            s = fma(vals[e], in[3 * (ii + (int64_t)nx_in * (jj + (int64_t)ny_in * kk)) + c], s);
        }
        out[t] = s;
    }
}

// Chebyshev step: d = c1 d + c2 dinv .* r;  x += d  (d is not read when c1 = 0)
__global__ void cheb_kernel(double* __restrict__ d, double* __restrict__ x, const double* __restrict__ r,
                            const double* __restrict__ dinv, double c1, double c2, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double step = c2 * dinv[i] * r[i];
        const double di = c1 == 0.0 ? step : fma(c1, d[i], step);
        d[i] = di;
        x[i] += di;
    }
}

static unsigned grid_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

hipError_t launch_axis_csr(const int* rowptr, const int* colidx, const double* vals, int axis, int nx_out,
                           int ny_out, int nz_out, int nx_in, int ny_in, const double* in, double* out,
                           hipStream_t s) {
    const int64_t n = (int64_t)nx_out * ny_out * nz_out * 3;
    hipLaunchKernelGGL(axis_csr_kernel, dim3(grid_of(n)), dim3(256), 0, s, rowptr, colidx, vals, axis, nx_out,
                       ny_out, nz_out, nx_in, ny_in, in, out);
    return hipGetLastError();
}

hipError_t launch_cheb(double* d, double* x, const double* r, const double* dinv, double c1, double c2, int64_t n,
                       hipStream_t s) {
    hipLaunchKernelGGL(cheb_kernel, dim3(grid_of(n)), dim3(256), 0, s, d, x, r, dinv, c1, c2, n);
    return hipGetLastError();
}

}  // namespace mfe
