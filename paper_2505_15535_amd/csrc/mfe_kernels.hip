// Cell kernels on structured boxes (the templates of mfe_cell.hpp
// instantiated for bricks of neighbouring cells), the launch dispatch between
// box and general-mesh kernels, and small vector kernels.

#include "mfe_cell.hpp"

namespace mfe {

void brick_shape(int n, int* bx, int* by, int* bz, int* points_per_brick) {
    switch (n) {
#define MFE_BRICK_CASE(K)                                                        \
    case K:                                                                      \
        *bx = Geo<K>::BX; *by = Geo<K>::BY; *bz = Geo<K>::BZ; *points_per_brick = Geo<K>::NQ; \
        return;
        MFE_BRICK_CASE(2) MFE_BRICK_CASE(3) MFE_BRICK_CASE(4) MFE_BRICK_CASE(5) MFE_BRICK_CASE(6)
        MFE_BRICK_CASE(7)
#undef MFE_BRICK_CASE
        default: *bx = *by = *bz = *points_per_brick = 0;
    }
}

void hex_group_shape(int n, int* cells, int* points_per_group) {
    switch (n) {
#define MFE_HEX_CASE(K)                                                          \
    case K:                                                                      \
        *cells = Geo<K, true>::CPB; *points_per_group = Geo<K, true>::NQ;         \
        return;
        MFE_HEX_CASE(2) MFE_HEX_CASE(3) MFE_HEX_CASE(4) MFE_HEX_CASE(5) MFE_HEX_CASE(6) MFE_HEX_CASE(7)
#undef MFE_HEX_CASE
        default: *cells = *points_per_group = 0;
    }
}

hipError_t launch_diagonal(const Tables1D& t, const KParams& p, double* diag, hipStream_t stream) {
    if (p.ne <= 0) return hipSuccess;
    if (p.conn) return launch_diagonal_hex(t, p, diag, stream);
    switch (t.n) {
        case 2: return launch_diag_n<2, false>(t, p, diag, stream);
        case 3: return launch_diag_n<3, false>(t, p, diag, stream);
        case 4: return launch_diag_n<4, false>(t, p, diag, stream);
        case 5: return launch_diag_n<5, false>(t, p, diag, stream);
        case 6: return launch_diag_n<6, false>(t, p, diag, stream);
        case 7: return launch_diag_n<7, false>(t, p, diag, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dense_tangent(const Tables1D& t, const KParams& p, double* A, int64_t n, hipStream_t stream) {
    if (p.ne <= 0) return hipSuccess;
    if (p.conn) return hipErrorInvalidValue;  // structured boxes only
    switch (t.n) {
        case 2: return launch_dense_n<2, false>(t, p, A, n, stream);
        case 3: return launch_dense_n<3, false>(t, p, A, n, stream);
        case 4: return launch_dense_n<4, false>(t, p, A, n, stream);
        case 5: return launch_dense_n<5, false>(t, p, A, n, stream);
        case 6: return launch_dense_n<6, false>(t, p, A, n, stream);
        case 7: return launch_dense_n<7, false>(t, p, A, n, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cell_kernel(int mode, const Tables1D& t, const KParams& p, hipStream_t stream, bool fp32,
                              int sweep, const LaunchTiming& tm) {
    if (p.ne <= 0) return hipSuccess;
    if (p.conn) return sweep ? hipErrorInvalidValue : launch_cell_kernel_hex(mode, t, p, stream, fp32, tm);
    if (wave_apply(t.n, mode, false, sweep, fp32, p.colour > 0))
        return launch_wave(mode, fp32, t, p, stream, tm);
    switch (t.n) {
        case 2: return launch_n<2, false>(mode, fp32, t, p, stream, sweep, tm);
        case 3: return launch_n<3, false>(mode, fp32, t, p, stream, sweep, tm);
        case 4: return launch_n<4, false>(mode, fp32, t, p, stream, sweep, tm);
        case 5: return launch_n<5, false>(mode, fp32, t, p, stream, sweep, tm);
        case 6: return launch_n<6, false>(mode, fp32, t, p, stream, sweep, tm);
        case 7: return launch_n<7, false>(mode, fp32, t, p, stream, sweep, tm);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Small vector kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ void fill_kernel(T* __restrict__ x, int64_t n, T value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = value;
}

template <typename T>
__global__ void copy_indexed_kernel(const int64_t* __restrict__ idx, int64_t n, const T* __restrict__ src,
                                    T* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[idx[i]];
}

template <typename T>
__global__ void set_indexed_kernel(const int64_t* __restrict__ idx, int64_t n, T value, T* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = value;
}

__global__ void diff_indexed_kernel(const int64_t* __restrict__ idx, int64_t n, const double* __restrict__ a,
                                    const double* __restrict__ b, double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = a[idx[i]] - b[idx[i]];
}

hipError_t launch_diff_indexed(const int64_t* idx, int64_t n, const double* a, const double* b, double* dst,
                               hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(diff_indexed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, idx, n, a, b,
                       dst);
    return hipGetLastError();
}

template <typename T>
static hipError_t fill_t(T* x, int64_t n, T value, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, stream, x, n, value);
    return hipGetLastError();
}
hipError_t launch_fill(double* x, int64_t n, double value, hipStream_t s) { return fill_t(x, n, value, s); }
hipError_t launch_fill(float* x, int64_t n, float value, hipStream_t s) { return fill_t(x, n, value, s); }

template <typename T>
static hipError_t copy_indexed_t(const int64_t* idx, int64_t n, const T* src, T* dst, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_indexed_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, idx, n,
                       src, dst);
    return hipGetLastError();
}
hipError_t launch_copy_indexed(const int64_t* idx, int64_t n, const double* src, double* dst, hipStream_t s) {
    return copy_indexed_t(idx, n, src, dst, s);
}
hipError_t launch_copy_indexed(const int64_t* idx, int64_t n, const float* src, float* dst, hipStream_t s) {
    return copy_indexed_t(idx, n, src, dst, s);
}

template <typename T>
static hipError_t set_indexed_t(const int64_t* idx, int64_t n, T value, T* dst, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(set_indexed_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, idx, n,
                       value, dst);
    return hipGetLastError();
}
hipError_t launch_set_indexed(const int64_t* idx, int64_t n, double value, double* dst, hipStream_t s) {
    return set_indexed_t(idx, n, value, dst, s);
}
hipError_t launch_set_indexed(const int64_t* idx, int64_t n, float value, float* dst, hipStream_t s) {
    return set_indexed_t(idx, n, value, dst, s);
}

}  // namespace mfe
