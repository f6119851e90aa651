// Kernels of the learned smoother correction: a three-layer 3D convolutional
// network (3x3x3 kernels, zero padding) acting on the 9x9x9 nodal grid of a
// patch of 4x4x4 Q2 cells, its backward pass, the squared-error loss, the Adam
// update, and the gather/scatter between the global nodal vectors and the
// per-patch arrays.  FP32 throughout; reductions are per-workgroup partial
// sums in a fixed order (deterministic).
//
// Activations are [patch][channel][voxel] with voxel v = i + 9 (j + 9 k).
// A layer with CI input and CO output channels stores its weights as
// W[co][ci][tap] (tap = a + 3 (b + 3 c), offsets (a-1, b-1, c-1)) followed by
// the bias[co].

#include <hip/hip_runtime.h>

#include "mfe_kernels.hpp"

namespace mfe {

constexpr int kG = 9;              // nodes per patch direction
constexpr int kV = kG * kG * kG;   // voxels per patch (729)
constexpr int kGP = kG + 2;        // padded tile edge
constexpr int kVP = kGP * kGP * kGP;
constexpr int kNetThreads = 256;
constexpr int kVPT = (kV + kNetThreads - 1) / kNetThreads;  // voxels per thread (3)
constexpr int kCIChunk = 8;        // input channels staged in LDS at a time
constexpr int kCOTile = 8;         // output channels per workgroup

__device__ __forceinline__ int padded_index(int v) {
    const int i = v % kG, j = (v / kG) % kG, k = v / (kG * kG);
    return (i + 1) + kGP * ((j + 1) + kGP * (k + 1));
}

// y[p][co][v] = act(bias[co] + sum_ci sum_tap W[co][ci][tap] x[p][ci][v + off(tap)])
// act: ReLU when relu; then y = 0 where mask[p][co][v] <= 0 when mask is given.
// Transposed use (backward data pass): flip = true reads W as W[ci][co][26 - tap]
// of a layer with CO inputs and CI outputs.
__global__ __launch_bounds__(kNetThreads) void conv3d_kernel(const float* __restrict__ x, const float* __restrict__ W,
                                                             const float* __restrict__ bias, int CI, int CO,
                                                             bool flip, bool relu, const float* __restrict__ mask,
                                                             float* __restrict__ y) {
    __shared__ float sX[kCIChunk * kVP];
    __shared__ float sW[kCOTile * kCIChunk * 27];
    const int p = blockIdx.x;
    const int co0 = blockIdx.y * kCOTile;
    const int nco = min(kCOTile, CO - co0);
    const int tid = threadIdx.x;
    float acc[kVPT][kCOTile];
#pragma unroll
    for (int a = 0; a < kVPT; ++a)
#pragma unroll
        for (int o = 0; o < kCOTile; ++o) acc[a][o] = 0.0f;
    int pv[kVPT];
#pragma unroll
    for (int a = 0; a < kVPT; ++a) {
        const int v = tid + a * kNetThreads;
        pv[a] = padded_index(v < kV ? v : 0);  // idle lanes read a valid tile entry
    }
    for (int ci0 = 0; ci0 < CI; ci0 += kCIChunk) {
        const int nci = min(kCIChunk, CI - ci0);
        __syncthreads();
        for (int e = tid; e < kCIChunk * kVP; e += kNetThreads) {
            const int c = e / kVP, q = e - c * kVP;
            const int i = q % kGP - 1, j = (q / kGP) % kGP - 1, k = q / (kGP * kGP) - 1;
            float val = 0.0f;
            if (c < nci && i >= 0 && i < kG && j >= 0 && j < kG && k >= 0 && k < kG)
                val = x[((int64_t)p * CI + ci0 + c) * kV + i + kG * (j + kG * k)];
            sX[e] = val;
        }
        for (int e = tid; e < kCOTile * kCIChunk * 27; e += kNetThreads) {
            const int o = e / (kCIChunk * 27), r = e - o * kCIChunk * 27;
            const int c = r / 27, t = r - c * 27;
            float w = 0.0f;
            if (o < nco && c < nci) {
                w = flip ? W[((int64_t)(ci0 + c) * CO + (co0 + o)) * 27 + (26 - t)]
                         : W[((int64_t)(co0 + o) * CI + (ci0 + c)) * 27 + t];
            }
            sW[e] = w;
        }
        __syncthreads();
        for (int c = 0; c < nci; ++c) {
            const float* xs = sX + c * kVP;
#pragma unroll
            for (int t = 0; t < 27; ++t) {
                const int off = (t % 3 - 1) + kGP * ((t / 3) % 3 - 1) + kGP * kGP * (t / 9 - 1);
                float xv[kVPT];
#pragma unroll
                for (int a = 0; a < kVPT; ++a) xv[a] = xs[pv[a] + off];
#pragma unroll
                for (int o = 0; o < kCOTile; ++o) {
                    const float w = sW[(o * kCIChunk + c) * 27 + t];
#pragma unroll
                    for (int a = 0; a < kVPT; ++a) acc[a][o] = fmaf(w, xv[a], acc[a][o]);
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < kVPT; ++a) {
        const int v = tid + a * kNetThreads;
        if (v >= kV) continue;
#pragma unroll
        for (int o = 0; o < kCOTile; ++o) {
            if (o >= nco) continue;
            const int64_t idx = ((int64_t)p * CO + co0 + o) * kV + v;
            float val = acc[a][o] + (bias ? bias[co0 + o] : 0.0f);
            if (relu) val = fmaxf(val, 0.0f);
            if (mask && !(mask[idx] > 0.0f)) val = 0.0f;
            y[idx] = val;
        }
    }
}

// dW[co][ci][tap] = sum_p sum_v dy[p][co][v] x[p][ci][v + off(tap)] and, for
// the blocks with ci = 0, db[co] = sum_p sum_v dy[p][co][v].  One workgroup
// per (co, ci); fixed-order tree reduction.
__global__ __launch_bounds__(kNetThreads) void conv3d_wgrad_kernel(const float* __restrict__ x,
                                                                   const float* __restrict__ dy, int P, int CI,
                                                                   int CO, float* __restrict__ dW,
                                                                   float* __restrict__ db) {
    __shared__ float sRed[kNetThreads / 64][28];
    const int co = blockIdx.x, ci = blockIdx.y;
    const int tid = threadIdx.x;
    float acc[28];
#pragma unroll
    for (int t = 0; t < 28; ++t) acc[t] = 0.0f;
    for (int p = 0; p < P; ++p) {
        const float* g = dy + ((int64_t)p * CO + co) * kV;
        const float* xs = x + ((int64_t)p * CI + ci) * kV;
        for (int v = tid; v < kV; v += kNetThreads) {
            const float gv = g[v];
            if (gv == 0.0f) continue;
            const int i = v % kG, j = (v / kG) % kG, k = v / (kG * kG);
            acc[27] += gv;
#pragma unroll
            for (int t = 0; t < 27; ++t) {
                const int ii = i + t % 3 - 1, jj = j + (t / 3) % 3 - 1, kk = k + t / 9 - 1;
                if (ii >= 0 && ii < kG && jj >= 0 && jj < kG && kk >= 0 && kk < kG)
                    acc[t] = fmaf(gv, xs[ii + kG * (jj + kG * kk)], acc[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 28; ++t) {
        float s = acc[t];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if ((tid & 63) == 0) sRed[tid >> 6][t] = s;
    }
    __syncthreads();
    if (tid < 28) {
        float s = 0.0f;
        for (int w = 0; w < kNetThreads / 64; ++w) s += sRed[w][tid];
        if (tid < 27) dW[((int64_t)co * CI + ci) * 27 + tid] = s;
        else if (ci == 0) db[co] = s;
    }
}

// squared error: dy = 2 (y - t) / count; partial[b] = sum over block b of (y - t)^2
__global__ __launch_bounds__(kNetThreads) void mse_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                          int64_t n, float inv_count, float* __restrict__ dy,
                                                          double* __restrict__ partial) {
    __shared__ double sh[kNetThreads / 64];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float d = y[i] - t[i];
        if (dy) dy[i] = 2.0f * d * inv_count;
        s += (double)d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w = 0; w < kNetThreads / 64; ++w) b += sh[w];
        partial[blockIdx.x] = b;
    }
}

// Adam (bias-corrected), step number `step` >= 1
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- patches
// The nodes of patch (px, py, pz) are the box nodes (8 px + i, 8 py + j,
// 8 pz + k), 0 <= i, j, k <= 8; neighbouring patches share their face nodes.

// Features of every patch: channels 0-2 the residual r / s_p with s_p the
// patch's RMS of r (scale[p] = s_p; 0 for a zero residual), channels 3-5 the
// node invariants (I1 - 3, I2 - 3, J - 1).  With `linear` (the network
// variant that is a linear map of r): s_p = 1 and channels 3-5 are 0.  One
// workgroup per patch.
__global__ __launch_bounds__(kNetThreads) void patch_features_kernel(const double* __restrict__ r,
                                                                     const float* __restrict__ inv, int Nx,
                                                                     int Ny, int npx, int npy, bool linear,
                                                                     float* __restrict__ feat,
                                                                     float* __restrict__ scale) {
    __shared__ double sh[kNetThreads / 64];
    __shared__ float s_scale;
    const int p = blockIdx.x;
    const int px = p % npx, py = (p / npx) % npy, pz = p / (npx * npy);
    const int tid = threadIdx.x;
    auto node_of = [&](int v) {
        const int i = v % kG, j = (v / kG) % kG, k = v / (kG * kG);
        return (int64_t)(8 * px + i) + (int64_t)Nx * ((8 * py + j) + (int64_t)Ny * (8 * pz + k));
    };
    double ss = 0.0;
    for (int v = tid; v < kV; v += kNetThreads) {
        const int64_t nd = node_of(v);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double x = r[3 * nd + c];
            ss += x * x;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
    if ((tid & 63) == 0) sh[tid >> 6] = ss;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kNetThreads / 64; ++w) t += sh[w];
        const double rms = linear ? 1.0 : sqrt(t / (3.0 * kV));
        s_scale = (float)rms;
        scale[p] = (float)rms;
    }
    __syncthreads();
    const float s = s_scale;
    const float is = s > 0.0f ? 1.0f / s : 0.0f;
    float* f = feat + (int64_t)p * 6 * kV;
    for (int v = tid; v < kV; v += kNetThreads) {
        const int64_t nd = node_of(v);
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c * kV + v] = (float)r[3 * nd + c] * is;
        f[3 * kV + v] = linear ? 0.0f : inv[3 * nd + 0] - 3.0f;
        f[4 * kV + v] = linear ? 0.0f : inv[3 * nd + 1] - 3.0f;
        f[5 * kV + v] = linear ? 0.0f : inv[3 * nd + 2] - 1.0f;
    }
}

// targets t[p][c][v] = e(node, c) / s_p (0 where s_p = 0)
__global__ void patch_targets_kernel(const double* __restrict__ e, const float* __restrict__ scale, int Nx, int Ny,
                                     int npx, int npy, int P, float* __restrict__ t) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)P * kV) return;
    const int p = (int)(idx / kV), v = (int)(idx % kV);
    const int px = p % npx, py = (p / npx) % npy, pz = p / (npx * npy);
    const int i = v % kG, j = (v / kG) % kG, k = v / (kG * kG);
    const int64_t nd = (int64_t)(8 * px + i) + (int64_t)Nx * ((8 * py + j) + (int64_t)Ny * (8 * pz + k));
    const float s = scale[p];
    const float is = s > 0.0f ? 1.0f / s : 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) t[((int64_t)p * 3 + c) * kV + v] = (float)e[3 * nd + c] * is;
}

// z(node, c) += alpha * mean over the patches that hold the node of s_p y[p][c][v]
__global__ void patch_scatter_kernel(const float* __restrict__ y, const float* __restrict__ scale, int Nx, int Ny,
                                     int Nz, int npx, int npy, int npz, double alpha, double* __restrict__ z) {
    const int64_t nd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (nd >= (int64_t)Nx * Ny * Nz) return;
    const int I = (int)(nd % Nx), J = (int)((nd / Nx) % Ny), K = (int)(nd / ((int64_t)Nx * Ny));
    int pxs[2], ixs[2], nxp = 0, pys[2], iys[2], nyp = 0, pzs[2], izs[2], nzp = 0;
    auto cand = [](int N, int np, int* ps, int* is, int& cnt) {
        const int q = N / 8, rr = N % 8;
        if (rr == 0) {
            if (q - 1 >= 0) { ps[cnt] = q - 1; is[cnt] = 8; ++cnt; }
            if (q < np) { ps[cnt] = q; is[cnt] = 0; ++cnt; }
        } else {
            ps[cnt] = q; is[cnt] = rr; ++cnt;
        }
    };
    cand(I, npx, pxs, ixs, nxp);
    cand(J, npy, pys, iys, nyp);
    cand(K, npz, pzs, izs, nzp);
    double acc[3] = {0.0, 0.0, 0.0};
    int cnt = 0;
    for (int a = 0; a < nxp; ++a)
        for (int b = 0; b < nyp; ++b)
            for (int c = 0; c < nzp; ++c) {
                const int p = pxs[a] + npx * (pys[b] + npy * pzs[c]);
                const int v = ixs[a] + kG * (iys[b] + kG * izs[c]);
                const double s = scale[p];
#pragma unroll
                for (int d = 0; d < 3; ++d) acc[d] += s * (double)y[((int64_t)p * 3 + d) * kV + v];
                ++cnt;
            }
    if (cnt == 0) return;
#pragma unroll
    for (int d = 0; d < 3; ++d) z[3 * nd + d] += alpha * acc[d] / cnt;
}

// Adjoint of the scatter: dy[p][c][v] = alpha * s_p * g(node, c) / (number of
// patches holding the node), the gradient of a loss of z with respect to the
// patch outputs when dL/dz = g.
__global__ void patch_adjoint_kernel(const double* __restrict__ g, const float* __restrict__ scale, int Nx, int Ny,
                                     int npx, int npy, int npz, int P, float alpha, float* __restrict__ dy) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)P * kV) return;
    const int p = (int)(idx / kV), v = (int)(idx % kV);
    const int px = p % npx, py = (p / npx) % npy, pz = p / (npx * npy);
    const int i = v % kG, j = (v / kG) % kG, k = v / (kG * kG);
    // patches sharing the node: 2 along an axis where the node is on an inner patch face
    const int mx = ((i == 0 && px > 0) || (i == kG - 1 && px < npx - 1)) ? 2 : 1;
    const int my = ((j == 0 && py > 0) || (j == kG - 1 && py < npy - 1)) ? 2 : 1;
    const int mz = ((k == 0 && pz > 0) || (k == kG - 1 && pz < npz - 1)) ? 2 : 1;
    const int64_t nd = (int64_t)(8 * px + i) + (int64_t)Nx * ((8 * py + j) + (int64_t)Ny * (8 * pz + k));
    const float f = alpha * scale[p] / (float)(mx * my * mz);
#pragma unroll
    for (int c = 0; c < 3; ++c) dy[((int64_t)p * 3 + c) * kV + v] = f * (float)g[3 * nd + c];
}

// Invariants of C = F^T F at the centre of every Q2 cell (GLL nodes: the
// centre is node (1,1,1) and d/dxi there is the central difference of the
// cell's nodes 0 and 2), then averaged over the cells around each node.
__global__ void cell_invariants_kernel(const double* __restrict__ u, const double* __restrict__ verts, int nx,
                                       int ny, int nz, int Nx, int Ny, float* __restrict__ cinv) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nx * ny * nz) return;
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
    auto vtx = [&](int a, int b, int c, int d) {
        return verts[3 * ((ex + a) + (int64_t)(nx + 1) * ((ey + b) + (int64_t)(ny + 1) * (ez + c))) + d];
    };
    auto un = [&](int a, int b, int c, int d) {
        return u[3 * ((2 * ex + a) + (int64_t)Nx * ((2 * ey + b) + (int64_t)Ny * (2 * ez + c))) + d];
    };
    double Jg[3][3], du[3][3];
    for (int d = 0; d < 3; ++d) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                sx += vtx(1, a, b, d) - vtx(0, a, b, d);
                sy += vtx(a, 1, b, d) - vtx(a, 0, b, d);
                sz += vtx(a, b, 1, d) - vtx(a, b, 0, d);
            }
        Jg[d][0] = 0.25 * sx;
        Jg[d][1] = 0.25 * sy;
        Jg[d][2] = 0.25 * sz;
        du[d][0] = un(2, 1, 1, d) - un(0, 1, 1, d);
        du[d][1] = un(1, 2, 1, d) - un(1, 0, 1, d);
        du[d][2] = un(1, 1, 2, d) - un(1, 1, 0, d);
    }
    // inverse of Jg by cofactors
    double C0[3][3];
    C0[0][0] = Jg[1][1] * Jg[2][2] - Jg[1][2] * Jg[2][1];
    C0[0][1] = Jg[0][2] * Jg[2][1] - Jg[0][1] * Jg[2][2];
    C0[0][2] = Jg[0][1] * Jg[1][2] - Jg[0][2] * Jg[1][1];
    C0[1][0] = Jg[1][2] * Jg[2][0] - Jg[1][0] * Jg[2][2];
    C0[1][1] = Jg[0][0] * Jg[2][2] - Jg[0][2] * Jg[2][0];
    C0[1][2] = Jg[0][2] * Jg[1][0] - Jg[0][0] * Jg[1][2];
    C0[2][0] = Jg[1][0] * Jg[2][1] - Jg[1][1] * Jg[2][0];
    C0[2][1] = Jg[0][1] * Jg[2][0] - Jg[0][0] * Jg[2][1];
    C0[2][2] = Jg[0][0] * Jg[1][1] - Jg[0][1] * Jg[1][0];
    const double det = Jg[0][0] * C0[0][0] + Jg[0][1] * C0[1][0] + Jg[0][2] * C0[2][0];
    double F[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += du[i][k] * C0[k][j] / det;
            F[i][j] = s + (i == j ? 1.0 : 0.0);
        }
    double C[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
    const double I1 = C[0][0] + C[1][1] + C[2][2];
    double trC2 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) trC2 += C[i][j] * C[j][i];
    const double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                     F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                     F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    cinv[3 * e + 0] = (float)I1;
    cinv[3 * e + 1] = (float)(0.5 * (I1 * I1 - trC2));
    cinv[3 * e + 2] = (float)J;
}

__global__ void node_invariants_kernel(const float* __restrict__ cinv, int nx, int ny, int nz, int Nx, int Ny,
                                       int Nz, float* __restrict__ ninv) {
    const int64_t nd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (nd >= (int64_t)Nx * Ny * Nz) return;
    const int I = (int)(nd % Nx), J = (int)((nd / Nx) % Ny), K = (int)(nd / ((int64_t)Nx * Ny));
    // cells holding the node: I in [2 ex, 2 ex + 2]
    int e0[3] = {(I - 1) / 2, (J - 1) / 2, (K - 1) / 2};
    int e1[3] = {I / 2, J / 2, K / 2};
    const int nmax[3] = {nx - 1, ny - 1, nz - 1};
    for (int d = 0; d < 3; ++d) {
        e0[d] = max(0, min(e0[d], nmax[d]));
        e1[d] = max(0, min(e1[d], nmax[d]));
    }
    float acc[3] = {0.0f, 0.0f, 0.0f};
    int cnt = 0;
    for (int cz = e0[2]; cz <= e1[2]; ++cz)
        for (int cy = e0[1]; cy <= e1[1]; ++cy)
            for (int cx = e0[0]; cx <= e1[0]; ++cx) {
                const int64_t e = cx + (int64_t)nx * (cy + (int64_t)ny * cz);
                for (int d = 0; d < 3; ++d) acc[d] += cinv[3 * e + d];
                ++cnt;
            }
    for (int d = 0; d < 3; ++d) ninv[3 * nd + d] = acc[d] / cnt;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_conv3d(const float* x, const float* W, const float* bias, int P, int CI, int CO, bool flip,
                         bool relu, const float* mask, float* y, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    const dim3 grid(P, (CO + kCOTile - 1) / kCOTile);
    hipLaunchKernelGGL(conv3d_kernel, grid, dim3(kNetThreads), 0, s, x, W, bias, CI, CO, flip, relu, mask, y);
    return hipGetLastError();
}

hipError_t launch_conv3d_wgrad(const float* x, const float* dy, int P, int CI, int CO, float* dW, float* db,
                               hipStream_t s) {
    hipLaunchKernelGGL(conv3d_wgrad_kernel, dim3(CO, CI), dim3(kNetThreads), 0, s, x, dy, P, CI, CO, dW, db);
    return hipGetLastError();
}

int mse_blocks(int64_t n) {
    int64_t b = (n + kNetThreads - 1) / kNetThreads;
    return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}

hipError_t launch_mse(const float* y, const float* t, int64_t n, float* dy, double* partial, hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3(mse_blocks(n)), dim3(kNetThreads), 0, s, y, t, n, 1.0f / (float)n, dy,
                       partial);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_patch_features(const double* r, const float* inv, int Nx, int Ny, int npx, int npy, int P,
                                 bool linear, float* feat, float* scale, hipStream_t s) {
    hipLaunchKernelGGL(patch_features_kernel, dim3(P), dim3(kNetThreads), 0, s, r, inv, Nx, Ny, npx, npy, linear,
                       feat, scale);
    return hipGetLastError();
}

hipError_t launch_patch_targets(const double* e, const float* scale, int Nx, int Ny, int npx, int npy, int P,
                                float* t, hipStream_t s) {
    const int64_t n = (int64_t)P * kV;
    hipLaunchKernelGGL(patch_targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, e, scale, Nx, Ny,
                       npx, npy, P, t);
    return hipGetLastError();
}

hipError_t launch_patch_scatter(const float* y, const float* scale, int Nx, int Ny, int Nz, int npx, int npy,
                                int npz, double alpha, double* z, hipStream_t s) {
    const int64_t n = (int64_t)Nx * Ny * Nz;
    hipLaunchKernelGGL(patch_scatter_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, scale, Nx, Ny,
                       Nz, npx, npy, npz, alpha, z);
    return hipGetLastError();
}

hipError_t launch_patch_adjoint(const double* g, const float* scale, int Nx, int Ny, int npx, int npy, int npz,
                                int P, float alpha, float* dy, hipStream_t s) {
    const int64_t n = (int64_t)P * kV;
    hipLaunchKernelGGL(patch_adjoint_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, scale, Nx, Ny,
                       npx, npy, npz, P, alpha, dy);
    return hipGetLastError();
}

hipError_t launch_node_invariants(const double* u, const double* verts, int nx, int ny, int nz, int Nx, int Ny,
                                  int Nz, float* cell_scratch, float* ninv, hipStream_t s) {
    const int64_t ne = (int64_t)nx * ny * nz, nn = (int64_t)Nx * Ny * Nz;
    hipLaunchKernelGGL(cell_invariants_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, u, verts, nx, ny,
                       nz, Nx, Ny, cell_scratch);
    hipLaunchKernelGGL(node_invariants_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, cell_scratch, nx,
                       ny, nz, Nx, Ny, Nz, ninv);
    return hipGetLastError();
}

}  // namespace mfe
