// Cell kernels of the matrix-free tangent, residual, state check and cache
// construction on gfx950 (FP64).
//
// One workgroup processes a batch of E consecutive cells (x fastest), with
// one thread per quadrature point of the batch for the point-wise work
// (Alg. 1/Alg. 2 quadrature loop) and one thread per 1D line ("pencil") of a
// component for each sum-factorization sweep (Sec. 2.4).  Intermediate
// tensors are staged in LDS; sweeps between stages are separated by
// workgroup barriers.  The scatter-add into the global result uses hardware
// FP64 atomics.
//
// Sum factorization (collocation form): nodal values are interpolated to the
// Gauss points with three sweeps of S (x, y, z), then the reference gradient
// is taken with the derivative D collocated on the Gauss points; the test
// contraction applies the transposes in reverse order.

#include "mfe_device.hpp"
#include "mfe_kernels.hpp"

namespace mfe {

template <int N>
struct Cfg;
template <> struct Cfg<2> { static constexpr int E = 32, NT = 256; };
template <> struct Cfg<3> { static constexpr int E = 7, NT = 192; };
template <> struct Cfg<4> { static constexpr int E = 4, NT = 256; };
template <> struct Cfg<5> { static constexpr int E = 2, NT = 256; };
template <> struct Cfg<6> { static constexpr int E = 1, NT = 256; };
template <> struct Cfg<7> { static constexpr int E = 1, NT = 384; };

// Map the hardware block index to a batch index so that each of the 8 XCDs
// (blocks are dealt round-robin to them) works on one contiguous range of
// cells and neighbouring cells share that XCD's L2.
__device__ __forceinline__ int xcd_batch(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

__device__ __forceinline__ void cell_coords(const KParams& p, int cell, int& ex, int& ey, int& ez) {
    ex = cell % p.nx;
    const int r = cell / p.nx;
    ey = r % p.ny;
    ez = r / p.ny;
}

// ---------------------------------------------------------------------------
// Forward sweeps of one vector field (3 components) of the batch.
// On exit: sG[((e*N3 + q)*3 + c)*3 + d] = d field_c / d xi_d at point q.
// Uses sA, sB as scratch.  Must be called by every thread of the block.
// MASK: read constrained dofs as zero (the input w of the tangent, not u).
// ---------------------------------------------------------------------------
template <int N, int NT, bool MASK>
__device__ __forceinline__ void forward_sweeps(const double* __restrict__ src, const KParams& p,
                                               int cell0, int nE, const Tables<N>& T,
                                               double* sA, double* sB, double* sG) {
    constexpr int N2 = N * N, N3 = N2 * N, P = N - 1;
    const int tid = threadIdx.x;
    // x: gather an x-row of nodal values, interpolate along x
    for (int t = tid; t < 3 * N2 * nE; t += NT) {
        const int c = t % 3;
        int r = t / 3;
        const int j = r % N;
        r /= N;
        const int k = r % N;
        const int e = r / N;
        int ex, ey, ez;
        cell_coords(p, cell0 + e, ex, ey, ez);
        const int base = P * ex + p.Nx * ((P * ey + j) + p.Ny * (P * ez + k));
        double x[N], y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int dof = 3 * (base + i) + c;
            double val = src[dof];
            if (MASK && p.cmask != nullptr && p.cmask[dof]) val = 0.0;
            x[i] = val;
        }
        apply_eo<N, false>(T.S, x, y);
#pragma unroll
        for (int qx = 0; qx < N; ++qx) sA[(e * N3 + qx + N * (j + N * k)) * 3 + c] = y[qx];
    }
    __syncthreads();
    // y: interpolate along y
    for (int t = tid; t < 3 * N2 * nE; t += NT) {
        const int c = t % 3;
        int r = t / 3;
        const int qx = r % N;
        r /= N;
        const int k = r % N;
        const int e = r / N;
        double x[N], y[N];
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = sA[(e * N3 + qx + N * (j + N * k)) * 3 + c];
        apply_eo<N, false>(T.S, x, y);
#pragma unroll
        for (int qy = 0; qy < N; ++qy) sB[(e * N3 + qx + N * (qy + N * k)) * 3 + c] = y[qy];
    }
    __syncthreads();
    // z: interpolate along z -> values at the Gauss points; z-derivative
    for (int t = tid; t < 3 * N2 * nE; t += NT) {
        const int c = t % 3;
        int r = t / 3;
        const int qx = r % N;
        r /= N;
        const int qy = r % N;
        const int e = r / N;
        double x[N], y[N], dz[N];
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = sB[(e * N3 + qx + N * (qy + N * k)) * 3 + c];
        apply_eo<N, false>(T.S, x, y);
        apply_eo<N, true>(T.D, y, dz);
#pragma unroll
        for (int qz = 0; qz < N; ++qz) {
            const int q = qx + N * (qy + N * qz);
            sA[(e * N3 + q) * 3 + c] = y[qz];
            sG[((e * N3 + q) * 3 + c) * 3 + 2] = dz[qz];
        }
    }
    __syncthreads();
    // x- and y-derivatives of the values at the Gauss points
    for (int t = tid; t < 2 * 3 * N2 * nE; t += NT) {
        const int dir = t & 1;
        int r = t >> 1;
        const int c = r % 3;
        r /= 3;
        const int s = r % N;
        r /= N;
        const int qz = r % N;
        const int e = r / N;
        double x[N], y[N];
        if (dir == 0) {  // line along x at (qy = s, qz)
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sA[(e * N3 + l + N * (s + N * qz)) * 3 + c];
            apply_eo<N, true>(T.D, x, y);
#pragma unroll
            for (int qx = 0; qx < N; ++qx) sG[((e * N3 + qx + N * (s + N * qz)) * 3 + c) * 3 + 0] = y[qx];
        } else {  // line along y at (qx = s, qz)
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sA[(e * N3 + s + N * (l + N * qz)) * 3 + c];
            apply_eo<N, true>(T.D, x, y);
#pragma unroll
            for (int qy = 0; qy < N; ++qy) sG[((e * N3 + s + N * (qy + N * qz)) * 3 + c) * 3 + 1] = y[qy];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Backward sweeps: on entry sG[((e*N3 + q)*3 + c)*3 + d] = Q[c][d] at q; adds
// sum_q sum_d Q[c][d](q) dN_a/dxi_d (q) to dst at the cell's dofs.
// ---------------------------------------------------------------------------
template <int N, int NT>
__device__ __forceinline__ void backward_sweeps(double* __restrict__ dst, const KParams& p, int cell0,
                                                int nE, const Tables<N>& T, double* sA, double* sB,
                                                const double* sG) {
    constexpr int N2 = N * N, N3 = N2 * N, P = N - 1;
    const int tid = threadIdx.x;
    // transposed x- and y-derivatives
    for (int t = tid; t < 2 * 3 * N2 * nE; t += NT) {
        const int dir = t & 1;
        int r = t >> 1;
        const int c = r % 3;
        r /= 3;
        const int s = r % N;
        r /= N;
        const int qz = r % N;
        const int e = r / N;
        double x[N], y[N];
        if (dir == 0) {
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sG[((e * N3 + l + N * (s + N * qz)) * 3 + c) * 3 + 0];
            apply_eo<N, true>(T.Dt, x, y);
#pragma unroll
            for (int qx = 0; qx < N; ++qx) sA[(e * N3 + qx + N * (s + N * qz)) * 3 + c] = y[qx];
        } else {
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sG[((e * N3 + s + N * (l + N * qz)) * 3 + c) * 3 + 1];
            apply_eo<N, true>(T.Dt, x, y);
#pragma unroll
            for (int qy = 0; qy < N; ++qy) sB[(e * N3 + s + N * (qy + N * qz)) * 3 + c] = y[qy];
        }
    }
    __syncthreads();
    // transposed z-derivative, sum of the three directions, transposed z-interpolation
    for (int t = tid; t < 3 * N2 * nE; t += NT) {
        const int c = t % 3;
        int r = t / 3;
        const int qx = r % N;
        r /= N;
        const int qy = r % N;
        const int e = r / N;
        double x[N], y[N], z[N];
#pragma unroll
        for (int l = 0; l < N; ++l) x[l] = sG[((e * N3 + qx + N * (qy + N * l)) * 3 + c) * 3 + 2];
        apply_eo<N, true>(T.Dt, x, y);
#pragma unroll
        for (int qz = 0; qz < N; ++qz) {
            const int q = qx + N * (qy + N * qz);
            y[qz] += sA[(e * N3 + q) * 3 + c] + sB[(e * N3 + q) * 3 + c];
        }
        apply_eo<N, false>(T.St, y, z);
#pragma unroll
        for (int k = 0; k < N; ++k) sA[(e * N3 + qx + N * (qy + N * k)) * 3 + c] = z[k];
    }
    __syncthreads();
    // transposed y-interpolation
    for (int t = tid; t < 3 * N2 * nE; t += NT) {
        const int c = t % 3;
        int r = t / 3;
        const int qx = r % N;
        r /= N;
        const int k = r % N;
        const int e = r / N;
        double x[N], y[N];
#pragma unroll
        for (int qy = 0; qy < N; ++qy) x[qy] = sA[(e * N3 + qx + N * (qy + N * k)) * 3 + c];
        apply_eo<N, false>(T.St, x, y);
#pragma unroll
        for (int j = 0; j < N; ++j) sB[(e * N3 + qx + N * (j + N * k)) * 3 + c] = y[j];
    }
    __syncthreads();
    // transposed x-interpolation and scatter-add
    for (int t = tid; t < 3 * N2 * nE; t += NT) {
        const int c = t % 3;
        int r = t / 3;
        const int j = r % N;
        r /= N;
        const int k = r % N;
        const int e = r / N;
        double x[N], y[N];
#pragma unroll
        for (int qx = 0; qx < N; ++qx) x[qx] = sB[(e * N3 + qx + N * (j + N * k)) * 3 + c];
        apply_eo<N, false>(T.St, x, y);
        int ex, ey, ez;
        cell_coords(p, cell0 + e, ex, ey, ez);
        const int base = P * ex + p.Nx * ((P * ey + j) + p.Ny * (P * ez + k));
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int dof = 3 * (base + i) + c;
            if (p.cmask != nullptr && p.cmask[dof]) continue;
            unsafeAtomicAdd(dst + dof, y[i]);
        }
    }
}

template <int N>
__device__ __forceinline__ void load_grad(const double* sG, int e, int q, double g[3][3]) {
    constexpr int N3 = N * N * N;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[c][d] = sG[((e * N3 + q) * 3 + c) * 3 + d];
}

template <int N>
__device__ __forceinline__ void store_grad(double* sG, int e, int q, const double g[3][3]) {
    constexpr int N3 = N * N * N;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) sG[((e * N3 + q) * 3 + c) * 3 + d] = g[c][d];
}

__device__ __forceinline__ void inverse3(const double Jg[3][3], double Jinv[3][3], double& det) {
    double adj[3][3];
    det = adj_det3(Jg, adj);
    const double r = 1.0 / det;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Jinv[i][j] = adj[i][j] * r;
}

template <int MODE>
struct ModeInfo {
    static constexpr bool fwd_u = MODE == MODE_APPLY_OTF || MODE == MODE_APPLY_OTF_GEOM ||
                                  MODE == MODE_APPLY_OTF_AD || MODE == MODE_RESIDUAL ||
                                  MODE == MODE_STATE || MODE == MODE_BUILD_T2 || MODE == MODE_BUILD_T4;
    static constexpr bool fwd_w = MODE == MODE_APPLY_OTF || MODE == MODE_APPLY_OTF_GEOM ||
                                  MODE == MODE_APPLY_OTF_AD || MODE == MODE_APPLY_T2 ||
                                  MODE == MODE_APPLY_T4;
    static constexpr bool backward = fwd_w || MODE == MODE_RESIDUAL;
    static constexpr bool vertex_geom = MODE == MODE_APPLY_OTF || MODE == MODE_APPLY_OTF_AD ||
                                        MODE == MODE_RESIDUAL || MODE == MODE_STATE ||
                                        MODE == MODE_BUILD_GEOM || MODE == MODE_BUILD_T2 ||
                                        MODE == MODE_BUILD_T4;
};

template <int N, int MODE>
__global__ __launch_bounds__(Cfg<N>::NT) void cell_kernel(const KParams p, const Tables<N> T) {
    constexpr int E = Cfg<N>::E, NT = Cfg<N>::NT;
    constexpr int N3 = N * N * N;
    using MI = ModeInfo<MODE>;
    __shared__ double sA[E * N3 * 3];
    __shared__ double sB[E * N3 * 3];
    __shared__ double sG[E * N3 * 9];
    __shared__ double sEdge[E * 36];

    const int nb = gridDim.x;
    const int batch = xcd_batch(blockIdx.x, nb);
    const int cell0 = batch * E;
    const int nE = min(E, p.ne - cell0);
    if (nE <= 0) return;  // uniform per block
    const int tid = threadIdx.x;
    const int el = tid / N3;
    const int q = tid - el * N3;
    const bool active = el < nE;
    const int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
    const int cell = cell0 + el;
    const int64_t gq = (int64_t)cell * N3 + q;  // global quadrature index

    if constexpr (MI::vertex_geom) {
        for (int t = tid; t < nE * 36; t += NT) {
            const int e = t / 36;
            const int r = t - 36 * e;
            const int edge = r / 3, d = r - 3 * (r / 3);
            int ex, ey, ez;
            cell_coords(p, cell0 + e, ex, ey, ez);
            // edge = 4*dir + a; endpoints differ in bit `dir`
            const int dir = edge >> 2, a = edge & 3;
            int v0;
            if (dir == 0) v0 = 0 | ((a & 1) << 1) | ((a >> 1) << 2);
            else if (dir == 1) v0 = (a & 1) | ((a >> 1) << 2);
            else v0 = (a & 1) | ((a >> 1) << 1);
            const int v1 = v0 | (1 << dir);
            auto vid = [&](int v) {
                return (ex + (v & 1)) + (p.nx + 1) * ((ey + ((v >> 1) & 1)) + (p.ny + 1) * (ez + (v >> 2)));
            };
            sEdge[e * 36 + r] = p.verts[3 * vid(v1) + d] - p.verts[3 * vid(v0) + d];
        }
        // made visible by the first barrier of the forward sweeps / below
    }

    double mu = p.mu, lam = p.lam;
    if (p.cell_mat != nullptr && active) {
        mu = p.cell_mat[2 * cell];
        lam = p.cell_mat[2 * cell + 1];
    }

    if constexpr (MODE == MODE_BUILD_GEOM) {
        __syncthreads();
        if (active) {
            double Jg[3][3], Jinv[3][3], det;
            jacobian_from_edges(sEdge + el * 36, T.qp[qx], T.qp[qy], T.qp[qz], Jg);
            inverse3(Jg, Jinv, det);
            const double JxW = det * T.qw[qx] * T.qw[qy] * T.qw[qz];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) p.cache_out[(3 * i + j) * p.nq_total + gq] = Jinv[i][j];
            p.cache_out[9 * p.nq_total + gq] = JxW;
        }
        return;
    }

    // ---------------- field u: gradients, geometry, kinematics
    double Jinv[3][3] = {}, JxW = 0.0;
    Kin kin = {};
    double F[3][3] = {};
    double du[3][3] = {};
    if constexpr (MI::fwd_u) {
        forward_sweeps<N, NT, false>(p.u, p, cell0, nE, T, sA, sB, sG);
        if (active) {
            load_grad<N>(sG, el, q, du);
            if constexpr (MODE == MODE_APPLY_OTF_GEOM) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Jinv[i][j] = p.cache[(3 * i + j) * p.nq_total + gq];
                JxW = p.cache[9 * p.nq_total + gq];
            } else {
                double Jg[3][3], det;
                jacobian_from_edges(sEdge + el * 36, T.qp[qx], T.qp[qy], T.qp[qz], Jg);
                inverse3(Jg, Jinv, det);
                JxW = det * T.qw[qx] * T.qw[qy] * T.qw[qz];
            }
            if constexpr (MODE != MODE_APPLY_OTF_AD) kinematics(du, Jinv, F, kin);
        }
    }

    if constexpr (MODE == MODE_STATE) {
        if (active && !(kin.J > 0.0)) atomicOr(p.flag, 1);
        return;
    }

    if constexpr (MODE == MODE_BUILD_T2 || MODE == MODE_BUILD_T4) {
        if (active) {
            double M[3][3], tau[6];
            spatial_map(Jinv, kin, M);
            kirchhoff_voigt(F, kin, mu, lam, JxW, tau);
            if constexpr (MODE == MODE_BUILD_T2) {
#pragma unroll
                for (int i = 0; i < 9; ++i) p.cache_out[i * p.nq_total + gq] = M[i / 3][i % 3];
#pragma unroll
                for (int i = 0; i < 6; ++i) p.cache_out[(9 + i) * p.nq_total + gq] = tau[i];
                p.cache_out[15 * p.nq_total + gq] = 2.0 * lam * JxW;
                p.cache_out[16 * p.nq_total + gq] = 2.0 * (mu - 2.0 * lam * kin.lJ) * JxW;
            } else {
                double D21[21];
                spatial_tangent_voigt(kin, mu, lam, JxW, D21);
#pragma unroll
                for (int i = 0; i < 21; ++i) p.cache_out[i * p.nq_total + gq] = D21[i];
#pragma unroll
                for (int i = 0; i < 6; ++i) p.cache_out[(21 + i) * p.nq_total + gq] = tau[i];
#pragma unroll
                for (int i = 0; i < 9; ++i) p.cache_out[(27 + i) * p.nq_total + gq] = M[i / 3][i % 3];
            }
        }
        return;
    }

    // ---------------- field w and the point-wise product
    double Q[3][3] = {};
    if constexpr (MI::fwd_w) {
        if constexpr (!MI::fwd_u) __syncthreads();  // edge table (unused) / uniform entry
        forward_sweeps<N, NT, true>(p.w, p, cell0, nE, T, sA, sB, sG);
        if (active) {
            double dw[3][3];
            load_grad<N>(sG, el, q, dw);
            if constexpr (MODE == MODE_APPLY_OTF || MODE == MODE_APPLY_OTF_GEOM) {
                pointwise_otf(dw, Jinv, kin, mu, lam, JxW, Q);
            } else if constexpr (MODE == MODE_APPLY_OTF_AD) {
                pointwise_otf_ad(du, dw, Jinv, mu, lam, JxW, Q);
            } else if constexpr (MODE == MODE_APPLY_T2) {
                double M[3][3], tau[6];
#pragma unroll
                for (int i = 0; i < 9; ++i) M[i / 3][i % 3] = p.cache[i * p.nq_total + gq];
#pragma unroll
                for (int i = 0; i < 6; ++i) tau[i] = p.cache[(9 + i) * p.nq_total + gq];
                const double c1 = p.cache[15 * p.nq_total + gq];
                const double c2 = p.cache[16 * p.nq_total + gq];
                pointwise_t2(dw, M, tau, c1, c2, Q);
            } else if constexpr (MODE == MODE_APPLY_T4) {
                double D21[21], tau[6], M[3][3];
#pragma unroll
                for (int i = 0; i < 21; ++i) D21[i] = p.cache[i * p.nq_total + gq];
#pragma unroll
                for (int i = 0; i < 6; ++i) tau[i] = p.cache[(21 + i) * p.nq_total + gq];
#pragma unroll
                for (int i = 0; i < 9; ++i) M[i / 3][i % 3] = p.cache[(27 + i) * p.nq_total + gq];
                pointwise_t4(dw, M, D21, tau, Q);
            }
        }
    } else if constexpr (MODE == MODE_RESIDUAL) {
        if (active) pointwise_piola(F, kin, mu, lam, Jinv, JxW, Q);
    }

    if constexpr (MI::backward) {
        // each thread overwrites only its own point's entries, which only it read
        if (active) store_grad<N>(sG, el, q, Q);
        __syncthreads();
        backward_sweeps<N, NT>(p.v, p, cell0, nE, T, sA, sB, sG);
    }
}

// ---------------------------------------------------------------------------
// Host-side launch
// ---------------------------------------------------------------------------
template <int N>
static void fold(const double A[8][8], bool anti, EO<N>& out) {
    constexpr int H = EO<N>::H, M = EO<N>::M;
    for (int q = 0; q < H; ++q)
        for (int i = 0; i < H; ++i) out.E[q][i] = 0.0;
    for (int q = 0; q < H; ++q)
        for (int i = 0; i < (M > 0 ? M : 1); ++i) out.O[q][i] = 0.0;
    for (int q = 0; q < M; ++q) {
        for (int i = 0; i < M; ++i) {
            out.E[q][i] = 0.5 * (A[q][i] + A[q][N - 1 - i]);
            out.O[q][i] = 0.5 * (A[q][i] - A[q][N - 1 - i]);
        }
        if (N % 2 == 1) out.E[q][M] = A[q][M];
    }
    if (N % 2 == 1) {
        if (anti) {
            for (int i = 0; i < M; ++i) out.O[M][i] = A[M][i];
        } else {
            for (int i = 0; i < H; ++i) out.E[M][i] = A[M][i];
        }
    }
}

template <int N>
static Tables<N> make_tables(const Tables1D& t) {
    Tables<N> T;
    double St[8][8], Dt[8][8];
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            St[a][b] = t.S[b][a];
            Dt[a][b] = t.D[b][a];
        }
    fold<N>(t.S, false, T.S);
    fold<N>(St, false, T.St);
    fold<N>(t.D, true, T.D);
    fold<N>(Dt, true, T.Dt);
    for (int i = 0; i < N; ++i) {
        T.qp[i] = t.qp[i];
        T.qw[i] = t.qw[i];
    }
    return T;
}

template <int N, int MODE>
static hipError_t launch_nm(const Tables<N>& T, const KParams& p, hipStream_t stream) {
    constexpr int E = Cfg<N>::E, NT = Cfg<N>::NT;
    const int nb = (p.ne + E - 1) / E;
    hipLaunchKernelGGL((cell_kernel<N, MODE>), dim3(nb), dim3(NT), 0, stream, p, T);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_n(int mode, const Tables1D& t, const KParams& p, hipStream_t s) {
    const Tables<N> T = make_tables<N>(t);
    switch (mode) {
        case MODE_APPLY_OTF: return launch_nm<N, MODE_APPLY_OTF>(T, p, s);
        case MODE_APPLY_OTF_GEOM: return launch_nm<N, MODE_APPLY_OTF_GEOM>(T, p, s);
        case MODE_APPLY_T2: return launch_nm<N, MODE_APPLY_T2>(T, p, s);
        case MODE_APPLY_T4: return launch_nm<N, MODE_APPLY_T4>(T, p, s);
        case MODE_APPLY_OTF_AD: return launch_nm<N, MODE_APPLY_OTF_AD>(T, p, s);
        case MODE_RESIDUAL: return launch_nm<N, MODE_RESIDUAL>(T, p, s);
        case MODE_STATE: return launch_nm<N, MODE_STATE>(T, p, s);
        case MODE_BUILD_GEOM: return launch_nm<N, MODE_BUILD_GEOM>(T, p, s);
        case MODE_BUILD_T2: return launch_nm<N, MODE_BUILD_T2>(T, p, s);
        case MODE_BUILD_T4: return launch_nm<N, MODE_BUILD_T4>(T, p, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cell_kernel(int mode, const Tables1D& t, const KParams& p, hipStream_t stream) {
    if (p.ne <= 0) return hipSuccess;
    switch (t.n) {
        case 2: return launch_n<2>(mode, t, p, stream);
        case 3: return launch_n<3>(mode, t, p, stream);
        case 4: return launch_n<4>(mode, t, p, stream);
        case 5: return launch_n<5>(mode, t, p, stream);
        case 6: return launch_n<6>(mode, t, p, stream);
        case 7: return launch_n<7>(mode, t, p, stream);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Small vector kernels
// ---------------------------------------------------------------------------
__global__ void fill_kernel(double* __restrict__ x, int64_t n, double value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = value;
}

__global__ void copy_indexed_kernel(const int64_t* __restrict__ idx, int64_t n,
                                    const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[idx[i]];
}

__global__ void zero_indexed_kernel(const int64_t* __restrict__ idx, int64_t n, double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = 0.0;
}

hipError_t launch_fill(double* x, int64_t n, double value, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, n, value);
    return hipGetLastError();
}

hipError_t launch_copy_indexed(const int64_t* idx, int64_t n, const double* src, double* dst,
                               hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_indexed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, idx, n,
                       src, dst);
    return hipGetLastError();
}

hipError_t launch_zero_indexed(const int64_t* idx, int64_t n, double* dst, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_indexed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, idx, n,
                       dst);
    return hipGetLastError();
}

}  // namespace mfe
