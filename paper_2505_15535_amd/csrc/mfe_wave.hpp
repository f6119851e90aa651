#pragma once

// Tangent apply for Q2 cells (three Gauss points per direction) on
// structured boxes, organised around the wavefront (gfx950, 64 lanes).
//
// A workgroup of four wavefronts owns a brick of eight neighbouring cells.
// Its nodal values are gathered once into LDS (one coalesced load per x-row
// of brick nodes), then every wavefront processes two of the cells on its
// own: lanes 0-26 one cell, lanes 32-58 the other.  A cell has 27 quadrature
// points and, per sweep stage, 27 one-dimensional lines (9 per component),
// so the lane of a half-wavefront is a line in the sum-factorization stages
// (Sec. 2.4, even-odd 1D kernels) and a quadrature point in the point-wise
// stage (the quadrature loop of Alg. 1 / Alg. 2).  The stages pass their
// tensors through a per-cell LDS scratch that only this wavefront touches,
// so they need no workgroup barrier: the LDS executes the instructions of one
// wavefront in issue order, and a compiler barrier between stages keeps that
// order.  Two workgroup barriers remain per brick: after the gather and
// before the brick's nodal sums are formed.
//
// The contributions of the cells to a brick node are summed in LDS in a fixed
// order (cells of lower position first), so within a brick the result does
// not depend on timing.  The sums are then added to v (zero on entry) with
// FP64 (FP32) atomics, or, in the coloured mode, with a plain read-add-write
// by a launch that only holds bricks of one of the eight parity classes of
// (bx, by, bz), none of which share a node -- eight launches in a fixed
// order give a result that is bitwise reproducible.
//
// Constrained dofs (identity rows and columns): the gather reads w as 0
// there, and the brick that owns the node writes v = w (owner: the brick
// whose half-open node range [lo, hi) contains it, the last brick of a
// direction also owning the closing plane).

#include "mfe_cell.hpp"

namespace mfe {

// Keep the compiler from moving LDS accesses across a stage boundary of one
// wavefront; the hardware already executes them in order.
__device__ __forceinline__ void wave_sync() { __asm__ __volatile__("" ::: "memory"); }

// the line of a half-wavefront lane in a stage: l = a + 3 b + 9 c
struct WLine {
    int a, b, c;
};

// ---------------------------------------------------------------------------
// Forward sweeps of one cell.  Input: the field's brick node array B with the
// cell's first node at B + bofs.  Scratch: T (81 values, component-major,
// point q = qx + 3 qy + 9 qz) and Gs (243: Gs[(3 c + d) 27 + q]).  On exit
// Gs holds d field_c / d xi_d at every point.
// ---------------------------------------------------------------------------
template <typename LT, typename TT>
__device__ __forceinline__ void wave_forward(const LT* B, int bofs, LT* Tc, LT* Gs, const Tables<3, TT>& TB,
                                             const WLine& L, bool on) {
    using G = Geo<3, false>;
    const int c27 = 27 * L.c;
    // x: node x-row (j, k) = (a, b) -> values at (qx, j, k)
    if (on) {
        const LT* src = B + bofs + (L.b * G::GY + L.a) * G::ROW + L.c;
        LT x[3] = {src[0], src[3], src[6]}, y[3];
        apply_eo<3, false>(TB.S, x, y);
        LT* o = Tc + c27 + 3 * L.a + 9 * L.b;
        o[0] = y[0];
        o[1] = y[1];
        o[2] = y[2];
    }
    wave_sync();
    // y: line (qx, k) = (a, b), in place
    if (on) {
        LT* o = Tc + c27 + L.a + 9 * L.b;
        LT x[3] = {o[0], o[3], o[6]}, y[3];
        apply_eo<3, false>(TB.S, x, y);
        o[0] = y[0];
        o[3] = y[1];
        o[6] = y[2];
    }
    wave_sync();
    // z: line (qx, qy) = (a, b): values in place, z-derivative into Gs
    if (on) {
        LT* o = Tc + c27 + L.a + 3 * L.b;
        LT x[3] = {o[0], o[9], o[18]}, y[3], dz[3];
        apply_eo<3, false>(TB.S, x, y);
        apply_eo<3, true>(TB.D, y, dz);
        o[0] = y[0];
        o[9] = y[1];
        o[18] = y[2];
        LT* g = Gs + (3 * L.c + 2) * 27 + L.a + 3 * L.b;
        g[0] = dz[0];
        g[9] = dz[1];
        g[18] = dz[2];
    }
    wave_sync();
    // x- and y-derivatives of the values: x-line (qy, qz) = (a, b) and
    // y-line (qx, qz) = (a, b)
    if (on) {
        const LT* vx = Tc + c27 + 3 * L.a + 9 * L.b;
        LT x[3] = {vx[0], vx[1], vx[2]}, y[3];
        apply_eo<3, true>(TB.D, x, y);
        LT* g = Gs + (3 * L.c) * 27 + 3 * L.a + 9 * L.b;
        g[0] = y[0];
        g[1] = y[1];
        g[2] = y[2];
        const LT* vy = Tc + c27 + L.a + 9 * L.b;
        LT x2[3] = {vy[0], vy[3], vy[6]}, y2[3];
        apply_eo<3, true>(TB.D, x2, y2);
        LT* g2 = Gs + (3 * L.c + 1) * 27 + L.a + 9 * L.b;
        g2[0] = y2[0];
        g2[3] = y2[1];
        g2[6] = y2[2];
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Backward sweeps of one cell: on entry Gs[(3 c + d) 27 + q] holds Q[c][d] at
// every point; on exit Tc[27 c + i + 3 j + 9 k] holds
// sum_q sum_d Q[c][d](q) dN_(ijk)/dxi_d(q), the cell's contribution to its
// node (i, j, k).
// ---------------------------------------------------------------------------
template <typename LT>
__device__ __forceinline__ void wave_backward(LT* Tc, LT* Gs, const Tables<3, LT>& TB, const WLine& L, bool on) {
    const int c27 = 27 * L.c;
    // transposed x- and y-derivatives, in place
    if (on) {
        LT* gx = Gs + (3 * L.c) * 27 + 3 * L.a + 9 * L.b;
        LT x[3] = {gx[0], gx[1], gx[2]}, y[3];
        apply_eo<3, true>(TB.Dt, x, y);
        gx[0] = y[0];
        gx[1] = y[1];
        gx[2] = y[2];
        LT* gy = Gs + (3 * L.c + 1) * 27 + L.a + 9 * L.b;
        LT x2[3] = {gy[0], gy[3], gy[6]}, y2[3];
        apply_eo<3, true>(TB.Dt, x2, y2);
        gy[0] = y2[0];
        gy[3] = y2[1];
        gy[6] = y2[2];
    }
    wave_sync();
    // transposed z-derivative, sum of the three directions, transposed
    // z-interpolation: line (qx, qy) = (a, b) -> Tc at (qx, qy, k)
    if (on) {
        const int p0 = L.a + 3 * L.b;
        const LT* g0 = Gs + (3 * L.c) * 27 + p0;
        const LT* g1 = g0 + 27;
        const LT* g2 = g0 + 54;
        LT x[3] = {g2[0], g2[9], g2[18]}, y[3], z[3];
        apply_eo<3, true>(TB.Dt, x, y);
        y[0] += g0[0] + g1[0];
        y[1] += g0[9] + g1[9];
        y[2] += g0[18] + g1[18];
        apply_eo<3, false>(TB.St, y, z);
        LT* o = Tc + c27 + p0;
        o[0] = z[0];
        o[9] = z[1];
        o[18] = z[2];
    }
    wave_sync();
    // transposed y-interpolation: line (qx, k) = (a, b), in place
    if (on) {
        LT* o = Tc + c27 + L.a + 9 * L.b;
        LT x[3] = {o[0], o[3], o[6]}, y[3];
        apply_eo<3, false>(TB.St, x, y);
        o[0] = y[0];
        o[3] = y[1];
        o[6] = y[2];
    }
    wave_sync();
    // transposed x-interpolation: line (j, k) = (a, b), in place
    if (on) {
        LT* o = Tc + c27 + 3 * L.a + 9 * L.b;
        LT x[3] = {o[0], o[1], o[2]}, y[3];
        apply_eo<3, false>(TB.St, x, y);
        o[0] = y[0];
        o[1] = y[1];
        o[2] = y[2];
    }
    wave_sync();
}

// Coefficients of the trilinear Jacobian of one cell: for the derivative
// direction d with the other two reference coordinates (s, t) in increasing
// order, dX/dxi_d = A + s B + t C + s t D with A = e0, B = e1 - e0,
// C = e2 - e0, D = e3 - e2 - e1 + e0 and e_(s_bit + 2 t_bit) the four cell
// edges along d.  Entry (4 d + k) * 3 + comp, k = A, B, C, D.
__device__ __forceinline__ double trilinear_coef(const double* sVert, int vx0, int vy0, int vz0, int idx) {
    using G = Geo<3, false>;
    constexpr int VX = G::BX + 1, VY = G::BY + 1;
    const int comp = idx % 3, dk = idx / 3, d = dk >> 2, k = dk & 3;
    auto X = [&](int v) {  // v = bx + 2 by + 4 bz
        return sVert[(((vz0 + (v >> 2)) * VY + vy0 + ((v >> 1) & 1)) * VX + vx0 + (v & 1)) * 3 + comp];
    };
    auto edge = [&](int a) {  // a = s_bit + 2 t_bit, (s, t) the directions other than d
        const int s_dir = d == 0 ? 1 : 0, t_dir = d == 2 ? 1 : 2;
        const int v0 = ((a & 1) << s_dir) | ((a >> 1) << t_dir);
        return X(v0 | (1 << d)) - X(v0);
    };
    if (k == 0) return edge(0);
    if (k == 1) return edge(1) - edge(0);
    if (k == 2) return edge(2) - edge(0);
    return (edge(3) - edge(2)) - (edge(1) - edge(0));
}

// Bytes of one cell's sweep scratch (324 values; FP64 whenever the u field
// is swept, which uses the same bytes before the w field does).
template <int MODE, typename R>
struct WaveScratch {
    static constexpr int cell_bytes = 324 * (ModeInfo<MODE>::fwd_u ? 8 : (int)sizeof(R));
    static constexpr int bytes = Geo<3, false>::CPB * cell_bytes;
};

// Threads of a workgroup (two cells per wavefront) and brick node entries per thread.
struct WaveGeo {
    static constexpr int NT = 32 * Geo<3, false>::CPB;
    static constexpr int GPT = (Geo<3, false>::BRICK + NT - 1) / NT;
};

// The brick node array entries of this thread: entry e = tid + k NT is
// (node row, offset) = (e / ROW, e % ROW), the x-rows of the brick's nodes
// contiguous as in the global vector; bit k of `exists`: a node of an
// existing cell.
struct WaveMap {
    int dof[WaveGeo::GPT];
    unsigned exists;
};

__device__ __forceinline__ WaveMap wave_map(const KParams& p, const BrickPos& bp) {
    using G = Geo<3, false>;
    WaveMap m;
    m.exists = 0u;
#pragma unroll
    for (int k = 0; k < WaveGeo::GPT; ++k) {
        const int e = threadIdx.x + k * WaveGeo::NT;
        const int row = e / G::ROW, off = e - row * G::ROW;
        const int jr = row % G::GY, kr = row / G::GY, i = off / 3;
        const bool ex = e < G::BRICK && i <= 2 * bp.ncx && jr <= 2 * bp.ncy && kr <= 2 * bp.ncz;
        m.dof[k] = 3 * (bp.node0 + p.Nx * (jr + p.Ny * kr)) + off;
        if (ex) m.exists |= 1u << k;
    }
    return m;
}

template <int MODE, typename R>
__global__ __launch_bounds__(WaveGeo::NT) void wave_kernel(const KParams p, const Tables<3> T, const Tables<3, R> TR) {
    using G = Geo<3, false>;
    static_assert(G::CPB % 2 == 0, "two cells per wavefront");
    constexpr int NT = WaveGeo::NT, GPT = WaveGeo::GPT;
    using MI = ModeInfo<MODE>;
    static_assert(MI::fwd_w, "tangent applies only");
    constexpr bool u_field = MI::fwd_u;
    constexpr bool cached_r = MODE == MODE_APPLY_T2 || MODE == MODE_APPLY_T4;
    using CT = std::conditional_t<cached_r, R, double>;
    constexpr int NCF = MI::cache_fields > 0 ? MI::cache_fields : 1;
    constexpr int NV = (G::BX + 1) * (G::BY + 1) * (G::BZ + 1);

    __shared__ R sW[G::BRICK];
    __shared__ double sU[u_field ? G::BRICK : 1];
    __shared__ double sVert[MI::vertex_geom ? NV * 3 : 1];
    __shared__ double sCoef[MI::vertex_geom ? G::CPB * 36 : 1];
    __shared__ __align__(16) unsigned char sScr[WaveScratch<MODE, R>::bytes];
    constexpr int CB = WaveScratch<MODE, R>::cell_bytes;

    const BrickPos bp = brick_pos<3, false>(p);
    const WaveMap bm = wave_map(p, bp);
    const int tid = threadIdx.x;
    const int lane = tid & 63, half = lane >> 5, l = lane & 31;
    const int lc = 2 * (tid >> 6) + half;
    const int cx = lc % G::BX, cy = (lc / G::BX) % G::BY, cz = lc / (G::BX * G::BY);
    const bool cell_ok = cx < bp.ncx && cy < bp.ncy && cz < bp.ncz;
    const bool on = cell_ok && l < 27;
    const WLine L = {l % 3, (l / 3) % 3, l / 9};
    const int qx = L.a, qy = L.b, qz = L.c;  // the point of this lane, q = l

    // ---- phase 1: global loads, in the order their values are needed (vector
    // memory loads return in issue order): the constraint bits, the brick
    // nodes of u and w, the cell vertices, then the per-point cache fields.
    // Every load is issued unconditionally from an in-bounds address (lanes
    // without data read entry 0 or their cell's last point and discard it), so
    // that no branch separates them and each value is waited for exactly.
    int gdof[GPT];
#pragma unroll
    for (int k = 0; k < GPT; ++k) gdof[k] = (bm.exists >> k & 1u) ? bm.dof[k] : 0;
    uint32_t cm[GPT];
    const uint32_t* cmask = p.cmask ? p.cmask : reinterpret_cast<const uint32_t*>(w_of<R>(p));
#pragma unroll
    for (int k = 0; k < GPT; ++k) cm[k] = cmask[gdof[k] >> 5];
    R wraw[GPT];
    const R* wsrc = w_of<R>(p);
#pragma unroll
    for (int k = 0; k < GPT; ++k) wraw[k] = wsrc[gdof[k]];
    double ub[u_field ? GPT : 1];
    if constexpr (u_field) {
#pragma unroll
        for (int k = 0; k < GPT; ++k) ub[k] = p.u[gdof[k]];
    }
    constexpr int VX = G::BX + 1, VY = G::BY + 1;
    static_assert(NV * 3 <= NT, "one vertex coordinate per thread");
    double vert = 0.0;
    if constexpr (MI::vertex_geom) {
        const int t = min(tid, NV * 3 - 1);
        const int v = t / 3, d = t - 3 * v;
        const int vx = v % VX, vy = (v / VX) % VY, vz = v / (VX * VY);
        // vertices beyond the box belong to no existing cell: clamp
        const int gx = min(bp.ex0 + vx, p.nx), gy = min(bp.ey0 + vy, p.ny), gz = min(bp.ez0 + vz, p.nz);
        vert = p.verts[3 * (gx + (p.nx + 1) * (gy + (p.ny + 1) * gz)) + d];
    }
    const int64_t cbase = (int64_t)bp.brick * NCF * G::NQ + lc * 27 + min(l, 26);
    auto cidx = [&](int f) { return cbase + (int64_t)f * G::NQ; };
    CT cf[NCF];
    const CT* cache = cached_r ? (const CT*)cache_of<R>(p) : (const CT*)p.cache;
    if constexpr (MI::cache_fields > 0) {
#pragma unroll
        for (int f = 0; f < MI::cache_fields; ++f) cf[f] = __builtin_nontemporal_load(cache + cidx(f));
    }
    if constexpr (MI::vertex_geom) {
        if (tid < NV * 3) sVert[tid] = vert;
    }
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
        const int e = tid + k * NT;
        if (e < G::BRICK) {
            const bool zero = !(bm.exists >> k & 1u) || (p.cmask && (cm[k] >> (gdof[k] & 31) & 1u));
            // constrained entries of w read as 0
            sW[e] = zero ? R(0) : wraw[k];
            if constexpr (u_field) sU[e] = (bm.exists >> k & 1u) ? ub[k] : 0.0;
        }
    }
    double mu = p.mu, lam = p.lam;
    if (p.cell_mat != nullptr && cell_ok) {
        const int cell = (bp.ex0 + cx) + p.nx * ((bp.ey0 + cy) + p.ny * (bp.ez0 + cz));
        mu = p.cell_mat[2 * cell];
        lam = p.cell_mat[2 * cell + 1];
    }
    __syncthreads();

    // ---- phase 2: the wavefront's two cells, no workgroup barrier
    const int bofs = ((2 * cz) * G::GY + 2 * cy) * G::ROW + 6 * cx;
    double Jinv[3][3] = {}, JxW = 0.0, du[3][3] = {}, F[3][3] = {};
    Kin kin = {};
    if constexpr (u_field) {
        double* Td = reinterpret_cast<double*>(sScr + lc * CB);
        wave_forward<double, double>(sU, bofs, Td, Td + 81, T, L, on);
        if (on) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) du[c][d] = Td[81 + (3 * c + d) * 27 + l];
        }
        if constexpr (MI::vertex_geom) {
            double* co = sCoef + lc * 36;
            if (cell_ok) {
                for (int i = l; i < 36; i += 32) co[i] = trilinear_coef(sVert, cx, cy, cz, i);
            }
            wave_sync();
            if (on) {
                const double xi[3] = {T.qp[qx], T.qp[qy], T.qp[qz]};
                double Jg[3][3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double s = xi[d == 0 ? 1 : 0], t = xi[d == 2 ? 1 : 2], st = s * t;
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) {
                        const double* cc = co + 12 * d + comp;
                        Jg[comp][d] = fma(st, cc[9], fma(t, cc[6], fma(s, cc[3], cc[0])));
                    }
                }
                double det;
                inverse3(Jg, Jinv, det);
                JxW = det * T.qw[qx] * T.qw[qy] * T.qw[qz];
            }
        } else {  // stored inverse Jacobian and JxW
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) Jinv[i][j] = cf[3 * i + j];
            JxW = cf[9];
        }
        if constexpr (!MI::otf_ad) {
            if (on) kinematics(du, Jinv, F, kin);
        }
        wave_sync();
    }

    R* Tw = reinterpret_cast<R*>(sScr + lc * CB);
    R* Gw = Tw + 81;
    wave_forward<R, R>(sW, bofs, Tw, Gw, TR, L, on);
    R Q[3][3] = {};
    if (on) {
        R dwr[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) dwr[c][d] = Gw[(3 * c + d) * 27 + l];
        if constexpr (u_field) {
            // the point-wise response of the on-the-fly strategies is FP64
            double dw[3][3], Qd[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dw[i][j] = dwr[i][j];
            if constexpr (MODE == MODE_APPLY_OTF_AD) pointwise_otf_ad(du, dw, Jinv, mu, lam, JxW, Qd);
            else if constexpr (MODE == MODE_APPLY_OTF_AD_SPLIT) pointwise_otf_ad_split(du, dw, Jinv, mu, lam, JxW, Qd);
            else pointwise_otf(dw, Jinv, kin, mu, lam, JxW, Qd);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) Q[i][j] = (R)Qd[i][j];
        } else if constexpr (MODE == MODE_APPLY_T2) {
            const R M[3][3] = {{cf[0], cf[1], cf[2]}, {cf[3], cf[4], cf[5]}, {cf[6], cf[7], cf[8]}};
            const R tau[6] = {cf[9], cf[10], cf[11], cf[12], cf[13], cf[14]};
            pointwise_t2(dwr, M, tau, cf[15], cf[16], Q);
        } else if constexpr (MODE == MODE_APPLY_T4) {
            const R M[3][3] = {{cf[27], cf[28], cf[29]}, {cf[30], cf[31], cf[32]}, {cf[33], cf[34], cf[35]}};
            const R tau[6] = {cf[21], cf[22], cf[23], cf[24], cf[25], cf[26]};
            pointwise_t4(dwr, M, cf, tau, Q);
        }
    }
    wave_sync();
    if (on) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) Gw[(3 * c + d) * 27 + l] = Q[c][d];
    }
    wave_sync();
    wave_backward<R>(Tw, Gw, TR, L, on);
    // cells of a ragged brick that lie outside the box contribute zeros
    if (!cell_ok && l < 27) {
        Tw[l] = R(0);
        Tw[l + 27] = R(0);
        Tw[l + 54] = R(0);
    }
    __syncthreads();

    // ---- phase 3: nodal sums of the brick in a fixed order, then the write
    R* vdst = v_of<R>(p);
    const int bx = bp.ex0 / G::BX, by = bp.ey0 / G::BY, bz = bp.ez0 / G::BZ;
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
        const int e = tid + k * NT;
        const int row = e / G::ROW, off = e - row * G::ROW;
        const int J = row % G::GY, K = row / G::GY, I = off / 3, c = off - 3 * I;
        // the cells of the brick holding node (I, J, K): up to two per
        // direction, cell-local index 2 (lower cell) or 0 (upper cell), in
        // the order lower z, y, x first
        R sum = R(0);
#pragma unroll
        for (int dz = (G::BZ > 1 ? -1 : 0); dz <= 0; ++dz) {
            const int ccz = G::BZ > 1 ? K / 2 + dz : 0, kk = K - 2 * ccz;
            const bool vz = ccz >= 0 && ccz < G::BZ && kk <= 2;
#pragma unroll
            for (int dy = -1; dy <= 0; ++dy) {
                const int ccy = J / 2 + dy, jj = J - 2 * ccy;
                const bool vy = ccy >= 0 && ccy < G::BY && jj <= 2;
#pragma unroll
                for (int dx = -1; dx <= 0; ++dx) {
                    const int ccx = I / 2 + dx, ii = I - 2 * ccx;
                    const bool ok = vz && vy && ccx >= 0 && ccx < G::BX && ii <= 2 && e < G::BRICK;
                    const int cell = ccx + G::BX * (ccy + G::BY * ccz);
                    const R val = reinterpret_cast<const R*>(sScr + (ok ? cell : 0) * CB)[ok ? 27 * c + ii + 3 * jj + 9 * kk : 0];
                    sum += ok ? val : R(0);
                }
            }
        }
        if (!(bm.exists >> k & 1u)) continue;
        const int dof = bm.dof[k];
        if (p.cmask && (cm[k] >> (dof & 31) & 1u)) {
            const bool own = (I < 2 * G::BX || bx == p.nbx - 1) && (J < 2 * G::BY || by == p.nby - 1) &&
                             (K < 2 * G::BZ || bz == p.nbz - 1);
            if (!own) continue;
            sum = wraw[k];
        }
        // Every node is added with an atomic, also those no other brick
        // touches: plain stores into cache lines that neighbouring bricks add
        // to atomically cost far more (measured: T2 apply 143 us against 88
        // us on the 48^3 Q2 box).  The coloured mode adds with plain
        // read-add-writes instead (no other launch of its class shares a node).
        if (p.colour > 0) vdst[dof] += sum;
        else unsafeAtomicAdd(vdst + dof, sum);
    }
}

}  // namespace mfe
