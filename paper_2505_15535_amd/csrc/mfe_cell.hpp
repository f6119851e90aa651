#pragma once

// Cell kernels of the matrix-free tangent, residual, state check and cache
// construction on gfx950.  Every kernel exists in FP64; the tangent applies
// and the T2/T4 cache builds also exist with FP32 input/output vectors and
// FP32 sum-factorization sweeps (mixed precision: F, J and log J, the
// geometry and the cached data are computed in FP64 and rounded once).
//
// Templates of the cell kernels, shared by the structured-box instantiations
// (mfe_kernels.hip) and the general-hexahedral-mesh ones (mfe_kernels_hex.hip).
//
// One workgroup processes a brick of neighbouring cells (4x2x1 for Q2), with
// one thread per quadrature point of the brick for the point-wise work
// (Alg. 1/Alg. 2 quadrature loop) and one thread per 1D line of a component
// for each sum-factorization sweep (Sec. 2.4).  The brick's nodal values are
// gathered once with coalesced row loads into LDS; intermediate tensors are
// staged in LDS with workgroup barriers between sweep stages.  The cells'
// contributions are summed in LDS, then every node of the brick is added to
// v with one atomic.  Per-point caches are stored brick-major so that a
// workgroup streams one contiguous range.
//
// Sum factorization (collocation form): nodal values are interpolated to the
// Gauss points with three sweeps of S (x, y, z), then the reference gradient
// is taken with the derivative D collocated on the Gauss points; the test
// contraction applies the transposes in reverse order.

#include <type_traits>

#include <hip/hip_ext.h>

#include "mfe_device.hpp"
#include "mfe_kernels.hpp"

namespace mfe {

// Bricks: a workgroup owns BX x BY x BZ neighbouring cells of the box.  The
// Q2 shape can be chosen at build time (cells per direction).
#ifndef MFE_Q2_BRICK_X
#define MFE_Q2_BRICK_X 4
#endif
#ifndef MFE_Q2_BRICK_Y
#define MFE_Q2_BRICK_Y 2
#endif
#ifndef MFE_Q2_BRICK_Z
#define MFE_Q2_BRICK_Z 1
#endif
template <int N> struct BrickDims;
template <> struct BrickDims<2> { static constexpr int BX = 4, BY = 4, BZ = 2; };
template <> struct BrickDims<3> {
    static constexpr int BX = MFE_Q2_BRICK_X, BY = MFE_Q2_BRICK_Y, BZ = MFE_Q2_BRICK_Z;
};
template <> struct BrickDims<4> { static constexpr int BX = 2, BY = 2, BZ = 1; };
template <> struct BrickDims<5> { static constexpr int BX = 2, BY = 1, BZ = 1; };
template <> struct BrickDims<6> { static constexpr int BX = 1, BY = 1, BZ = 1; };
template <> struct BrickDims<7> { static constexpr int BX = 1, BY = 1, BZ = 1; };

// HX = false: a brick of neighbouring cells of a structured box, whose cells
// share their face nodes in the LDS node array.  HX = true: a group of the
// same number of consecutive cells of a general hexahedral mesh (cells listed
// in x, BY = BZ = 1); the LDS node array holds the group's distinct nodes
// (at most cells x n^3 slots) and a table of slots addresses each cell node.
template <int N, bool HX = false>
struct Geo {
    static constexpr int P = N - 1, N2 = N * N, N3 = N2 * N;
    static constexpr int CELLS = BrickDims<N>::BX * BrickDims<N>::BY * BrickDims<N>::BZ;
    static constexpr int BX = HX ? CELLS : BrickDims<N>::BX;
    static constexpr int BY = HX ? 1 : BrickDims<N>::BY;
    static constexpr int BZ = HX ? 1 : BrickDims<N>::BZ;
    static constexpr int CPB = BX * BY * BZ;               // cells per brick
    static constexpr int NQ = CPB * N3;                    // quadrature points per brick
    static constexpr int NT = (NQ + 63) / 64 * 64;         // threads: one per point
    static constexpr int TASKS = 3 * N2 * CPB;             // 1D lines per sweep stage
    static constexpr int TPT = (TASKS + NT - 1) / NT;      // lines per thread
    // brick node array extents (HX: the cells' node blocks stacked along z)
    static constexpr int GX = HX ? N : P * BX + 1;
    static constexpr int GY = HX ? N : P * BY + 1;
    static constexpr int GZ = HX ? N * CPB : P * BZ + 1;
    static constexpr int ROW = 3 * GX;                     // doubles in a brick node row
    static constexpr int BRICK = ROW * GY * GZ;            // doubles of the brick node array
    static constexpr int GPT = (BRICK + NT - 1) / NT;      // brick entries per thread
};

// Map the hardware block index to a brick index so that each of the 8 XCDs
// (blocks are dealt round-robin to them) works on one contiguous range of
// bricks and neighbouring bricks share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Position of the workgroup's brick and which of its cells exist.
struct BrickPos {
    int brick;
    int ex0, ey0, ez0;     // first cell (HX: ex0 = first cell of the group)
    int ncx, ncy, ncz;     // existing cells per direction
    int node0;             // global index of the brick's first node
};

template <int N, bool HX>
__device__ __forceinline__ BrickPos brick_pos(const KParams& p) {
    using G = Geo<N, HX>;
    BrickPos b;
    b.brick = xcd_remap(blockIdx.x, gridDim.x);
    if (!HX && p.colour > 0) {  // the launch holds only the bricks of one parity class
        const int c = p.colour - 1, ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
        const int mx = (p.nbx - ox + 1) / 2, my = (p.nby - oy + 1) / 2;
        const int i = b.brick % mx, r = b.brick / mx;
        b.brick = (2 * i + ox) + p.nbx * ((2 * (r % my) + oy) + p.nby * (2 * (r / my) + oz));
    }
    if constexpr (HX) {
        b.ex0 = b.brick * G::CPB;
        b.ey0 = b.ez0 = 0;
        b.ncx = min(G::CPB, p.ne - b.ex0);
        b.ncy = b.ncz = 1;
        b.node0 = 0;
        return b;
    }
    const int bx = b.brick % p.nbx, r = b.brick / p.nbx;
    const int by = r % p.nby, bz = r / p.nby;
    b.ex0 = bx * G::BX;
    b.ey0 = by * G::BY;
    b.ez0 = bz * G::BZ;
    b.ncx = min(G::BX, p.nx - b.ex0);
    b.ncy = min(G::BY, p.ny - b.ey0);
    b.ncz = min(G::BZ, p.nz - b.ez0);
    b.node0 = G::P * b.ex0 + p.Nx * (G::P * b.ey0 + p.Ny * G::P * b.ez0);
    return b;
}

// One 1D line of a sweep stage: component c, line coordinates (a, b) and
// brick-local cell lc = lx + BX*(ly + BY*lz).
struct Line {
    int c, a, b, lc, lx, ly, lz;
    bool valid;
};

template <int N, bool HX>
__device__ __forceinline__ Line line_of(int t, const BrickPos& bp) {
    using G = Geo<N, HX>;
    Line L;
    L.c = t % 3;
    const int r = t / 3;
    L.a = r % N;
    L.b = (r / N) % N;
    L.lc = r / G::N2;
    L.lx = L.lc % G::BX;
    L.ly = (L.lc / G::BX) % G::BY;
    L.lz = L.lc / (G::BX * G::BY);
    L.valid = t < G::TASKS && L.lx < bp.ncx && L.ly < bp.ncy && L.lz < bp.ncz;
    return L;
}

// The brick node array entries handled by this thread: entry
// e = tid + k*NT is (node row, offset) = (e / ROW, e % ROW) with the x-row of
// the brick's nodes contiguous, exactly as in the global vector.
template <int N, bool HX>
struct BrickMap {
    int dof[Geo<N, HX>::GPT];
    unsigned exists;   // bit k: entry k is a node of an existing cell
    unsigned face;     // bit k: that node lies on a face of the brick
};

template <int N, bool HX>
__device__ __forceinline__ BrickMap<N, HX> brick_map(const KParams& p, const BrickPos& bp) {
    using G = Geo<N, HX>;
    BrickMap<N, HX> m;
    m.exists = 0u;
    m.face = 0u;
    if constexpr (HX) {
        // entry e = (slot e / 3 of the group's node list, component e % 3);
        // every node may be shared with cells outside the group
        constexpr int MAXU = G::CPB * G::N3;
#pragma unroll
        for (int k = 0; k < G::GPT; ++k) {
            const int e = threadIdx.x + k * G::NT;
            const int u = e / 3;
            const int node = e < G::BRICK ? p.gnodes[(int64_t)bp.brick * MAXU + u] : -1;
            m.dof[k] = node >= 0 ? 3 * node + (e - 3 * u) : 0;
            if (node >= 0) m.exists |= 1u << k;
            m.face |= 1u << k;
        }
        return m;
    }
#pragma unroll
    for (int k = 0; k < G::GPT; ++k) {
        const int e = threadIdx.x + k * G::NT;
        const int row = e / G::ROW;
        const int off = e - row * G::ROW;
        const int jr = row % G::GY, kr = row / G::GY;
        const int i = off / 3;
        const bool ex = e < G::BRICK && i <= G::P * bp.ncx && jr <= G::P * bp.ncy && kr <= G::P * bp.ncz;
        m.dof[k] = 3 * (bp.node0 + p.Nx * (jr + p.Ny * kr)) + off;
        if (ex) m.exists |= 1u << k;
        if (i == 0 || i == G::GX - 1 || jr == 0 || jr == G::GY - 1 || kr == 0 || kr == G::GZ - 1)
            m.face |= 1u << k;
    }
    return m;
}

template <int N, bool HX, typename R>
__device__ __forceinline__ void brick_load(const R* __restrict__ src, const BrickMap<N, HX>& m,
                                           R (&r)[Geo<N, HX>::GPT]) {
#pragma unroll
    for (int k = 0; k < Geo<N, HX>::GPT; ++k) r[k] = (m.exists >> k & 1u) ? src[m.dof[k]] : R(0);
}

template <int N, bool HX, typename L, typename R>
__device__ __forceinline__ void brick_store(L* sBrick, const R (&r)[Geo<N, HX>::GPT]) {
#pragma unroll
    for (int k = 0; k < Geo<N, HX>::GPT; ++k) {
        const int e = threadIdx.x + k * Geo<N, HX>::NT;
        if (e < Geo<N, HX>::BRICK) sBrick[e] = (L)r[k];
    }
}

// Offset in the brick node array of node (i, j, k) of line L's cell,
// component L.c: along x-rows of the brick, or through the group's slot table
// sL (general meshes).
template <int N, bool HX>
__device__ __forceinline__ int brick_node(const Line& L, int i, int j, int k, const unsigned short* sL) {
    using G = Geo<N, HX>;
    if constexpr (HX) return 3 * sL[L.lc * G::N3 + i + N * (j + N * k)] + L.c;
    else return ((G::P * L.lz + k) * G::GY + (G::P * L.ly + j)) * G::ROW + 3 * (G::P * L.lx + i) + L.c;
}

// LDS layout.  sG holds 9 doubles per quadrature point, addressed as
// slot s of component c at point idx of cell lc:  ((lc*N3 + idx)*3 + c)*3 + s.
// The sweep stages pass their intermediate tensors through the three slots;
// after the forward sweeps slot d holds d field_c / d xi_d, before the
// backward sweeps slot d holds Q[c][d].  sV holds 3 doubles per point
// ((lc*N3 + idx)*3 + c): the values at the Gauss points, then scratch of the
// backward sweeps.
template <int N>
__device__ __forceinline__ int gofs(int lc, int idx, int c) {
    return ((lc * Geo<N>::N3 + idx) * 3 + c) * 3;
}

// ---------------------------------------------------------------------------
// Forward sweeps of one vector field whose brick nodal values are in sBrick
// (made visible by a barrier before the call).  On exit slot d of sG holds
// the reference gradient d field_c / d xi_d at every point.
// ---------------------------------------------------------------------------
template <int N, bool HX, typename R>
__device__ __forceinline__ void forward_sweeps(const BrickPos& bp, const Tables<N, R>& T, R* sG, R* sV,
                                               R* sBrick, bool clear_brick, const unsigned short* sL) {
    using G = Geo<N, HX>;
    constexpr int N2 = G::N2;
    // x: interpolate every cell's node x-rows -> slot 0 at (qx, j, k)
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        const int j = L.a, k = L.b;
        R x[N], y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] = sBrick[brick_node<N, HX>(L, i, j, k, sL)];
        apply_eo<N, false>(T.S, x, y);
        R* out = sG + gofs<N>(L.lc, N * (j + N * k), L.c);
#pragma unroll
        for (int qx = 0; qx < N; ++qx) out[9 * qx] = y[qx];
    }
    __syncthreads();
    // the brick array is free again: clear it for the backward accumulation
    if (clear_brick)
        for (int e = threadIdx.x; e < G::BRICK; e += G::NT) sBrick[e] = R(0);
    // y: slot 0 at (qx, j, k) -> slot 1 at (qx, qy, k)
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        const int base = gofs<N>(L.lc, L.a + N2 * L.b, L.c);
        R x[N], y[N];
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = sG[base + 9 * N * j];
        apply_eo<N, false>(T.S, x, y);
#pragma unroll
        for (int qy = 0; qy < N; ++qy) sG[base + 9 * N * qy + 1] = y[qy];
    }
    __syncthreads();
    // z: slot 1 -> values at the Gauss points (sV) and their z-derivative (slot 2)
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        const int base = gofs<N>(L.lc, L.a + N * L.b, L.c);
        R x[N], y[N], dz[N];
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = sG[base + 9 * N2 * k + 1];
        apply_eo<N, false>(T.S, x, y);
        apply_eo<N, true>(T.D, y, dz);
#pragma unroll
        for (int qz = 0; qz < N; ++qz) {
            sV[(base + 9 * N2 * qz) / 3] = y[qz];
            sG[base + 9 * N2 * qz + 2] = dz[qz];
        }
    }
    __syncthreads();
    // x- and y-derivatives of the values -> slots 0 and 1
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        {   // x-line at (qy, qz) = (a, b)
            const int base = gofs<N>(L.lc, N * (L.a + N * L.b), L.c);
            R x[N], y[N];
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sV[(base + 9 * l) / 3];
            apply_eo<N, true>(T.D, x, y);
#pragma unroll
            for (int qx = 0; qx < N; ++qx) sG[base + 9 * qx] = y[qx];
        }
        {   // y-line at (qx, qz) = (a, b)
            const int base = gofs<N>(L.lc, L.a + N2 * L.b, L.c);
            R x[N], y[N];
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sV[(base + 9 * N * l) / 3];
            apply_eo<N, true>(T.D, x, y);
#pragma unroll
            for (int qy = 0; qy < N; ++qy) sG[base + 9 * N * qy + 1] = y[qy];
        }
    }
    __syncthreads();
}

// The brick's summed node values (sBrick, made visible by a barrier, type R)
// added to dst (type D) with one atomic per node.  Every node takes an
// atomic, also those inside the brick that no other brick touches: plain
// stores into cache lines that neighbouring bricks update atomically cost
// more than the atomics (T2 at Q4 71 against 56 us).
template <int N, bool HX, typename D, typename R>
__device__ __forceinline__ void brick_scatter(D* __restrict__ dst, const BrickMap<N, HX>& bm, const R* sBrick) {
#pragma unroll
    for (int k = 0; k < Geo<N, HX>::GPT; ++k) {
        if (!(bm.exists >> k & 1u)) continue;
        const R val = sBrick[threadIdx.x + k * Geo<N, HX>::NT];
        unsafeAtomicAdd(dst + bm.dof[k], (D)val);
    }
}

// ---------------------------------------------------------------------------
// Backward sweeps: on entry slot d of sG holds Q[c][d] at every point (made
// visible by a barrier) and sBrick is zero.  Adds
// sum_q sum_d Q[c][d](q) dN_a/dxi_d(q) of every cell to dst (sweeps in R,
// dst of type D).  The cells' contributions are summed in LDS, then every
// node of the brick is added to dst with an atomic.
// ---------------------------------------------------------------------------
template <int N, bool HX, typename R, typename D>
__device__ __forceinline__ void backward_sweeps(D* __restrict__ dst, const BrickPos& bp, const BrickMap<N, HX>& bm,
                                                const Tables<N, R>& T, R* sG, R* sV, R* sBrick,
                                                const unsigned short* sL) {
    using G = Geo<N, HX>;
    constexpr int N2 = G::N2;
    // transposed x- and y-derivatives, in place in slots 0 and 1
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        {
            const int base = gofs<N>(L.lc, N * (L.a + N * L.b), L.c);
            R x[N], y[N];
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sG[base + 9 * l];
            apply_eo<N, true>(T.Dt, x, y);
#pragma unroll
            for (int qx = 0; qx < N; ++qx) sG[base + 9 * qx] = y[qx];
        }
        {
            const int base = gofs<N>(L.lc, L.a + N2 * L.b, L.c);
            R x[N], y[N];
#pragma unroll
            for (int l = 0; l < N; ++l) x[l] = sG[base + 9 * N * l + 1];
            apply_eo<N, true>(T.Dt, x, y);
#pragma unroll
            for (int qy = 0; qy < N; ++qy) sG[base + 9 * N * qy + 1] = y[qy];
        }
    }
    __syncthreads();
    // transposed z-derivative, sum of the three directions, transposed
    // z-interpolation -> sV at (qx, qy, k)
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        const int base = gofs<N>(L.lc, L.a + N * L.b, L.c);
        R x[N], y[N], z[N];
#pragma unroll
        for (int l = 0; l < N; ++l) x[l] = sG[base + 9 * N2 * l + 2];
        apply_eo<N, true>(T.Dt, x, y);
#pragma unroll
        for (int qz = 0; qz < N; ++qz) y[qz] += sG[base + 9 * N2 * qz] + sG[base + 9 * N2 * qz + 1];
        apply_eo<N, false>(T.St, y, z);
#pragma unroll
        for (int k = 0; k < N; ++k) sV[(base + 9 * N2 * k) / 3] = z[k];
    }
    __syncthreads();
    // transposed y-interpolation: sV at (qx, qy, k) -> slot 0 at (qx, j, k)
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        const int base = gofs<N>(L.lc, L.a + N2 * L.b, L.c);
        R x[N], y[N];
#pragma unroll
        for (int qy = 0; qy < N; ++qy) x[qy] = sV[(base + 9 * N * qy) / 3];
        apply_eo<N, false>(T.St, x, y);
#pragma unroll
        for (int j = 0; j < N; ++j) sG[base + 9 * N * j] = y[j];
    }
    __syncthreads();
    // transposed x-interpolation, summed into the brick's nodes in LDS
#pragma unroll
    for (int it = 0; it < G::TPT; ++it) {
        const Line L = line_of<N, HX>(threadIdx.x + it * G::NT, bp);
        if (!L.valid) continue;
        const int j = L.a, k = L.b;
        const int base = gofs<N>(L.lc, N * (j + N * k), L.c);
        R x[N], y[N];
#pragma unroll
        for (int qx = 0; qx < N; ++qx) x[qx] = sG[base + 9 * qx];
        apply_eo<N, false>(T.St, x, y);
#pragma unroll
        for (int i = 0; i < N; ++i) atomicAdd(sBrick + brick_node<N, HX>(L, i, j, k, sL), y[i]);
    }
    __syncthreads();
    brick_scatter<N, HX>(dst, bm, sBrick);
}

// ---------------------------------------------------------------------------
// Sweeps of the w field on the matrix cores (MFE_SF_BF16: SW = 1,
// MFE_SF_BF16X3: SW = 3).  A sweep stage is a batch of small dense products
// out[q] = sum_k M[q][k] in[k], one per 1D line, done as 16 x 16 x 16 bf16
// matrix-core products with FP32 accumulation.  A column of the 16 x 16 B
// operand stacks LPC = floor(16 / n) lines (rows j n .. j n + n - 1 hold line
// j), and A is the block-diagonal matrix of LPC copies of M, so one product
// handles 16 LPC lines and the C operand holds the outputs in the same row
// layout; tiles of 16 LPC lines are dealt to the wavefronts.  With SW = 3
// both operands are split into three bf16 pieces, x = x0 + x1 + x2 (8
// significant bits each, so the FP32 value exactly), and the six products of
// total order <= 2 are accumulated, smallest first: about FP32 accuracy.
// With SW = 1 a single bf16 product (unit roundoff 2^-9).  The LDS layouts and
// the addresses of every stage are those of the vector-ALU sweeps.
// ---------------------------------------------------------------------------
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(short h) { return __uint_as_float((uint32_t)(unsigned short)h << 16); }

// x = p[0] + ... + p[NP-1], each piece rounded to the nearest bf16
template <int NP>
__device__ __forceinline__ void split_bf16(float x, short (&p)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        p[i] = bf16_rne(x);
        if (i + 1 < NP) x -= bf16_value(p[i]);
    }
}

// c += sum over i + j < NP of A_i B_j, products of the highest order first
template <int NP>
__device__ __forceinline__ f32x4_t mfma_pieces(const bf16x4_t (&a)[NP], const bf16x4_t (&b)[NP], f32x4_t c) {
#pragma unroll
    for (int o = NP - 1; o >= 0; --o)
#pragma unroll
        for (int i = 0; i <= o; ++i) c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[o - i], c, 0, 0, 0);
    return c;
}

// this lane's pieces of the block-diagonal A operand: lane l holds
// A[l % 16][4 (l / 16) + r], i.e. M[i % n][k % n] when rows i and k belong to
// the same stacked line (i / n == k / n < LPC), else 0
template <int N, int NP, typename MatFn>
__device__ __forceinline__ void a_fragment(MatFn mat, bf16x4_t (&a)[NP]) {
    constexpr int LPC = 16 / N;
    const int l = threadIdx.x & 63, i = l & 15, ji = i / N;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = 4 * (l >> 4) + r, jk = k / N;
        short pc[NP];
        split_bf16<NP>(ji == jk && ji < LPC ? mat(i - N * ji, k - N * jk) : 0.0f, pc);
#pragma unroll
        for (int p = 0; p < NP; ++p) a[p][r] = pc[p];
    }
}

// the B pieces of one input: rows 4 (l / 16) + r of this lane's column
template <int N, int NP, typename In>
__device__ __forceinline__ void b_fragment(In in, const Line& L0, const Line& L1, int j0, bf16x4_t (&b)[NP]) {
    constexpr int LPC = 16 / N;
    const int r0 = 4 * ((threadIdx.x & 63) >> 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = (r0 + r) / N, k = r0 + r - N * j;
        const Line& L = j == j0 ? L0 : L1;
        short pc[NP];
        split_bf16<NP>(j < LPC && L.valid ? in(L, k) : 0.0f, pc);
#pragma unroll
        for (int p = 0; p < NP; ++p) b[p][r] = pc[p];
    }
}

template <int N, typename Out>
__device__ __forceinline__ void c_store(Out out, const Line& L0, const Line& L1, int j0, const f32x4_t& c) {
    constexpr int LPC = 16 / N;
    const int r0 = 4 * ((threadIdx.x & 63) >> 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = (r0 + r) / N, q = r0 + r - N * j;
        const Line& L = j == j0 ? L0 : L1;
        if (j < LPC && L.valid) out(L, q, c[r]);
    }
}

enum { MF_ONE = 0, MF_SUM = 1, MF_DUAL = 2 };

// One stage over every line L of the brick (in*(L, k) read for k < n, out*(L,
// q) written for q < n):
//   MF_ONE   out1 = M1 in1
//   MF_SUM   out1 = M1 in1 + M2 in2
//   MF_DUAL  out1 = M1 in1, out2 = M2 in1
// A lane's four rows span at most two stacked lines (n >= 2), L0 and L1; the
// products run with every lane of the wavefront active.
template <int N, bool HX, int NP, int KIND, typename M1, typename I1, typename M2, typename I2, typename O1,
          typename O2>
__device__ __forceinline__ void mfma_stage(const BrickPos& bp, M1 mat1, I1 in1, M2 mat2, I2 in2, O1 out1, O2 out2) {
    using G = Geo<N, HX>;
    constexpr int LPC = 16 / N, NW = G::NT / 64, TILES = (G::TASKS + 16 * LPC - 1) / (16 * LPC);
    bf16x4_t a1[NP], a2[NP];
    a_fragment<N, NP>(mat1, a1);
    if constexpr (KIND != MF_ONE) a_fragment<N, NP>(mat2, a2);
    const int l = threadIdx.x & 63, j0 = 4 * (l >> 4) / N;
    for (int tile = threadIdx.x >> 6; tile < TILES; tile += NW) {
        const int t0 = (tile * 16 + (l & 15)) * LPC + j0;
        const Line L0 = line_of<N, HX>(t0, bp), L1 = line_of<N, HX>(t0 + 1, bp);
        bf16x4_t b1[NP];
        b_fragment<N, NP>(in1, L0, L1, j0, b1);
        f32x4_t c1 = {0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (KIND == MF_SUM) {
            bf16x4_t b2[NP];
            b_fragment<N, NP>(in2, L0, L1, j0, b2);
            c1 = mfma_pieces<NP>(a2, b2, c1);
        }
        c1 = mfma_pieces<NP>(a1, b1, c1);
        if constexpr (KIND == MF_DUAL) {
            f32x4_t c2 = {0.0f, 0.0f, 0.0f, 0.0f};
            c2 = mfma_pieces<NP>(a2, b1, c2);
            c_store<N>(out2, L0, L1, j0, c2);
        }
        c_store<N>(out1, L0, L1, j0, c1);
    }
}

// Dense 1D matrices of the sweeps (row = output index): S, the collocated
// derivative D, D S, and the transposes St, Dt, St Dt.
template <int N>
struct MfmaMats {
    float S[N][N], D[N][N], DS[N][N], St[N][N], Dt[N][N], StDt[N][N];
};

// the matrix-core counterparts of forward_sweeps / backward_sweeps for the
// w field (FP32 in LDS)
template <int N, bool HX, int NP>
__device__ __forceinline__ void forward_sweeps_mfma(const BrickPos& bp, const MfmaMats<N>& MM, float* sG, float* sV,
                                                    float* sBrick, const unsigned short* sL) {
    using G = Geo<N, HX>;
    constexpr int N2 = G::N2;
    auto none = [](int, int) { return 0.0f; };
    auto no_in = [](const Line&, int) { return 0.0f; };
    auto no_out = [](const Line&, int, float) {};
    auto S = [&](int q, int k) { return MM.S[q][k]; };
    auto D = [&](int q, int k) { return MM.D[q][k]; };
    auto DS = [&](int q, int k) { return MM.DS[q][k]; };
    // x: node x-rows -> slot 0 at (qx, j, k)
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, S, [&](const Line& L, int k) { return sBrick[brick_node<N, HX>(L, k, L.a, L.b, sL)]; }, none, no_in,
        [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, N * (L.a + N * L.b), L.c) + 9 * q] = v; }, no_out);
    __syncthreads();
    for (int e = threadIdx.x; e < G::BRICK; e += G::NT) sBrick[e] = 0.0f;  // for the backward accumulation
    // y: slot 0 -> slot 1
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, S, [&](const Line& L, int k) { return sG[gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * k]; }, none, no_in,
        [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * q + 1] = v; }, no_out);
    __syncthreads();
    // z: slot 1 -> values (S, into sV) and their z-derivative (D S, slot 2)
    mfma_stage<N, HX, NP, MF_DUAL>(
        bp, S, [&](const Line& L, int k) { return sG[gofs<N>(L.lc, L.a + N * L.b, L.c) + 9 * N2 * k + 1]; }, DS,
        no_in, [&](const Line& L, int q, float v) { sV[(gofs<N>(L.lc, L.a + N * L.b, L.c) + 9 * N2 * q) / 3] = v; },
        [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, L.a + N * L.b, L.c) + 9 * N2 * q + 2] = v; });
    __syncthreads();
    // x- and y-derivatives of the values -> slots 0 and 1
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, D, [&](const Line& L, int k) { return sV[(gofs<N>(L.lc, N * (L.a + N * L.b), L.c) + 9 * k) / 3]; },
        none, no_in,
        [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, N * (L.a + N * L.b), L.c) + 9 * q] = v; }, no_out);
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, D, [&](const Line& L, int k) { return sV[(gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * k) / 3]; },
        none, no_in,
        [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * q + 1] = v; }, no_out);
    __syncthreads();
}

template <int N, bool HX, int NP>
__device__ __forceinline__ void backward_sweeps_mfma(float* __restrict__ dst, const BrickPos& bp,
                                                     const BrickMap<N, HX>& bm, const MfmaMats<N>& MM, float* sG,
                                                     float* sV, float* sBrick, const unsigned short* sL) {
    using G = Geo<N, HX>;
    constexpr int N2 = G::N2;
    auto none = [](int, int) { return 0.0f; };
    auto no_in = [](const Line&, int) { return 0.0f; };
    auto no_out = [](const Line&, int, float) {};
    auto St = [&](int q, int k) { return MM.St[q][k]; };
    auto Dt = [&](int q, int k) { return MM.Dt[q][k]; };
    auto StDt = [&](int q, int k) { return MM.StDt[q][k]; };
    // transposed x- and y-derivatives, in place in slots 0 and 1 (a column's
    // lines are read into registers before the product and written after it,
    // all by one wavefront)
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, Dt, [&](const Line& L, int k) { return sG[gofs<N>(L.lc, N * (L.a + N * L.b), L.c) + 9 * k]; }, none,
        no_in, [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, N * (L.a + N * L.b), L.c) + 9 * q] = v; },
        no_out);
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, Dt, [&](const Line& L, int k) { return sG[gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * k + 1]; }, none,
        no_in, [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * q + 1] = v; },
        no_out);
    __syncthreads();
    // z: St Dt (slot 2) + St (slot 0 + slot 1) -> sV at (qx, qy, k)
    mfma_stage<N, HX, NP, MF_SUM>(
        bp, StDt, [&](const Line& L, int k) { return sG[gofs<N>(L.lc, L.a + N * L.b, L.c) + 9 * N2 * k + 2]; }, St,
        [&](const Line& L, int k) {
            const int b = gofs<N>(L.lc, L.a + N * L.b, L.c) + 9 * N2 * k;
            return sG[b] + sG[b + 1];
        },
        [&](const Line& L, int q, float v) { sV[(gofs<N>(L.lc, L.a + N * L.b, L.c) + 9 * N2 * q) / 3] = v; },
        no_out);
    __syncthreads();
    // transposed y-interpolation: sV at (qx, qy, k) -> slot 0 at (qx, j, k)
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, St, [&](const Line& L, int k) { return sV[(gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * k) / 3]; },
        none, no_in,
        [&](const Line& L, int q, float v) { sG[gofs<N>(L.lc, L.a + N2 * L.b, L.c) + 9 * N * q] = v; }, no_out);
    __syncthreads();
    // transposed x-interpolation, summed into the brick's nodes in LDS
    mfma_stage<N, HX, NP, MF_ONE>(
        bp, St, [&](const Line& L, int k) { return sG[gofs<N>(L.lc, N * (L.a + N * L.b), L.c) + 9 * k]; }, none,
        no_in,
        [&](const Line& L, int q, float v) { atomicAdd(sBrick + brick_node<N, HX>(L, q, L.a, L.b, sL), v); },
        no_out);
    __syncthreads();
    brick_scatter<N, HX>(dst, bm, sBrick);
}

template <int N, typename R>
__device__ __forceinline__ void load_slots(const R* sG, int tid, R g[3][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[c][d] = sG[(tid * 3 + c) * 3 + d];
}

template <int N, typename R>
__device__ __forceinline__ void store_slots(R* sG, int tid, const R g[3][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) sG[(tid * 3 + c) * 3 + d] = g[c][d];
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
    static constexpr bool split = MODE == MODE_APPLY_OTF_AD_SPLIT || MODE == MODE_RESIDUAL_SPLIT ||
                                  MODE == MODE_BUILD_T4_SPLIT || MODE == MODE_ENERGY_SPLIT;
    static constexpr bool otf_ad = MODE == MODE_APPLY_OTF_AD || MODE == MODE_APPLY_OTF_AD_SPLIT;
    static constexpr bool residual = MODE == MODE_RESIDUAL || MODE == MODE_RESIDUAL_SPLIT;
    static constexpr bool build_t4 = MODE == MODE_BUILD_T4 || MODE == MODE_BUILD_T4_SPLIT;
    static constexpr bool energy = MODE == MODE_ENERGY || MODE == MODE_ENERGY_SPLIT;
    static constexpr bool fwd_u = MODE == MODE_APPLY_OTF || MODE == MODE_APPLY_OTF_GEOM || otf_ad || residual ||
                                  MODE == MODE_STATE || MODE == MODE_BUILD_T2 || build_t4 || energy;
    static constexpr bool fwd_w = MODE == MODE_APPLY_OTF || MODE == MODE_APPLY_OTF_GEOM || otf_ad ||
                                  MODE == MODE_APPLY_T2 || MODE == MODE_APPLY_T4;
    static constexpr bool backward = fwd_w || residual;
    static constexpr bool vertex_geom = MODE == MODE_APPLY_OTF || otf_ad || residual || MODE == MODE_STATE ||
                                        MODE == MODE_BUILD_GEOM || MODE == MODE_BUILD_T2 || build_t4 || energy;
    static constexpr int cache_fields = MODE == MODE_APPLY_OTF_GEOM ? kGeomFields
                                      : MODE == MODE_APPLY_T2       ? kT2Fields
                                      : MODE == MODE_APPLY_T4       ? kT4Fields
                                                                    : 0;
};

#ifndef MFE_MIN_WAVES_PER_EU
#define MFE_MIN_WAVES_PER_EU 1
#endif
// Vector and cache element types of a launch: R is the type of w, v and the
// T2/T4 caches; the u field, the geometry and the per-point kinematics are
// always FP64.  The sweeps of the w field run in R for the cached strategies
// and in FP64 for the on-the-fly ones: they are bound by their arithmetic,
// and without packed FP32 arithmetic (which the build disables) an FP32
// vector instruction costs what an FP64 one does, so FP32 sweeps would only
// add conversions around the FP64 point-wise response.
template <typename R>
__device__ __forceinline__ const R* w_of(const KParams& p) {
    if constexpr (std::is_same_v<R, float>) return p.w32; else return p.w;
}
template <typename R>
__device__ __forceinline__ R* v_of(const KParams& p) {
    if constexpr (std::is_same_v<R, float>) return p.v32; else return p.v;
}
template <typename R>
__device__ __forceinline__ const R* cache_of(const KParams& p) {
    if constexpr (std::is_same_v<R, float>) return p.cache32; else return p.cache;
}
template <typename R>
__device__ __forceinline__ R* cache_out_of(const KParams& p) {
    if constexpr (std::is_same_v<R, float>) return p.cache_out32; else return p.cache_out;
}

// SW: sweeps of the w field on the vector ALUs (0) or on the matrix cores
// with one (1) or three (3) bf16 pieces per operand (R = float only).
template <int N, int MODE, typename R, bool HX, int SW = 0>
__global__ __launch_bounds__((Geo<N, HX>::NT)) __attribute__((amdgpu_waves_per_eu(MFE_MIN_WAVES_PER_EU)))
void cell_kernel(const KParams p, const Tables<N> T, const Tables<N, R> TR, const MfmaMats<N> MM) {
    static_assert(SW == 0 || std::is_same_v<R, float>, "matrix-core sweeps take FP32 operands");
    using G = Geo<N, HX>;
    constexpr int N3 = G::N3;
    using MI = ModeInfo<MODE>;
    // LDS element type: FP64 whenever the u field is swept, else R
    using LT = std::conditional_t<MI::fwd_u, double, R>;
    // type of the cached per-point data read by an apply
    constexpr bool cached_r = MODE == MODE_APPLY_T2 || MODE == MODE_APPLY_T4;
    using CT = std::conditional_t<cached_r, R, double>;
    // type of the sweeps of the w field (FP64 in the on-the-fly modes, whose
    // LDS arrays are FP64 for the u field anyway)
    using WT = std::conditional_t<MI::fwd_u && SW == 0, double, R>;
    __shared__ LT sG[G::NQ * 9];
    __shared__ LT sV[G::NQ * 3];
    __shared__ LT sBrick[G::BRICK];
    __shared__ double sEdge[G::CPB * 36];
    __shared__ unsigned short sL[HX ? G::CPB * N3 : 1];

    const BrickPos bp = brick_pos<N, HX>(p);
    const BrickMap<N, HX> bm = brick_map<N, HX>(p, bp);
    const int tid = threadIdx.x;
    if constexpr (HX) {  // slot table of the group's cell nodes (read after the first barrier)
        for (int t = tid; t < bp.ncx * N3; t += G::NT) sL[t] = p.lidx[(int64_t)bp.ex0 * N3 + t];
    }
    // the quadrature point of this thread
    const int lc = tid / N3;
    const int q = tid - lc * N3;
    const int lx = lc % G::BX, ly = (lc / G::BX) % G::BY, lz = lc / (G::BX * G::BY);
    const bool active = lc < G::CPB && lx < bp.ncx && ly < bp.ncy && lz < bp.ncz;
    const int qx = q % N, qy = (q / N) % N, qz = q / G::N2;
    // per-point caches are brick-major: the CF fields of a brick's points are one
    // contiguous block, field f of this thread's point at cidx(f)
    constexpr int CF = MODE == MODE_BUILD_GEOM ? kGeomFields
                     : MODE == MODE_BUILD_T2   ? kT2Fields
                     : MI::build_t4            ? kT4Fields
                                               : (MI::cache_fields > 0 ? MI::cache_fields : 1);
    const int64_t cbase = (int64_t)bp.brick * CF * G::NQ + tid;
    auto cidx = [&](int f) { return cbase + (int64_t)f * G::NQ; };

    // issue the global loads early: nodal values of the fields, per-point data
    double ub[G::GPT];
    R wb[G::GPT];
    if constexpr (MI::fwd_u) brick_load<N, HX>(p.u, bm, ub);
    if constexpr (MI::fwd_w) brick_load<N, HX>(w_of<R>(p), bm, wb);
    constexpr int NCF = MI::cache_fields > 0 ? MI::cache_fields : 1;
    // Fields read before the sweeps (the rest right before their first use).
    // Issuing every load early hides its latency behind the sweeps; with one
    // 7^3-point cell per workgroup (p = 6) the FP64 T2/T4 fields held through
    // the sweeps cost more occupancy than that hides, and those applies are
    // 16-20% faster reading them late.  Q2 and Q4 are 5-10% faster reading
    // early.
    constexpr int kEarly = (N >= 7 && cached_r && std::is_same_v<CT, double>) ? 0 : MI::cache_fields;
    CT cf[NCF];
    if constexpr (MI::cache_fields > 0) {
        const CT* cache = cached_r ? (const CT*)cache_of<R>(p) : (const CT*)p.cache;
#pragma unroll
        // read once per apply: non-temporal, so the streamed cache does not
        // evict the gathered and scattered vectors from the caches
        for (int f = 0; f < kEarly; ++f) cf[f] = active ? __builtin_nontemporal_load(cache + cidx(f)) : CT(0);
    }
    // the remaining fields, read right before their first use
    auto load_late = [&]() {
        if constexpr (kEarly < MI::cache_fields) {
            const CT* cache = cached_r ? (const CT*)cache_of<R>(p) : (const CT*)p.cache;
#pragma unroll
            for (int f = kEarly; f < MI::cache_fields; ++f)
                cf[f] = active ? __builtin_nontemporal_load(cache + cidx(f)) : CT(0);
        }
    };

    if constexpr (MI::vertex_geom) {
        // the 12 edge vectors of every cell's trilinear map, one thread per
        // (cell, edge) for its three components (fewer wavefronts spend
        // index arithmetic here than with one thread per component)
        for (int t = tid; t < G::CPB * 12; t += G::NT) {
            const int c = t / 12;
            const int edge = t - 12 * c;
            const int cx = c % G::BX, cy = (c / G::BX) % G::BY, cz = c / (G::BX * G::BY);
            if (cx >= bp.ncx || cy >= bp.ncy || cz >= bp.ncz) continue;
            const int dir = edge >> 2, a = edge & 3;
            int v0;  // edge = 4*dir + a; its end points differ in bit `dir`
            if (dir == 0) v0 = ((a & 1) << 1) | ((a >> 1) << 2);
            else if (dir == 1) v0 = (a & 1) | ((a >> 1) << 2);
            else v0 = (a & 1) | ((a >> 1) << 1);
            const int v1 = v0 | (1 << dir);
            int vid0, vid1;
            if constexpr (HX) {
                const int64_t cell = bp.ex0 + cx;
                vid0 = p.ev[8 * cell + v0];
                vid1 = p.ev[8 * cell + v1];
            } else {
                const int ex = bp.ex0 + cx, ey = bp.ey0 + cy, ez = bp.ez0 + cz;
                vid0 = (ex + (v0 & 1)) + (p.nx + 1) * ((ey + ((v0 >> 1) & 1)) + (p.ny + 1) * (ez + (v0 >> 2)));
                vid1 = (ex + (v1 & 1)) + (p.nx + 1) * ((ey + ((v1 >> 1) & 1)) + (p.ny + 1) * (ez + (v1 >> 2)));
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) sEdge[36 * c + 3 * edge + d] = p.verts[3 * vid1 + d] - p.verts[3 * vid0 + d];
        }
    }

    double mu = p.mu, lam = p.lam;
    if (p.cell_mat != nullptr && active) {
        const int cell = HX ? bp.ex0 + lc : (bp.ex0 + lx) + p.nx * ((bp.ey0 + ly) + p.ny * (bp.ez0 + lz));
        mu = p.cell_mat[2 * cell];
        lam = p.cell_mat[2 * cell + 1];
    }

    if constexpr (MODE == MODE_BUILD_GEOM) {
        __syncthreads();
        if (active) {
            double Jg[3][3], Jinv[3][3], det;
            jacobian_from_edges(sEdge + lc * 36, T.qp[qx], T.qp[qy], T.qp[qz], Jg);
            inverse3(Jg, Jinv, det);
            const double JxW = det * T.qw[qx] * T.qw[qy] * T.qw[qz];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) p.cache_out[cidx(3 * i + j)] = Jinv[i][j];
            p.cache_out[cidx(9)] = JxW;
        }
        return;
    }

    // ---------------- field u: gradients, geometry, kinematics
    double Jinv[3][3] = {}, JxW = 0.0;
    Kin kin = {};
    double F[3][3] = {};
    double du[3][3] = {};
    if constexpr (MI::fwd_u) {
        brick_store<N, HX>(reinterpret_cast<double*>(sBrick), ub);
        __syncthreads();
        forward_sweeps<N, HX>(bp, T, reinterpret_cast<double*>(sG), reinterpret_cast<double*>(sV),
                              reinterpret_cast<double*>(sBrick), !MI::fwd_w, sL);
        if (active) {
            load_slots<N>(reinterpret_cast<const double*>(sG), tid, du);
            if constexpr (MODE == MODE_APPLY_OTF_GEOM) {
                load_late();
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Jinv[i][j] = cf[3 * i + j];
                JxW = cf[9];
            } else {
                double Jg[3][3], det;
                jacobian_from_edges(sEdge + lc * 36, T.qp[qx], T.qp[qy], T.qp[qz], Jg);
                inverse3(Jg, Jinv, det);
                JxW = det * T.qw[qx] * T.qw[qy] * T.qw[qz];
            }
            if constexpr (!MI::otf_ad) kinematics(du, Jinv, F, kin);
        }
    }

    if constexpr (MODE == MODE_STATE) {
        if (active && !(kin.J > 0.0)) atomicOr(p.flag, 1);
        return;
    }

    if constexpr (MI::energy) {
        // stored energy of the law, summed over the brick's points in a fixed
        // order (one partial per brick)
        __shared__ double sRed[G::NT / 64];
        double e = 0.0;
        if (active) e = (MI::split ? energy_split(F, kin, mu, lam) : energy_nh(F, kin, mu, lam)) * JxW;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
        if ((tid & 63) == 0) sRed[tid >> 6] = e;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < G::NT / 64; ++w) sum += sRed[w];
            p.v[bp.brick] = sum;
        }
        return;
    }

    if constexpr (MODE == MODE_BUILD_T2 || MI::build_t4) {
        if (active) {
            R* out = cache_out_of<R>(p);
            double M[3][3], tau[6];
            spatial_map(Jinv, kin, M);
            if constexpr (MI::split) kirchhoff_split_voigt(F, kin, mu, lam, JxW, tau);
            else kirchhoff_voigt(F, kin, mu, lam, JxW, tau);
            if constexpr (MODE == MODE_BUILD_T2) {
#pragma unroll
                for (int i = 0; i < 9; ++i) out[cidx(i)] = (R)M[i / 3][i % 3];
#pragma unroll
                for (int i = 0; i < 6; ++i) out[cidx(9 + i)] = (R)tau[i];
                out[cidx(15)] = (R)(2.0 * lam * JxW);
                out[cidx(16)] = (R)(2.0 * (mu - 2.0 * lam * kin.lJ) * JxW);
            } else {
                double D21[21];
                if constexpr (MI::split) spatial_tangent_split_voigt(F, mu, lam, JxW, D21);
                else spatial_tangent_voigt(kin, mu, lam, JxW, D21);
#pragma unroll
                for (int i = 0; i < 21; ++i) out[cidx(i)] = (R)D21[i];
#pragma unroll
                for (int i = 0; i < 6; ++i) out[cidx(21 + i)] = (R)tau[i];
#pragma unroll
                for (int i = 0; i < 9; ++i) out[cidx(27 + i)] = (R)M[i / 3][i % 3];
            }
        }
        return;
    }

    // ---------------- field w and the point-wise product
    WT* gW = reinterpret_cast<WT*>(sG);
    WT* vW = reinterpret_cast<WT*>(sV);
    WT* bW = reinterpret_cast<WT*>(sBrick);
    const auto& TW = [&]() -> const Tables<N, WT>& {
        if constexpr (std::is_same_v<WT, R>) return TR; else return T;
    }();
    WT Q[3][3] = {};
    if constexpr (MI::fwd_w) {
        // sBrick was last read before the forward sweeps' first barrier
        brick_store<N, HX>(bW, wb);
        __syncthreads();
        if constexpr (SW > 0) forward_sweeps_mfma<N, HX, SW>(bp, MM, gW, vW, bW, sL);
        else forward_sweeps<N, HX>(bp, TW, gW, vW, bW, true, sL);
        if constexpr (MODE != MODE_APPLY_OTF_GEOM) load_late();
        if (active) {
            WT dwr[3][3];
            load_slots<N>(gW, tid, dwr);
            if constexpr (MODE == MODE_APPLY_OTF || MODE == MODE_APPLY_OTF_GEOM || MI::otf_ad) {
                // the point-wise response is evaluated in FP64
                double dw[3][3], Qd[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) dw[i][j] = dwr[i][j];
                if constexpr (MODE == MODE_APPLY_OTF_AD) pointwise_otf_ad(du, dw, Jinv, mu, lam, JxW, Qd);
                else if constexpr (MODE == MODE_APPLY_OTF_AD_SPLIT)
                    pointwise_otf_ad_split(du, dw, Jinv, mu, lam, JxW, Qd);
                else pointwise_otf(dw, Jinv, kin, mu, lam, JxW, Qd);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) Q[i][j] = (WT)Qd[i][j];
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
    } else if constexpr (MI::residual) {
        static_assert(std::is_same_v<R, double>, "the residual is FP64 only");
        if (active) {
            if constexpr (MI::split) pointwise_piola_split(F, kin, mu, lam, Jinv, JxW, Q);
            else pointwise_piola(F, kin, mu, lam, Jinv, JxW, Q);
        }
    }

    if constexpr (MI::backward) {
        // each thread overwrites only its own point's slots, which only it read
        if (active) store_slots<N>(gW, tid, Q);
        __syncthreads();
        if constexpr (SW > 0) backward_sweeps_mfma<N, HX, SW>(v_of<R>(p), bp, bm, MM, gW, vW, bW, sL);
        else backward_sweeps<N, HX>(v_of<R>(p), bp, bm, TW, gW, vW, bW, sL);
    }
}

// ---------------------------------------------------------------------------
// Diagonal of the tangent, for the Jacobi / Chebyshev smoothers of the
// multigrid-preconditioned CG (Sec. 2.3), from the second-order cache in the
// current configuration: with g = grad N_a = (dN_a/dxi) M,
//   K_(a,i),(a,i) = sum_q [ c1 g_i^2 + c2 (|g|^2 + g_i^2) / 2 + g tau g ].
// One thread per (cell, node) of a brick; contributions of all cells are
// added with atomics.
// ---------------------------------------------------------------------------
template <int N, bool HX>
__global__ __launch_bounds__((Geo<N, HX>::NT)) void diag_kernel(const KParams p, const DiagTables T,
                                                          double* __restrict__ diag) {
    using G = Geo<N, HX>;
    constexpr int N3 = G::N3, P = G::P;
    __shared__ double sS[N * N], sSd[N * N];
    const int tid = threadIdx.x;
    if (tid < N * N) {
        sS[tid] = T.S[tid / N][tid % N];
        sSd[tid] = T.Sd[tid / N][tid % N];
    }
    __syncthreads();
    const BrickPos bp = brick_pos<N, HX>(p);
    const int lc = tid / N3;
    const int a = tid - lc * N3;
    const int lx = lc % G::BX, ly = (lc / G::BX) % G::BY, lz = lc / (G::BX * G::BY);
    if (!(lc < G::CPB && lx < bp.ncx && ly < bp.ncy && lz < bp.ncz)) return;
    const int i = a % N, j = (a / N) % N, k = a / G::N2;
    const double* cache = p.cache + (int64_t)bp.brick * kT2Fields * G::NQ + lc * N3;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < N3; ++q) {
        const int qx = q % N, qy = (q / N) % N, qz = q / G::N2;
        const double Si = sS[qx * N + i], Sj = sS[qy * N + j], Sk = sS[qz * N + k];
        const double d0 = sSd[qx * N + i] * Sj * Sk;
        const double d1 = Si * sSd[qy * N + j] * Sk;
        const double d2 = Si * Sj * sSd[qz * N + k];
        double M[9], t[6];
#pragma unroll
        for (int f = 0; f < 9; ++f) M[f] = cache[f * G::NQ + q];
#pragma unroll
        for (int f = 0; f < 6; ++f) t[f] = cache[(9 + f) * G::NQ + q];
        const double c1 = cache[15 * G::NQ + q], c2 = cache[16 * G::NQ + q];
        double g[3];
#pragma unroll
        for (int n = 0; n < 3; ++n) g[n] = fma(d0, M[n], fma(d1, M[3 + n], d2 * M[6 + n]));
        const double gg = fma(g[0], g[0], fma(g[1], g[1], g[2] * g[2]));
        const double gtg = t[0] * g[0] * g[0] + t[1] * g[1] * g[1] + t[2] * g[2] * g[2] +
                           2.0 * (t[3] * g[1] * g[2] + t[4] * g[0] * g[2] + t[5] * g[0] * g[1]);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += c1 * g[c] * g[c] + 0.5 * c2 * (gg + g[c] * g[c]) + gtg;
    }
    const int node = HX ? p.conn[(int64_t)(bp.ex0 + lc) * N3 + a]
                        : (P * (bp.ex0 + lx) + i) + p.Nx * ((P * (bp.ey0 + ly) + j) + p.Ny * (P * (bp.ez0 + lz) + k));
#pragma unroll
    for (int c = 0; c < 3; ++c) unsafeAtomicAdd(diag + 3 * node + c, acc[c]);
}

// ---------------------------------------------------------------------------
// Dense tangent of a small mesh (the coarsest multigrid level) from the
// second-order cache: with g^a = (dN_a/dxi) M at a point,
//   K_(a,i),(b,j) = sum_q [ c1 g^a_i g^b_j + c2/2 (delta_ij g^a.g^b + g^a_j g^b_i)
//                           + delta_ij g^a tau g^b ],
// the T2 point-wise product applied to w = N_b e_j and tested with N_a e_i.
// One workgroup per cell, one thread per pair of local nodes; entries are
// added into A (n x n, row-major, dof = 3 node + component) with atomics.
// ---------------------------------------------------------------------------
template <int N, bool HX>
__global__ __launch_bounds__(256) void dense_kernel(const KParams p, const DiagTables T, double* __restrict__ A,
                                                    int64_t n) {
    using G = Geo<N, HX>;
    constexpr int N3 = G::N3, P = G::P;
    __shared__ double sS[N * N], sSd[N * N];
    const int tid = threadIdx.x;
    if (tid < N * N) {
        sS[tid] = T.S[tid / N][tid % N];
        sSd[tid] = T.Sd[tid / N][tid % N];
    }
    __syncthreads();
    const int cell = blockIdx.x;
    int ex = 0, ey = 0, ez = 0, brick, lc;
    if constexpr (HX) {
        brick = cell / G::CPB;
        lc = cell - brick * G::CPB;
    } else {
        ex = cell % p.nx;
        ey = (cell / p.nx) % p.ny;
        ez = cell / (p.nx * p.ny);
        const int bx = ex / G::BX, by = ey / G::BY, bz = ez / G::BZ;
        brick = bx + p.nbx * (by + p.nby * bz);
        lc = (ex - bx * G::BX) + G::BX * ((ey - by * G::BY) + G::BY * (ez - bz * G::BZ));
    }
    const double* cache = p.cache + (int64_t)brick * kT2Fields * G::NQ + lc * N3;
    for (int pr = tid; pr < N3 * N3; pr += blockDim.x) {
        const int a = pr / N3, b = pr - a * N3;
        const int ai = a % N, aj = (a / N) % N, ak = a / G::N2;
        const int bi = b % N, bj = (b / N) % N, bk = b / G::N2;
        double K[3][3] = {};
        for (int q = 0; q < N3; ++q) {
            const int qx = q % N, qy = (q / N) % N, qz = q / G::N2;
            const double da[3] = {sSd[qx * N + ai] * sS[qy * N + aj] * sS[qz * N + ak],
                                  sS[qx * N + ai] * sSd[qy * N + aj] * sS[qz * N + ak],
                                  sS[qx * N + ai] * sS[qy * N + aj] * sSd[qz * N + ak]};
            const double db[3] = {sSd[qx * N + bi] * sS[qy * N + bj] * sS[qz * N + bk],
                                  sS[qx * N + bi] * sSd[qy * N + bj] * sS[qz * N + bk],
                                  sS[qx * N + bi] * sS[qy * N + bj] * sSd[qz * N + bk]};
            double M[9], t[6];
#pragma unroll
            for (int f = 0; f < 9; ++f) M[f] = cache[f * G::NQ + q];
#pragma unroll
            for (int f = 0; f < 6; ++f) t[f] = cache[(9 + f) * G::NQ + q];
            const double c1 = cache[15 * G::NQ + q], c2 = cache[16 * G::NQ + q];
            double ga[3], gb[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                ga[m] = fma(da[0], M[m], fma(da[1], M[3 + m], da[2] * M[6 + m]));
                gb[m] = fma(db[0], M[m], fma(db[1], M[3 + m], db[2] * M[6 + m]));
            }
            const double gab = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
            const double gtg = ga[0] * (t[0] * gb[0] + t[5] * gb[1] + t[4] * gb[2]) +
                               ga[1] * (t[5] * gb[0] + t[1] * gb[1] + t[3] * gb[2]) +
                               ga[2] * (t[4] * gb[0] + t[3] * gb[1] + t[2] * gb[2]);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j) K[i][j] += c1 * ga[i] * gb[j] + 0.5 * c2 * ga[j] * gb[i];
                K[i][i] += 0.5 * c2 * gab + gtg;
            }
        }
        int64_t na, nb;
        if constexpr (HX) {
            na = p.conn[(int64_t)cell * N3 + a];
            nb = p.conn[(int64_t)cell * N3 + b];
        } else {
            na = (P * ex + ai) + (int64_t)p.Nx * ((P * ey + aj) + (int64_t)p.Ny * (P * ez + ak));
            nb = (P * ex + bi) + (int64_t)p.Nx * ((P * ey + bj) + (int64_t)p.Ny * (P * ez + bk));
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) unsafeAtomicAdd(A + (3 * na + i) * n + 3 * nb + j, K[i][j]);
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

template <int N>
static Tables<N, float> to_float(const Tables<N>& T) {
    Tables<N, float> F;
    auto cvt = [](const EO<N>& a, EO<N, float>& b) {
        for (int q = 0; q < EO<N>::H; ++q) {
            for (int i = 0; i < EO<N>::H; ++i) b.E[q][i] = (float)a.E[q][i];
            for (int i = 0; i < (EO<N>::M > 0 ? EO<N>::M : 1); ++i) b.O[q][i] = (float)a.O[q][i];
        }
    };
    cvt(T.S, F.S);
    cvt(T.St, F.St);
    cvt(T.D, F.D);
    cvt(T.Dt, F.Dt);
    for (int i = 0; i < N; ++i) {
        F.qp[i] = T.qp[i];
        F.qw[i] = T.qw[i];
    }
    return F;
}

template <int N>
static MfmaMats<N> make_mfma_mats(const Tables1D& t) {
    MfmaMats<N> M;
    for (int q = 0; q < N; ++q)
        for (int i = 0; i < N; ++i) {
            double ds = 0.0, stdt = 0.0;
            for (int l = 0; l < N; ++l) {
                ds += t.D[q][l] * t.S[l][i];    // (D S)[q][i]
                stdt += t.S[l][q] * t.D[i][l];  // (St Dt)[q][i]
            }
            M.S[q][i] = (float)t.S[q][i];
            M.D[q][i] = (float)t.D[q][i];
            M.St[q][i] = (float)t.S[i][q];
            M.Dt[q][i] = (float)t.D[i][q];
            M.DS[q][i] = (float)ds;
            M.StDt[q][i] = (float)stdt;
        }
    return M;
}

template <int N, int MODE, typename R, bool HX, int SW = 0>
static hipError_t launch_nm(const Tables<N>& T, const KParams& p, hipStream_t stream, const MfmaMats<N>& MM,
                            const LaunchTiming& tm) {
    const int nb = p.nbx * p.nby * p.nbz;
    Tables<N, R> TR;
    if constexpr (std::is_same_v<R, float>) TR = to_float<N>(T);
    else TR = T;
    if (tm.start)
        hipExtLaunchKernelGGL((cell_kernel<N, MODE, R, HX, SW>), dim3(nb), dim3(Geo<N, HX>::NT), 0, stream, tm.start,
                              tm.stop, 0, p, T, TR, MM);
    else
        hipLaunchKernelGGL((cell_kernel<N, MODE, R, HX, SW>), dim3(nb), dim3(Geo<N, HX>::NT), 0, stream, p, T, TR, MM);
    return hipGetLastError();
}

// the apply modes with matrix-core sweeps of the w field (boxes)
template <int N, int SW>
static hipError_t launch_mfma_n(int mode, const Tables<N>& T, const MfmaMats<N>& MM, const KParams& p,
                                hipStream_t s, const LaunchTiming& tm) {
    switch (mode) {
        case MODE_APPLY_OTF: return launch_nm<N, MODE_APPLY_OTF, float, false, SW>(T, p, s, MM, tm);
        case MODE_APPLY_OTF_GEOM: return launch_nm<N, MODE_APPLY_OTF_GEOM, float, false, SW>(T, p, s, MM, tm);
        case MODE_APPLY_T2: return launch_nm<N, MODE_APPLY_T2, float, false, SW>(T, p, s, MM, tm);
        case MODE_APPLY_T4: return launch_nm<N, MODE_APPLY_T4, float, false, SW>(T, p, s, MM, tm);
        case MODE_APPLY_OTF_AD: return launch_nm<N, MODE_APPLY_OTF_AD, float, false, SW>(T, p, s, MM, tm);
        case MODE_APPLY_OTF_AD_SPLIT: return launch_nm<N, MODE_APPLY_OTF_AD_SPLIT, float, false, SW>(T, p, s, MM, tm);
        default: return hipErrorInvalidValue;
    }
}

template <int N, bool HX>
static hipError_t launch_n(int mode, bool fp32, const Tables1D& t, const KParams& p, hipStream_t s, int sweep = 0,
                           const LaunchTiming& tm = LaunchTiming{}) {
    const Tables<N> T = make_tables<N>(t);
    if (sweep != 0) {  // matrix-core sweeps: FP32 vectors and caches, structured boxes
        if constexpr (HX) {
            return hipErrorInvalidValue;
        } else {
            if (!fp32) return hipErrorInvalidValue;
            const MfmaMats<N> MM = make_mfma_mats<N>(t);
            if (sweep == 1) return launch_mfma_n<N, 1>(mode, T, MM, p, s, tm);
            if (sweep == 3) return launch_mfma_n<N, 3>(mode, T, MM, p, s, tm);
            return hipErrorInvalidValue;
        }
    }
    if (fp32) {
        switch (mode) {
            case MODE_APPLY_OTF: return launch_nm<N, MODE_APPLY_OTF, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_APPLY_OTF_GEOM: return launch_nm<N, MODE_APPLY_OTF_GEOM, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_APPLY_T2: return launch_nm<N, MODE_APPLY_T2, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_APPLY_T4: return launch_nm<N, MODE_APPLY_T4, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_APPLY_OTF_AD: return launch_nm<N, MODE_APPLY_OTF_AD, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_BUILD_T2: return launch_nm<N, MODE_BUILD_T2, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_BUILD_T4: return launch_nm<N, MODE_BUILD_T4, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_APPLY_OTF_AD_SPLIT: return launch_nm<N, MODE_APPLY_OTF_AD_SPLIT, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            case MODE_BUILD_T4_SPLIT: return launch_nm<N, MODE_BUILD_T4_SPLIT, float, HX>(T, p, s, MfmaMats<N>{}, tm);
            default: return hipErrorInvalidValue;
        }
    }
    switch (mode) {
        case MODE_APPLY_OTF: return launch_nm<N, MODE_APPLY_OTF, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_APPLY_OTF_GEOM: return launch_nm<N, MODE_APPLY_OTF_GEOM, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_APPLY_T2: return launch_nm<N, MODE_APPLY_T2, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_APPLY_T4: return launch_nm<N, MODE_APPLY_T4, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_APPLY_OTF_AD: return launch_nm<N, MODE_APPLY_OTF_AD, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_RESIDUAL: return launch_nm<N, MODE_RESIDUAL, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_STATE: return launch_nm<N, MODE_STATE, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_BUILD_GEOM: return launch_nm<N, MODE_BUILD_GEOM, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_BUILD_T2: return launch_nm<N, MODE_BUILD_T2, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_BUILD_T4: return launch_nm<N, MODE_BUILD_T4, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_ENERGY: return launch_nm<N, MODE_ENERGY, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_APPLY_OTF_AD_SPLIT: return launch_nm<N, MODE_APPLY_OTF_AD_SPLIT, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_RESIDUAL_SPLIT: return launch_nm<N, MODE_RESIDUAL_SPLIT, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_BUILD_T4_SPLIT: return launch_nm<N, MODE_BUILD_T4_SPLIT, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        case MODE_ENERGY_SPLIT: return launch_nm<N, MODE_ENERGY_SPLIT, double, HX>(T, p, s, MfmaMats<N>{}, tm);
        default: return hipErrorInvalidValue;
    }
}

template <int N, bool HX>
static hipError_t launch_diag_n(const Tables1D& t, const KParams& p, double* diag, hipStream_t stream) {
    DiagTables T;
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            T.S[a][b] = t.S[a][b];
            double s = 0.0;  // derivative of the nodal basis at the Gauss points: D S
            for (int l = 0; l < t.n; ++l) s += t.D[a][l] * t.S[l][b];
            T.Sd[a][b] = (a < t.n && b < t.n) ? s : 0.0;
        }
    const int nb = p.nbx * p.nby * p.nbz;
    hipLaunchKernelGGL((diag_kernel<N, HX>), dim3(nb), dim3(Geo<N, HX>::NT), 0, stream, p, T, diag);
    return hipGetLastError();
}

template <int N, bool HX>
static hipError_t launch_dense_n(const Tables1D& t, const KParams& p, double* A, int64_t n, hipStream_t stream) {
    DiagTables T;
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            T.S[a][b] = t.S[a][b];
            double s = 0.0;  // derivative of the nodal basis at the Gauss points: D S
            for (int l = 0; l < t.n; ++l) s += t.D[a][l] * t.S[l][b];
            T.Sd[a][b] = (a < t.n && b < t.n) ? s : 0.0;
        }
    hipLaunchKernelGGL((dense_kernel<N, HX>), dim3(p.ne), dim3(256), 0, stream, p, T, A, n);
    return hipGetLastError();
}

}  // namespace mfe
