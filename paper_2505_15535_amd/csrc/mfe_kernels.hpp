// Host-visible declarations of the HIP kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfe {

// What a launch of the cell kernel computes.
enum Mode : int {
    MODE_APPLY_OTF = 0,       // v += K(u) w, geometry from vertices, closed form
    MODE_APPLY_OTF_GEOM = 1,  // v += K(u) w, stored inverse Jacobian and JxW
    MODE_APPLY_T2 = 2,        // v += K w from the second-order cache
    MODE_APPLY_T4 = 3,        // v += K w from the fourth-order cache
    MODE_APPLY_OTF_AD = 4,    // v += K(u) w, dual-number directional derivative
    MODE_RESIDUAL = 5,        // v += R(u)
    MODE_STATE = 6,           // flag det F <= 0
    MODE_BUILD_GEOM = 7,      // cache <- (Jg^-1, JxW)
    MODE_BUILD_T2 = 8,        // cache <- (M, tau JxW, c1, c2)
    MODE_BUILD_T4 = 9,        // cache <- (Jc JxW, tau JxW, M)
    MODE_ENERGY = 10,         // v[brick] <- sum over the brick's points of JxW psi(F)
    // the split neo-Hookean law (mu, kappa); the other modes do not depend on it
    MODE_APPLY_OTF_AD_SPLIT = 11,
    MODE_RESIDUAL_SPLIT = 12,
    MODE_BUILD_T4_SPLIT = 13,
    MODE_ENERGY_SPLIT = 14,
    MODE_COUNT = 15
};

// Doubles per quadrature point of each cache.
constexpr int kGeomFields = 10;
constexpr int kT2Fields = 17;
constexpr int kT4Fields = 36;

struct KParams {
    int nx, ny, nz;            // cells per direction
    int ne;                    // nx*ny*nz
    int Nx, Ny;                // nodes per direction (x, y)
    int nbx, nby, nbz;         // bricks per direction (one workgroup per brick)
    int64_t nq_stride;         // bricks * points per brick: stride between cache fields
    const double* verts;       // (nx+1)(ny+1)(nz+1) x 3
    const double* u;           // state (gather source of the u field)
    const double* w;           // input vector (gather source of the w field)
    double* v;                 // output, accumulated with atomics
    const double* cache;       // SoA cache read by OTF_GEOM/T2/T4 applies
    double* cache_out;         // SoA cache written by BUILD modes
    const float* w32;          // FP32 launches: input vector
    float* v32;                // FP32 launches: output vector
    const float* cache32;      // FP32 T2/T4 applies: cache (OTF_GEOM reads `cache`)
    float* cache_out32;        // FP32 T2/T4 builds: cache written
    const double* cell_mat;    // ne x (mu, lambda) or null
    // general hexahedral meshes (null for a structured box): global node id of
    // every (cell, local node), ne x n^3, and the 8 vertex ids of every cell
    const int* conn;
    const int* ev;
    // general meshes: distinct nodes of each workgroup's cells (cells x n^3
    // slots per group, -1 padded) and each cell node's slot
    const int* gnodes;
    const unsigned short* lidx;
    double mu, lam;            // uniform material
    int* flag;                 // STATE: set to 1 if det F <= 0 somewhere
    // Q2 box applies: constrained dofs as a bitmap (bit d % 32 of word d / 32),
    // or null; colour 0 runs every brick with atomics on shared faces, colour
    // 1..8 only the bricks of parity class colour - 1 (bx & 1 | (by & 1) << 1 |
    // (bz & 1) << 2) with plain read-add-writes
    const uint32_t* cmask;
    int colour;
};

// 1D data of degree p = N-1 computed on the host: S (Lagrange basis on
// Gauss-Lobatto support points, evaluated at Gauss points), D (derivative
// collocated on the Gauss points), Gauss points and weights on [0, 1].
struct Tables1D {
    int n;
    double S[8][8];
    double D[8][8];
    double qp[8];
    double qw[8];
};

// Cells per brick in each direction and quadrature points per brick for
// n = p+1 points per direction (zeros for an unsupported n).
void brick_shape(int n, int* bx, int* by, int* bz, int* points_per_brick);

// Cells per workgroup and quadrature points per workgroup of the general-mesh
// kernels (zeros for an unsupported n); workgroup g owns cells
// [g*cells, (g+1)*cells).
void hex_group_shape(int n, int* cells, int* points_per_group);

// Launch the cell kernel of `mode` for degree p = n-1 (n in 2..7).  With
// fp32 the w/v vectors (w32, v32), the T2/T4 caches (cache32, cache_out32)
// and the sweeps of w are FP32; only the apply and T2/T4 build modes exist so.
// sweep = 1 or 3: the FP32 apply modes with the w-field sweeps on the matrix
// cores (one or three bf16 pieces per operand; structured boxes only).
// Start and stop events of a timed launch, recorded by the kernel's dispatch
// itself (no extra commands on the stream); both null for an untimed launch.
struct LaunchTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

hipError_t launch_cell_kernel(int mode, const Tables1D& t, const KParams& p, hipStream_t stream,
                              bool fp32 = false, int sweep = 0, const LaunchTiming& tm = LaunchTiming{});
// True when launch_cell_kernel runs a tangent apply of this kind with the
// wavefront-per-two-cells kernel (Q2 structured boxes, vector-ALU sweeps),
// which reads the constraint bitmap and the colour of KParams itself; fp32:
// FP32 vectors; coloured: the coloured mode (p.colour > 0), which only that
// kernel has, so every apply mode it holds runs there.
bool wave_apply(int n, int mode, bool hex, int sweep, bool fp32, bool coloured);
// The launch of those applies (reached through launch_cell_kernel).
hipError_t launch_wave(int mode, bool fp32, const Tables1D& t, const KParams& p, hipStream_t stream,
                       const LaunchTiming& tm);
// Number of bricks of parity class `colour` - 1 (1..8) of a box of
// nbx x nby x nbz bricks.
int64_t colour_bricks(int nbx, int nby, int nbz, int colour);
// The general-mesh instantiations (p.conn != null), reached through
// launch_cell_kernel and launch_diagonal.
hipError_t launch_cell_kernel_hex(int mode, const Tables1D& t, const KParams& p, hipStream_t stream, bool fp32,
                                  const LaunchTiming& tm);

// Nodal basis values S and their derivatives Sd at the Gauss points.
struct DiagTables {
    double S[8][8];
    double Sd[8][8];
};

// diag += diagonal of the tangent, from the second-order cache in p.cache
// (which must be built for the current state).
hipError_t launch_diagonal(const Tables1D& t, const KParams& p, double* diag, hipStream_t stream);
hipError_t launch_diagonal_hex(const Tables1D& t, const KParams& p, double* diag, hipStream_t stream);

// A += dense tangent of a structured box (n = its dof count, A row-major
// n x n) from the second-order cache in p.cache.
hipError_t launch_dense_tangent(const Tables1D& t, const KParams& p, double* A, int64_t n, hipStream_t stream);
// Ainv (nf x nf) = inverse of the block of A (n x n, row-major) on the dofs
// free_idx[0..nf), nf <= kDenseMax, for a symmetric positive definite block;
// *fail = 1 (Ainv undefined) when a pivot is not positive and finite.  One
// workgroup, the block in LDS.
constexpr int kDenseMax = 196;
hipError_t launch_sweep_inverse(const double* A, int n, const int* free_idx, int nf, double* Ainv, int* fail,
                                hipStream_t s);
// x = Ainv b on the free dofs (pos[dof] = its row of Ainv, or -1 for a
// constrained dof, where x = 0)
hipError_t launch_dense_matvec(const double* Ainv, const int* pos, const int* free_idx, int nf, const double* b,
                               double* x, int n, hipStream_t s);
hipError_t launch_dense_matvec(const float* Ainv, const int* pos, const int* free_idx, int nf, const float* b,
                               float* x, int n, hipStream_t s);
hipError_t launch_fill(double* x, int64_t n, double value, hipStream_t stream);
hipError_t launch_fill(float* x, int64_t n, float value, hipStream_t stream);

// Solver vector kernels.  Reductions use kDotBlocks partial sums (scratch of
// 2*kDotBlocks doubles) and a fixed-order second pass, so they are
// deterministic; `out` receives two doubles.
constexpr int kDotBlocks = 1024;
hipError_t launch_dot2(const double* a, const double* b, const double* c, const double* d, int64_t n,
                       double* partials, double* out, hipStream_t s);
hipError_t launch_cg_update(double* x, double* r, double* z, const double* p, const double* Ap, const double* dinv,
                            double alpha, int64_t n, double* partials, double* out, hipStream_t s);
hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
// x += (nd[0] / nd[1]) y, the ratio read on the device (no update unless both
// are positive and the ratio finite)
hipError_t launch_axpy_ratio(const double* nd, const double* y, double* x, int64_t n, hipStream_t s);
// launch_cg_update with alpha = rz[0] / pAp[0] read on the device (alpha = 0,
// so x and r unchanged, unless both are positive)
hipError_t launch_cg_update_dev(double* x, double* r, double* z, const double* p, const double* Ap,
                                const double* dinv, const double* rz, const double* pAp, int64_t n, double* partials,
                                double* out, hipStream_t s);
// p = z + (rz_new[0] / rz_old[0]) p with the ratio formed on the device (0
// unless rz_old[0] > 0)
hipError_t launch_p_update_dev(const double* z, const double* rz_new, const double* rz_old, double* p, int64_t n,
                               hipStream_t s);
hipError_t launch_scale_mul(double scale, const double* sc, const double* x, double* y, int64_t n, hipStream_t s);
// d = 1/d (1/|d| with absolute); *bad = 1 where that is not positive and finite
// Flexible CG with a window of kMaxDirs earlier directions: out[j] = z . Y[j]
// (Y: m rows of n, m <= kMaxDirs; partials need m * 256 doubles), and
// p = z - sum_j c[j] P[j].
constexpr int kMaxDirs = 8;
struct DirCoeffs {
    double c[kMaxDirs];
};
hipError_t launch_multidot(const double* z, const double* Y, int m, int64_t n, double* partials, double* out,
                           hipStream_t s);
hipError_t launch_multi_axpy(const double* z, const double* P, const DirCoeffs& c, int m, int64_t n, double* p,
                             hipStream_t s);
// out[0] = sum of x[0..n) (one workgroup, fixed order)
hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s);
hipError_t launch_invert(double* d, int64_t n, int* bad, hipStream_t s, bool absolute = false);

// Multigrid kernels (FP64 and FP32).  out = M in with the 1D CSR matrix M
// acting along `axis` of nodal arrays [nz][ny][nx][3] (out extents nx_out,
// ny_out, nz_out; in has nx_in, ny_in and the out extents elsewhere).
// Fused forms: with rb, `in` is read as (dinv != 0) ? rb - in : 0 (the free
// residual); with x, the result is added to x where dinv != 0 and `clear` is
// zeroed instead of writing out.
hipError_t launch_axis_csr(const int* rowptr, const int* colidx, const double* vals, int axis, int nx_out,
                           int ny_out, int nz_out, int nx_in, int ny_in, const double* in, double* out,
                           hipStream_t s, const double* rb = nullptr, const double* dinv = nullptr,
                           double* x = nullptr, double* clear = nullptr);
hipError_t launch_axis_csr(const int* rowptr, const int* colidx, const float* vals, int axis, int nx_out,
                           int ny_out, int nz_out, int nx_in, int ny_in, const float* in, float* out,
                           hipStream_t s, const float* rb = nullptr, const float* dinv = nullptr,
                           float* x = nullptr, float* clear = nullptr);
// d = c1 d + c2 dinv .* (b - Ax);  x += d (x = d with x_init);  Ax = 0
// (Ax null: b; d is not read when c1 = 0)
hipError_t launch_cheb(double* d, double* x, const double* b, double* Ax, const double* dinv, double c1,
                       double c2, int64_t n, hipStream_t s, bool x_init = false);
hipError_t launch_cheb(float* d, float* x, const float* b, float* Ax, const float* dinv, float c1, float c2,
                       int64_t n, hipStream_t s, bool x_init = false);
// x += y;  y = 0
hipError_t launch_add_clear(double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_add_clear(float* x, float* y, int64_t n, hipStream_t s);
// y = x
hipError_t launch_copy(const double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_copy(const float* x, float* y, int64_t n, hipStream_t s);
hipError_t launch_axpby(float a, const float* x, float b, float* y, int64_t n, hipStream_t s);
hipError_t launch_convert(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_convert(const float* src, double* dst, int64_t n, hipStream_t s);
// Learned smoother correction (mfe_net.hip): patches of 4x4x4 Q2 cells
// (9^3 nodes), activations [patch][channel][729].
hipError_t launch_conv3d(const float* x, const float* W, const float* bias, int P, int CI, int CO, bool flip,
                         bool relu, const float* mask, float* y, hipStream_t s);
hipError_t launch_conv3d_wgrad(const float* x, const float* dy, int P, int CI, int CO, float* dW, float* db,
                               hipStream_t s);
int mse_blocks(int64_t n);
hipError_t launch_mse(const float* y, const float* t, int64_t n, float* dy, double* partial, hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_patch_features(const double* r, const float* inv, int Nx, int Ny, int npx, int npy, int P,
                                 bool linear, float* feat, float* scale, hipStream_t s);
hipError_t launch_patch_targets(const double* e, const float* scale, int Nx, int Ny, int npx, int npy, int P,
                                float* t, hipStream_t s);
hipError_t launch_patch_scatter(const float* y, const float* scale, int Nx, int Ny, int Nz, int npx, int npy,
                                int npz, double alpha, double* z, hipStream_t s);
hipError_t launch_patch_adjoint(const double* g, const float* scale, int Nx, int Ny, int npx, int npy, int npz,
                                int P, float alpha, float* dy, hipStream_t s);
hipError_t launch_node_invariants(const double* u, const double* verts, int nx, int ny, int nz, int Nx, int Ny,
                                  int Nz, float* cell_scratch, float* ninv, hipStream_t s);

hipError_t launch_copy_indexed(const int64_t* idx, int64_t n, const double* src, double* dst,
                               hipStream_t stream);
hipError_t launch_copy_indexed(const int64_t* idx, int64_t n, const float* src, float* dst, hipStream_t stream);
// dst[idx[i]] = a[idx[i]] - b[idx[i]]
hipError_t launch_diff_indexed(const int64_t* idx, int64_t n, const double* a, const double* b, double* dst,
                               hipStream_t stream);
// dst[idx[i]] = src[i] for i < n
hipError_t launch_scatter_indexed(const int64_t* idx, int64_t n, const double* src, double* dst, hipStream_t stream);
hipError_t launch_set_indexed(const int64_t* idx, int64_t n, double value, double* dst, hipStream_t stream);
hipError_t launch_set_indexed(const int64_t* idx, int64_t n, float value, float* dst, hipStream_t stream);

}  // namespace mfe
