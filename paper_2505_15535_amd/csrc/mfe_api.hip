// C ABI of libmfe: context, mesh, material, constraints, state, caches,
// tangent apply and residual.  Host-side 1D tables (Gauss rule, Gauss-Lobatto
// support points, Lagrange matrices) are computed here.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mfe.h"
#include "mfe_kernels.hpp"
#include "mfe_mesh.hpp"

using mfe::KParams;
using mfe::Tables1D;

namespace {

constexpr int kNumCaches = 3;  // OTF_GEOM, T2, T4
int cache_slot(int strategy) {
    switch (strategy) {
        case MFE_OTF_GEOM: return 0;
        case MFE_T2: return 1;
        case MFE_T4: return 2;
        default: return -1;
    }
}
// strategies that do not depend on the law, or that differentiate it with
// dual numbers, exist for the split law; the closed-form ones are model specific
bool strategy_supported(int model, int strategy) {
    return model == MFE_MODEL_NH || strategy == MFE_OTF_AD || strategy == MFE_T4;
}

int cache_fields(int slot) {
    return slot == 0 ? mfe::kGeomFields : (slot == 1 ? mfe::kT2Fields : mfe::kT4Fields);
}

// ----------------------------------------------------------------- 1D tables
// Legendre polynomial P_n and its derivative at x in [-1, 1] (three-term recurrence).
void legendre(int n, double x, double& P, double& dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        P = 1.0;
        dP = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    P = p1;
    dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// n-point Gauss-Legendre rule on [0, 1] by Newton iteration on P_n.
void gauss_rule(int n, double* x01, double* w01) {
    std::vector<double> x(n), w(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, z, P, dP);
            const double dz = P / dP;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        double P, dP;
        legendre(n, z, P, dP);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dP * dP);
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return x[a] < x[b]; });
    for (int i = 0; i < n; ++i) {
        x01[i] = 0.5 * (x[order[i]] + 1.0);
        w01[i] = 0.5 * w[order[i]];
    }
    // exact symmetry about 1/2
    for (int i = 0; i < n / 2; ++i) {
        const double a = 0.5 * (x01[i] + (1.0 - x01[n - 1 - i]));
        x01[i] = a;
        x01[n - 1 - i] = 1.0 - a;
        const double b = 0.5 * (w01[i] + w01[n - 1 - i]);
        w01[i] = w01[n - 1 - i] = b;
    }
    if (n % 2 == 1) x01[n / 2] = 0.5;
}

// Gauss-Lobatto-Legendre points of degree p on [0, 1]: end points and the
// roots of P_p' (Newton on P_p' with P_p'' from Legendre's equation).
void gll_points(int p, double* x01) {
    std::vector<double> x(p + 1);
    x[0] = -1.0;
    x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double z = -std::cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, z, P, dP);
            const double d2P = (2.0 * z * dP - p * (p + 1.0) * P) / (1.0 - z * z);
            const double dz = dP / d2P;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[i] = z;
    }
    std::sort(x.begin(), x.end());
    for (int i = 0; i <= p; ++i) x01[i] = 0.5 * (x[i] + 1.0);
    for (int i = 0; i < (p + 1) / 2; ++i) {
        const double a = 0.5 * (x01[i] + (1.0 - x01[p - i]));
        x01[i] = a;
        x01[p - i] = 1.0 - a;
    }
    if (p % 2 == 0) x01[p / 2] = 0.5;
}

void make_tables(int degree, Tables1D& t) {
    const int n = degree + 1;
    std::memset(&t, 0, sizeof(t));
    t.n = n;
    double nodes[8];
    gll_points(degree, nodes);
    gauss_rule(n, t.qp, t.qw);
    // S[q][i] = l_i(x_q), Lagrange basis through the support points
    for (int q = 0; q < n; ++q)
        for (int i = 0; i < n; ++i) {
            double v = 1.0;
            for (int j = 0; j < n; ++j)
                if (j != i) v *= (t.qp[q] - nodes[j]) / (nodes[i] - nodes[j]);
            t.S[q][i] = v;
        }
    // D[q][l] = derivative at x_q of the Lagrange polynomial through the Gauss
    // points that is 1 at x_l (barycentric form)
    double bw[8];
    for (int l = 0; l < n; ++l) {
        double prod = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != l) prod *= (t.qp[l] - t.qp[m]);
        bw[l] = 1.0 / prod;
    }
    for (int q = 0; q < n; ++q) {
        double diag = 0.0;
        for (int l = 0; l < n; ++l) {
            if (l == q) continue;
            t.D[q][l] = (bw[l] / bw[q]) / (t.qp[q] - t.qp[l]);
            diag += 1.0 / (t.qp[q] - t.qp[l]);
        }
        t.D[q][q] = diag;
    }
    // enforce the exact centro-(anti)symmetry used by the even-odd sweeps
    for (int q = 0; q < n; ++q)
        for (int i = 0; i < n; ++i) {
            const int q2 = n - 1 - q, i2 = n - 1 - i;
            if (q * n + i > q2 * n + i2) continue;
            const double s = 0.5 * (t.S[q][i] + t.S[q2][i2]);
            t.S[q][i] = t.S[q2][i2] = s;
            const double d = 0.5 * (t.D[q][i] - t.D[q2][i2]);
            t.D[q][i] = d;
            t.D[q2][i2] = -d;
        }
}

// Partial sums of the allocation-free energy (mfe_energy_noalloc): one double
// per brick of cells.  Each GPU the library runs on holds its own copy for
// the life of the process.
constexpr int64_t kNoAllocDoubles = (int64_t)1 << 18;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

// Device address of `scratch` on the current device (the array's name in host
// code is a stand-in, not that address), looked up once per device.
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

hipError_t scratch_address(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// 1D matrix in CSR form on the device (values in FP64 and FP32)
struct DevCSR {
    int rows = 0, cols = 0;
    int* rowptr = nullptr;
    int* col = nullptr;
    double* val = nullptr;
    float* valf = nullptr;
    const double* vals(double*) const { return val; }
    const float* vals(float*) const { return valf; }
};

// Work vectors of one level in one precision
template <typename T>
struct MGVec {
    T *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr, *dinv = nullptr, *tmp1 = nullptr, *tmp2 = nullptr;
};

}  // namespace

// One level of the geometric multigrid hierarchy.  Level 0 is the context
// itself; coarser levels own a child context.  Transfers to the next coarser
// level are stored with the finer level.
struct MGLevel {
    mfe_ctx* ctx = nullptr;
    bool own = false;
    double* vec = nullptr;     // FP64: b, x, r, d, dinv, tmp1, tmp2, rnd (n_dofs each)
    float* vec32 = nullptr;    // FP32: b, x, r, d, dinv, tmp1, tmp2 (allocated on first FP32 use)
    MGVec<double> v64;
    MGVec<float> v32;
    double* rnd = nullptr;     // fixed random start of the eigenvalue estimate
    double lmax = 0.0;         // estimate of the largest eigenvalue of D^-1 K
    // coarsest level solved directly: the inverse of its tangent on the nf
    // free dofs (nf x nf, followed by the n x n assembled tangent), an FP32
    // copy, and the maps dof -> free row (-1: constrained), row -> dof
    double* dense = nullptr;
    float* dense32 = nullptr;
    int* dense_pos = nullptr;
    int* dense_free = nullptr;
    int dense_nf = 0;
    bool dense_ok = false;
    // per axis, between this level and the next coarser one: prolongation
    // (fine x coarse), restriction (its transpose) and interpolation of the
    // state to the coarse nodes (coarse x fine)
    DevCSR P[3], R[3], I[3];
    MGVec<double>& vecs(double*) { return v64; }
    MGVec<float>& vecs(float*) { return v32; }
};

struct mfe_ctx {
    int device = 0;
    std::string err;
    // mesh
    bool has_mesh = false;
    // general hexahedral mesh (mfe_mesh_hex): nx = ny = nz = 0, cells gathered
    // through the cell-node table d_conn, geometry from d_ev
    // Cells are processed in an internal order (Morton order of their
    // centroids, h_perm[internal] = caller's index) in groups of consecutive
    // cells, each group with its list of distinct nodes (d_gnodes, padded
    // with -1) and every cell node's position in that list (d_lidx).
    bool hex = false;
    int* d_conn = nullptr;
    int* d_ev = nullptr;
    int* d_gnodes = nullptr;
    unsigned short* d_lidx = nullptr;
    std::vector<int32_t> h_ev, h_conn, h_perm;
    int nx = 0, ny = 0, nz = 0, degree = 0;
    int Nx = 0, Ny = 0, Nz = 0;
    int64_t n_nodes = 0, n_dofs = 0, ne = 0, nq = 0;
    int nbx = 0, nby = 0, nbz = 0;  // bricks per direction
    int64_t nq_stride = 0;          // cache entries per field (bricks * points per brick)
    Tables1D tab;
    double* d_verts = nullptr;
    // material: law (MFE_MODEL_*) and its two moduli (mu, lambda) or (mu, kappa)
    int model = MFE_MODEL_NH;
    double mu = 1.0, lam = 1.0;
    double* d_cellmat = nullptr;
    // constraints
    double* d_wmask = nullptr;   // w with constrained entries zeroed
    int64_t* d_cidx = nullptr;
    uint32_t* d_cmask = nullptr; // constrained dofs as a bitmap (bit d % 32 of word d / 32)
    int64_t n_con = 0;
    // tangent applies in the coloured, bitwise reproducible mode
    bool deterministic = false;
    // state and caches
    double* d_u = nullptr;
    bool has_state = false;
    uint64_t state_version = 0;
    double* d_cache[kNumCaches] = {nullptr, nullptr, nullptr};
    uint64_t cache_version[kNumCaches] = {0, 0, 0};
    bool cache_valid[kNumCaches] = {false, false, false};
    // FP32 copies of the T2 and T4 caches (slots 1, 2) for mixed-precision applies
    float* d_cache32[kNumCaches] = {nullptr, nullptr, nullptr};
    uint64_t cache32_version[kNumCaches] = {0, 0, 0};
    bool cache32_valid[kNumCaches] = {false, false, false};
    int* d_flag = nullptr;
    // solver work space: 8 vectors (CG r, z, p, Kp, 1/diag; Newton R, du, dg),
    // partial sums, pinned scalars, flag
    double* d_work = nullptr;
    double* d_path = nullptr;    // load-path driver: trial state, full and compact prescribed values
    double* d_energy = nullptr;  // per-brick energy partials and their sum
    double* d_partials = nullptr;
    double* h_scalars = nullptr;
    double* d_lz = nullptr;  // eigenvalue estimates: device history of their CG coefficients
    double* h_lz = nullptr;  // and its pinned host copy
    size_t lz_levels = 0;    // levels the two hold
    double* d_lz_part = nullptr;         // per-level partial sums of their dot products
    std::vector<hipStream_t> lz_streams;  // one stream per level for them (default priority)
    std::vector<hipEvent_t> lz_join;
    hipEvent_t lz_fork = nullptr;
    int* d_bad = nullptr;
    // host copies used to derive coarser levels
    std::vector<double> h_verts;
    std::vector<double> h_cellmat;
    std::vector<int64_t> h_cidx;
    // geometric multigrid hierarchy (empty until the first GMG solve)
    std::vector<MGLevel> mg;
    int mg_request = -1;  // mg_levels the hierarchy was built for
    // HIP graph of one preconditioner application
    hipStream_t mg_stream = nullptr;
    // the coarsest level's direct-solve set-up runs on its own stream beside
    // the other levels' eigenvalue estimates (default priority)
    hipStream_t side_stream = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    int* d_bad_dense = nullptr;
    hipGraphExec_t mg_exec = nullptr;
    bool mg_graph_valid = false;
    // lagged multigrid set-up: CG solves left that may reuse the spectrum
    // estimates and the coarse inverse, and the options they were made with
    int mg_lag_left = 0;
    int mg_lag_prec = -1, mg_lag_direct = -1;
    const double* mg_graph_r = nullptr;
    double* mg_graph_z = nullptr;
    int mg_graph_prec = -1;
    mfe_solve_opts mg_graph_opts = {};
    // what the level data were last set up for
    uint64_t mg_ready_version = 0;
    int mg_ready_strategy = -1, mg_ready_prec = -1;
    mfe_solve_opts mg_ready_opts = {};
    // learned smoother correction: network parameters, node invariants of the
    // state, per-patch buffers of the preconditioner
    float* d_net = nullptr;
    int net_variant = MFE_NET_RELU;
    bool net_off = false;        // set when a solve had to drop the correction; cleared by mfe_set_network
    bool net_in_cycle = false;   // the next V-cycle takes the learned step on the finest level
    bool mg_graph_net = false;   // the captured V-cycle graph holds that step
    double* d_netdot = nullptr;  // N.r1 and N.K N of the learned step (device)
    float* d_ninv = nullptr;     // [n_nodes][3] I1, I2, J
    float* d_cinv = nullptr;     // [ne][3] scratch
    uint64_t ninv_version = 0;
    bool ninv_valid = false;
    float* d_nbuf = nullptr;     // features, two hidden layers, output, scale
    double* d_fcg = nullptr;     // flexible CG directions and their images
    // timing of the apply kernel
    int timing = 0;          // record every timing-th apply (0: none)
    int64_t timing_seq = 0;  // applies since timing was set
    std::vector<hipEvent_t> ev_start, ev_stop;
    int ev_used = 0;
    hipEvent_t ev_scratch = nullptr;  // unused end of a timed coloured launch
    double* d_scratch = nullptr;      // this device's `scratch` array (not owned)
};

namespace {

int fail(mfe_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(mfe_ctx* c, hipError_t e, const char* where) {
    return fail(c, e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EHIP,
                std::string(where) + ": " + hipGetErrorString(e));
}

#define MFE_HIP(ctx, call)                                  \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #call); \
    } while (0)

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_csr(DevCSR& m) {
    dfree(m.rowptr);
    dfree(m.col);
    dfree(m.val);
    dfree(m.valf);
    m.rows = m.cols = 0;
}

void mg_free(mfe_ctx* c) {
    for (auto& L : c->mg) {
        dfree(L.vec);
        dfree(L.vec32);
        dfree(L.dense);
        dfree(L.dense32);
        dfree(L.dense_pos);
        dfree(L.dense_free);
        for (int a = 0; a < 3; ++a) {
            free_csr(L.P[a]);
            free_csr(L.R[a]);
            free_csr(L.I[a]);
        }
        if (L.own && L.ctx) mfe_destroy(L.ctx);
    }
    c->mg.clear();
    if (c->mg_exec) (void)hipGraphExecDestroy(c->mg_exec);
    c->mg_exec = nullptr;
    c->mg_graph_valid = false;
    c->mg_lag_left = 0;
}

void free_mesh_data(mfe_ctx* c) {
    mg_free(c);
    dfree(c->d_work);
    dfree(c->d_path);
    dfree(c->d_energy);
    dfree(c->d_ninv);
    dfree(c->d_cinv);
    dfree(c->d_nbuf);
    dfree(c->d_netdot);
    dfree(c->d_fcg);
    c->ninv_valid = false;
    dfree(c->d_verts);
    dfree(c->d_conn);
    dfree(c->d_ev);
    dfree(c->d_gnodes);
    dfree(c->d_lidx);
    c->hex = false;
    c->h_ev.clear();
    c->h_conn.clear();
    c->h_perm.clear();
    dfree(c->d_cellmat);
    dfree(c->d_wmask);
    dfree(c->d_cidx);
    dfree(c->d_cmask);
    dfree(c->d_u);
    for (int i = 0; i < kNumCaches; ++i) {
        dfree(c->d_cache[i]);
        dfree(c->d_cache32[i]);
        c->cache_valid[i] = false;
        c->cache32_valid[i] = false;
    }
    c->n_con = 0;
    c->has_state = false;
    c->has_mesh = false;
}

KParams base_params(const mfe_ctx* c) {
    KParams p;
    std::memset(&p, 0, sizeof(p));
    p.nx = c->nx;
    p.ny = c->ny;
    p.nz = c->nz;
    p.ne = (int)c->ne;
    p.Nx = c->Nx;
    p.Ny = c->Ny;
    p.nbx = c->nbx;
    p.nby = c->nby;
    p.nbz = c->nbz;
    p.nq_stride = c->nq_stride;
    p.verts = c->d_verts;
    p.u = c->d_u;
    p.cell_mat = c->d_cellmat;
    p.conn = c->d_conn;
    p.ev = c->d_ev;
    p.gnodes = c->d_gnodes;
    p.lidx = c->d_lidx;
    p.mu = c->mu;
    p.lam = c->lam;
    p.flag = c->d_flag;
    return p;
}

bool overlaps(const void* a, const void* b, int64_t bytes) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + bytes && y < x + bytes;
}

// det J_g > 0 at every Gauss point of the trilinear map of one cell
int check_cell_geometry(mfe_ctx* c, const double X[8][3], const Tables1D& t, int64_t e) {
    const int n = t.n;
    for (int qz = 0; qz < n; ++qz)
        for (int qy = 0; qy < n; ++qy)
            for (int qx = 0; qx < n; ++qx) {
                const double xi[3] = {t.qp[qx], t.qp[qy], t.qp[qz]};
                double J[3][3] = {};
                for (int v = 0; v < 8; ++v) {
                    const int b[3] = {v & 1, (v >> 1) & 1, v >> 2};
                    double f[3], df[3];
                    for (int d = 0; d < 3; ++d) {
                        f[d] = b[d] ? xi[d] : 1.0 - xi[d];
                        df[d] = b[d] ? 1.0 : -1.0;
                    }
                    const double g[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
                    for (int d = 0; d < 3; ++d)
                        for (int A = 0; A < 3; ++A) J[d][A] += X[v][d] * g[A];
                }
                const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                   J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                   J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                if (!(det > 0.0)) {
                    char buf[160];
                    std::snprintf(buf, sizeof(buf), "det J_g = %g <= 0 in cell %lld", det, (long long)e);
                    return fail(c, MFE_EJACOBIAN, buf);
                }
            }
    return MFE_OK;
}

// Reference position of every node: the trilinear image of the cell's
// Gauss-Lobatto support points (cells sharing a node agree on it).
void node_positions(const mfe_ctx* c, double* xyz) {
    const int p = c->degree, n = p + 1, n3 = n * n * n;
    double gll[8];
    gll_points(p, gll);
    for (int64_t e = 0; e < c->ne; ++e) {
        double X[8][3];
        int64_t ex = 0, ey = 0, ez = 0;
        if (!c->hex) {
            ex = e % c->nx;
            ey = (e / c->nx) % c->ny;
            ez = e / ((int64_t)c->nx * c->ny);
        }
        for (int v = 0; v < 8; ++v) {
            const int64_t id = c->hex ? c->h_ev[8 * e + v]
                                      : (ex + (v & 1)) + (int64_t)(c->nx + 1) * ((ey + ((v >> 1) & 1)) +
                                                                                (int64_t)(c->ny + 1) * (ez + (v >> 2)));
            for (int d = 0; d < 3; ++d) X[v][d] = c->h_verts[3 * id + d];
        }
        for (int a = 0; a < n3; ++a) {
            const int i = a % n, j = (a / n) % n, k = a / (n * n);
            const double xi[3] = {gll[i], gll[j], gll[k]};
            const int64_t node = c->hex ? c->h_conn[e * n3 + a]
                                        : (p * ex + i) + (int64_t)c->Nx * ((p * ey + j) + (int64_t)c->Ny * (p * ez + k));
            double x[3] = {0.0, 0.0, 0.0};
            for (int v = 0; v < 8; ++v) {
                const double w = ((v & 1) ? xi[0] : 1.0 - xi[0]) * (((v >> 1) & 1) ? xi[1] : 1.0 - xi[1]) *
                                 ((v >> 2) ? xi[2] : 1.0 - xi[2]);
                for (int d = 0; d < 3; ++d) x[d] += w * X[v][d];
            }
            for (int d = 0; d < 3; ++d) xyz[3 * node + d] = x[d];
        }
    }
}

}  // namespace

extern "C" {

int mfe_create(mfe_ctx** out, int hip_device) {
    if (!out) return MFE_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return MFE_EINVAL;
    mfe_ctx* c = new (std::nothrow) mfe_ctx();
    if (!c) return MFE_ENOMEM;
    c->device = hip_device;
    DeviceGuard g(hip_device);
    if (!g.ok || hipMalloc(&c->d_flag, sizeof(int)) != hipSuccess) {
        delete c;
        return MFE_EHIP;
    }
    if (scratch_address(hip_device, &c->d_scratch) != hipSuccess) {
        (void)hipFree(c->d_flag);
        delete c;
        return MFE_EHIP;
    }
    *out = c;
    return MFE_OK;
}

void mfe_destroy(mfe_ctx* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    free_mesh_data(c);
    dfree(c->d_flag);
    dfree(c->d_work);
    dfree(c->d_path);
    dfree(c->d_net);
    dfree(c->d_partials);
    dfree(c->d_bad);
    if (c->h_scalars) (void)hipHostFree(c->h_scalars);
    dfree(c->d_lz);
    if (c->h_lz) (void)hipHostFree(c->h_lz);
    for (auto e : c->ev_start) (void)hipEventDestroy(e);
    for (auto e : c->ev_stop) (void)hipEventDestroy(e);
    if (c->ev_scratch) (void)hipEventDestroy(c->ev_scratch);
    if (c->mg_stream) (void)hipStreamDestroy(c->mg_stream);
    if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
    if (c->side_fork) (void)hipEventDestroy(c->side_fork);
    if (c->side_join) (void)hipEventDestroy(c->side_join);
    for (auto st : c->lz_streams) (void)hipStreamDestroy(st);
    for (auto e : c->lz_join) (void)hipEventDestroy(e);
    if (c->lz_fork) (void)hipEventDestroy(c->lz_fork);
    dfree(c->d_lz_part);
    if (c->d_bad_dense) (void)hipFree(c->d_bad_dense);
    delete c;
}

const char* mfe_last_error(const mfe_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

int mfe_mesh_box(mfe_ctx* c, int nx, int ny, int nz, int degree, const double* vxyz) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (nx < 1 || ny < 1 || nz < 1) return fail(c, MFE_EINVAL, "cell counts must be >= 1");
    if (degree < 1 || degree > 6) return fail(c, MFE_EINVAL, "degree must be in 1..6");
    if (!vxyz) return fail(c, MFE_EINVAL, "vertex array is null");
    const int64_t Nx = (int64_t)degree * nx + 1, Ny = (int64_t)degree * ny + 1, Nz = (int64_t)degree * nz + 1;
    const int64_t n_nodes = Nx * Ny * Nz;
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t nq = ne * (degree + 1) * (degree + 1) * (degree + 1);
    if (3 * n_nodes >= (int64_t)1 << 31 || ne >= (int64_t)1 << 31)
        return fail(c, MFE_EINVAL, "mesh too large for 32-bit dof indices");
    // host-side check of det J_g > 0 at every Gauss point (trilinear map)
    Tables1D t;
    make_tables(degree, t);
    for (int64_t e = 0; e < ne; ++e) {
        const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
        double X[8][3];
        for (int v = 0; v < 8; ++v) {
            const int64_t id = (ex + (v & 1)) + (int64_t)(nx + 1) * ((ey + ((v >> 1) & 1)) + (int64_t)(ny + 1) * (ez + (v >> 2)));
            for (int d = 0; d < 3; ++d) X[v][d] = vxyz[3 * id + d];
        }
        const int rc = check_cell_geometry(c, X, t, e);
        if (rc != MFE_OK) return rc;
    }
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, MFE_EHIP, "hipSetDevice failed");
    MFE_HIP(c, hipDeviceSynchronize());
    free_mesh_data(c);
    const int64_t nv = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    MFE_HIP(c, hipMalloc(&c->d_verts, nv * 3 * sizeof(double)));
    MFE_HIP(c, hipMemcpy(c->d_verts, vxyz, nv * 3 * sizeof(double), hipMemcpyHostToDevice));
    c->h_verts.assign(vxyz, vxyz + nv * 3);
    c->h_cellmat.clear();
    c->h_cidx.clear();
    MFE_HIP(c, hipMalloc(&c->d_u, 3 * n_nodes * sizeof(double)));
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->degree = degree;
    c->Nx = (int)Nx;
    c->Ny = (int)Ny;
    c->Nz = (int)Nz;
    c->n_nodes = n_nodes;
    c->n_dofs = 3 * n_nodes;
    c->ne = ne;
    c->nq = nq;
    int bx, by, bz, ppb;
    mfe::brick_shape(degree + 1, &bx, &by, &bz, &ppb);
    c->nbx = (nx + bx - 1) / bx;
    c->nby = (ny + by - 1) / by;
    c->nbz = (nz + bz - 1) / bz;
    c->nq_stride = (int64_t)c->nbx * c->nby * c->nbz * ppb;
    c->tab = t;
    c->mu = 1.0;
    c->lam = 1.0;
    c->has_mesh = true;
    return MFE_OK;
}

int mfe_mesh_hex(mfe_ctx* c, int64_t nv, const double* vxyz, int64_t ne, const int32_t* ev, int degree) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (nv < 8 || ne < 1) return fail(c, MFE_EINVAL, "need at least 8 vertices and one cell");
    if (degree < 1 || degree > 6) return fail(c, MFE_EINVAL, "degree must be in 1..6");
    if (!vxyz || !ev) return fail(c, MFE_EINVAL, "vertex or cell array is null");
    const int n = degree + 1, n3 = n * n * n;
    if (nv >= ((int64_t)1 << 31) || ne * n3 >= ((int64_t)1 << 31))
        return fail(c, MFE_EINVAL, "mesh too large for 32-bit indices");
    std::vector<int32_t> conn;
    int64_t n_nodes = 0;
    const std::string bad = mfe::number_hex_nodes(nv, ne, ev, degree, conn, n_nodes);
    if (!bad.empty()) return fail(c, MFE_EINVAL, bad);
    Tables1D t;
    make_tables(degree, t);
    for (int64_t e = 0; e < ne; ++e) {
        double X[8][3];
        for (int v = 0; v < 8; ++v)
            for (int d = 0; d < 3; ++d) X[v][d] = vxyz[3 * (int64_t)ev[8 * e + v] + d];
        const int rc = check_cell_geometry(c, X, t, e);
        if (rc != MFE_OK) return rc;
    }
    // internal cell order and the per-group node lists
    std::vector<int32_t> perm;
    mfe::morton_order(nv, vxyz, ne, ev, perm);
    int cells, ppg;
    mfe::hex_group_shape(n, &cells, &ppg);
    const int64_t n_groups = (ne + cells - 1) / cells;
    const int maxu = cells * n3;
    std::vector<int32_t> ev_i((size_t)ne * 8), conn_i((size_t)ne * n3), gnodes((size_t)n_groups * maxu, -1);
    std::vector<unsigned short> lidx((size_t)ne * n3);
    for (int64_t e = 0; e < ne; ++e) {
        std::copy(ev + 8 * (int64_t)perm[e], ev + 8 * (int64_t)perm[e] + 8, ev_i.begin() + 8 * e);
        std::copy(conn.begin() + n3 * (int64_t)perm[e], conn.begin() + n3 * (int64_t)perm[e] + n3,
                  conn_i.begin() + n3 * e);
    }
    for (int64_t gi = 0; gi < n_groups; ++gi) {
        const int64_t e0 = gi * cells, e1 = std::min<int64_t>(ne, e0 + cells);
        std::vector<int32_t> u(conn_i.begin() + e0 * n3, conn_i.begin() + e1 * n3);
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        std::copy(u.begin(), u.end(), gnodes.begin() + gi * maxu);
        for (int64_t t = e0 * n3; t < e1 * n3; ++t)
            lidx[t] = (unsigned short)(std::lower_bound(u.begin(), u.end(), conn_i[t]) - u.begin());
    }
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, MFE_EHIP, "hipSetDevice failed");
    MFE_HIP(c, hipDeviceSynchronize());
    free_mesh_data(c);
    MFE_HIP(c, hipMalloc(&c->d_verts, nv * 3 * sizeof(double)));
    MFE_HIP(c, hipMemcpy(c->d_verts, vxyz, nv * 3 * sizeof(double), hipMemcpyHostToDevice));
    MFE_HIP(c, hipMalloc(&c->d_ev, ne * 8 * sizeof(int32_t)));
    MFE_HIP(c, hipMemcpy(c->d_ev, ev_i.data(), ne * 8 * sizeof(int32_t), hipMemcpyHostToDevice));
    MFE_HIP(c, hipMalloc(&c->d_conn, ne * n3 * sizeof(int32_t)));
    MFE_HIP(c, hipMemcpy(c->d_conn, conn_i.data(), ne * n3 * sizeof(int32_t), hipMemcpyHostToDevice));
    MFE_HIP(c, hipMalloc(&c->d_gnodes, gnodes.size() * sizeof(int32_t)));
    MFE_HIP(c, hipMemcpy(c->d_gnodes, gnodes.data(), gnodes.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MFE_HIP(c, hipMalloc(&c->d_lidx, lidx.size() * sizeof(unsigned short)));
    MFE_HIP(c, hipMemcpy(c->d_lidx, lidx.data(), lidx.size() * sizeof(unsigned short), hipMemcpyHostToDevice));
    MFE_HIP(c, hipMalloc(&c->d_u, 3 * n_nodes * sizeof(double)));
    c->h_verts.assign(vxyz, vxyz + nv * 3);
    c->h_ev.swap(ev_i);
    c->h_conn.swap(conn_i);
    c->h_perm.swap(perm);
    c->h_cellmat.clear();
    c->h_cidx.clear();
    c->hex = true;
    c->nx = c->ny = c->nz = 0;
    c->Nx = c->Ny = c->Nz = 0;
    c->degree = degree;
    c->n_nodes = n_nodes;
    c->n_dofs = 3 * n_nodes;
    c->ne = ne;
    c->nq = ne * n3;
    c->nbx = (int)n_groups;
    c->nby = c->nbz = 1;
    c->nq_stride = (int64_t)c->nbx * ppg;
    c->tab = t;
    c->mu = 1.0;
    c->lam = 1.0;
    c->has_mesh = true;
    return MFE_OK;
}

int mfe_hex_numbering(int64_t nv, int64_t ne, const int32_t* ev, int degree, int32_t* cell_nodes,
                      int64_t* n_nodes_out) {
    if (!ev || !n_nodes_out || nv < 8 || ne < 1 || degree < 1 || degree > 6) return MFE_EINVAL;
    const int64_t n = degree + 1;
    if (nv >= ((int64_t)1 << 31) || ne * n * n * n >= ((int64_t)1 << 31)) return MFE_EINVAL;
    std::vector<int32_t> conn;
    int64_t n_nodes = 0;
    if (!mfe::number_hex_nodes(nv, ne, ev, degree, conn, n_nodes).empty()) return MFE_EINVAL;
    *n_nodes_out = n_nodes;
    if (cell_nodes) std::memcpy(cell_nodes, conn.data(), conn.size() * sizeof(int32_t));
    return MFE_OK;
}

int mfe_node_coordinates(mfe_ctx* c, double* xyz) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!xyz) return fail(c, MFE_EINVAL, "null output array");
    node_positions(c, xyz);
    return MFE_OK;
}

int64_t mfe_n_dofs(const mfe_ctx* c) { return (c && c->has_mesh) ? c->n_dofs : 0; }
int64_t mfe_n_cells(const mfe_ctx* c) { return (c && c->has_mesh) ? c->ne : 0; }
int64_t mfe_n_qpoints(const mfe_ctx* c) { return (c && c->has_mesh) ? c->nq : 0; }

int mfe_set_material(mfe_ctx* c, double mu, double lam, const double* per_cell) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!std::isfinite(mu) || !std::isfinite(lam)) return fail(c, MFE_EINVAL, "non-finite material");
    DeviceGuard g(c->device);
    MFE_HIP(c, hipDeviceSynchronize());
    dfree(c->d_cellmat);
    mg_free(c);
    c->h_cellmat.clear();
    if (per_cell) {
        c->h_cellmat.assign(per_cell, per_cell + 2 * c->ne);
        std::vector<double> internal;
        const double* src = per_cell;
        if (c->hex) {  // the kernels read cells in their internal order
            internal.resize(2 * c->ne);
            for (int64_t e = 0; e < c->ne; ++e) {
                internal[2 * e] = per_cell[2 * (int64_t)c->h_perm[e]];
                internal[2 * e + 1] = per_cell[2 * (int64_t)c->h_perm[e] + 1];
            }
            src = internal.data();
        }
        MFE_HIP(c, hipMalloc(&c->d_cellmat, c->ne * 2 * sizeof(double)));
        MFE_HIP(c, hipMemcpy(c->d_cellmat, src, c->ne * 2 * sizeof(double), hipMemcpyHostToDevice));
    }
    c->mu = mu;
    c->lam = lam;
    c->cache_valid[1] = c->cache_valid[2] = false;  // material enters T2/T4
    c->cache32_valid[1] = c->cache32_valid[2] = false;
    return MFE_OK;
}

int mfe_set_model(mfe_ctx* c, int model) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (model != MFE_MODEL_NH && model != MFE_MODEL_SPLIT) return fail(c, MFE_EINVAL, "unknown model");
    if (model != c->model) {
        DeviceGuard g(c->device);
        MFE_HIP(c, hipDeviceSynchronize());
        mg_free(c);
        c->model = model;
        c->cache_valid[1] = c->cache_valid[2] = false;  // the law enters T2/T4
        c->cache32_valid[1] = c->cache32_valid[2] = false;
    }
    return MFE_OK;
}

int mfe_set_constraints(mfe_ctx* c, int64_t n, const int64_t* dofs) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (n < 0 || (n > 0 && !dofs)) return fail(c, MFE_EINVAL, "bad constraint list");
    std::vector<unsigned char> mask(c->n_dofs, 0);
    for (int64_t i = 0; i < n; ++i) {
        if (dofs[i] < 0 || dofs[i] >= c->n_dofs) return fail(c, MFE_EINVAL, "constrained dof out of range");
        mask[dofs[i]] = 1;
    }
    std::vector<int64_t> idx;
    for (int64_t i = 0; i < c->n_dofs; ++i)
        if (mask[i]) idx.push_back(i);
    DeviceGuard g(c->device);
    MFE_HIP(c, hipDeviceSynchronize());
    dfree(c->d_cidx);
    dfree(c->d_wmask);
    dfree(c->d_cmask);
    if (!idx.empty()) {
        MFE_HIP(c, hipMalloc(&c->d_wmask, c->n_dofs * sizeof(double)));
        MFE_HIP(c, hipMalloc(&c->d_cidx, idx.size() * sizeof(int64_t)));
        MFE_HIP(c, hipMemcpy(c->d_cidx, idx.data(), idx.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        std::vector<uint32_t> bits((c->n_dofs + 31) / 32, 0u);
        for (int64_t d : idx) bits[d >> 5] |= 1u << (d & 31);
        MFE_HIP(c, hipMalloc(&c->d_cmask, bits.size() * sizeof(uint32_t)));
        MFE_HIP(c, hipMemcpy(c->d_cmask, bits.data(), bits.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    }
    c->n_con = (int64_t)idx.size();
    c->h_cidx = idx;
    mg_free(c);
    return MFE_OK;
}

// The state update of mfe_set_state without its host wait: the det F check
// is queued into c->d_flag, which the caller reads (and acts on) later.
int set_state_queued(mfe_ctx* c, const double* u, hipStream_t s) {
    MFE_HIP(c, hipMemcpyAsync(c->d_u, u, c->n_dofs * sizeof(double), hipMemcpyDeviceToDevice, s));
    MFE_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    KParams p = base_params(c);
    MFE_HIP(c, mfe::launch_cell_kernel(mfe::MODE_STATE, c->tab, p, s));
    c->state_version++;
    c->cache_valid[1] = c->cache_valid[2] = false;
    c->cache32_valid[1] = c->cache32_valid[2] = false;
    c->has_state = true;
    return MFE_OK;
}

int mfe_set_state(mfe_ctx* c, const double* u, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!u) return fail(c, MFE_EINVAL, "u is null");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    MFE_HIP(c, hipMemcpyAsync(c->d_u, u, c->n_dofs * sizeof(double), hipMemcpyDeviceToDevice, s));
    MFE_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    KParams p = base_params(c);
    MFE_HIP(c, mfe::launch_cell_kernel(mfe::MODE_STATE, c->tab, p, s));
    int flag = 0;
    MFE_HIP(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    MFE_HIP(c, hipStreamSynchronize(s));
    c->state_version++;
    c->cache_valid[1] = c->cache_valid[2] = false;
    c->cache32_valid[1] = c->cache32_valid[2] = false;
    if (flag) {
        c->has_state = false;
        return fail(c, MFE_EJACOBIAN, "det F <= 0 at some quadrature point");
    }
    c->has_state = true;
    return MFE_OK;
}

int mfe_build_cache(mfe_ctx* c, int strategy, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (strategy == MFE_OTF || strategy == MFE_OTF_AD) return MFE_OK;
    const int slot = cache_slot(strategy);
    if (slot < 0) return fail(c, MFE_EINVAL, "unknown strategy");
    if (slot == 1 && c->model != MFE_MODEL_NH)
        return fail(c, MFE_EUNSUPPORTED, "the second-order cache is specific to the neo-Hookean law of eq. hypref");
    if (slot > 0 && !c->has_state) return fail(c, MFE_ESTATE, "no state set");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!c->d_cache[slot]) MFE_HIP(c, hipMalloc(&c->d_cache[slot], (size_t)cache_fields(slot) * c->nq_stride * sizeof(double)));
    KParams p = base_params(c);
    p.cache_out = c->d_cache[slot];
    const int t4 = c->model == MFE_MODEL_SPLIT ? mfe::MODE_BUILD_T4_SPLIT : mfe::MODE_BUILD_T4;
    const int mode = slot == 0 ? mfe::MODE_BUILD_GEOM : (slot == 1 ? mfe::MODE_BUILD_T2 : t4);
    MFE_HIP(c, mfe::launch_cell_kernel(mode, c->tab, p, s));
    c->cache_valid[slot] = true;
    c->cache_version[slot] = c->state_version;
    return MFE_OK;
}

int mfe_build_cache_fp32(mfe_ctx* c, int strategy, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    const int slot = cache_slot(strategy);
    if (strategy == MFE_OTF || strategy == MFE_OTF_AD) return MFE_OK;
    if (slot < 0) return fail(c, MFE_EINVAL, "unknown strategy");
    if (slot == 0) return mfe_build_cache(c, strategy, stream);  // FP32 OTF_GEOM applies read FP64 geometry
    if (slot == 1 && c->model != MFE_MODEL_NH)
        return fail(c, MFE_EUNSUPPORTED, "the second-order cache is specific to the neo-Hookean law of eq. hypref");
    if (!c->has_state) return fail(c, MFE_ESTATE, "no state set");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!c->d_cache32[slot])
        MFE_HIP(c, hipMalloc(&c->d_cache32[slot], (size_t)cache_fields(slot) * c->nq_stride * sizeof(float)));
    KParams p = base_params(c);
    p.cache_out32 = c->d_cache32[slot];
    const int t4 = c->model == MFE_MODEL_SPLIT ? mfe::MODE_BUILD_T4_SPLIT : mfe::MODE_BUILD_T4;
    MFE_HIP(c, mfe::launch_cell_kernel(slot == 1 ? mfe::MODE_BUILD_T2 : t4, c->tab, p, s, true));
    c->cache32_valid[slot] = true;
    c->cache32_version[slot] = c->state_version;
    return MFE_OK;
}

int64_t mfe_cache_bytes(const mfe_ctx* c, int strategy) {
    if (!c || !c->has_mesh) return 0;
    const int slot = cache_slot(strategy);
    if (slot < 0 || !c->d_cache[slot]) return 0;
    return (int64_t)cache_fields(slot) * c->nq_stride * (int64_t)sizeof(double);
}

static int apply_impl(mfe_ctx* c, const void* w, void* v, int strategy, int precision, bool constrained,
                      void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!w || !v) return fail(c, MFE_EINVAL, "null vector");
    if (precision < MFE_FP64 || precision > MFE_SF_BF16X3) return fail(c, MFE_EINVAL, "unknown precision");
    // BF16 / BF16X3: the FP32 path (float vectors, FP32 caches) with the
    // sweeps of w on the matrix cores
    const bool fp32 = precision != MFE_FP64;
    const int sweep = precision == MFE_SF_BF16 ? 1 : precision == MFE_SF_BF16X3 ? 3 : 0;
    if (sweep && c->hex) return fail(c, MFE_EUNSUPPORTED, "matrix-core sweeps are built for structured boxes");
    const int64_t esize = fp32 ? (int64_t)sizeof(float) : (int64_t)sizeof(double);
    if (overlaps(w, v, c->n_dofs * esize)) return fail(c, MFE_EINVAL, "w and v overlap");
    int mode;
    switch (strategy) {
        case MFE_OTF: mode = mfe::MODE_APPLY_OTF; break;
        case MFE_OTF_GEOM: mode = mfe::MODE_APPLY_OTF_GEOM; break;
        case MFE_T2: mode = mfe::MODE_APPLY_T2; break;
        case MFE_T4: mode = mfe::MODE_APPLY_T4; break;
        case MFE_OTF_AD:
            mode = c->model == MFE_MODEL_SPLIT ? mfe::MODE_APPLY_OTF_AD_SPLIT : mfe::MODE_APPLY_OTF_AD;
            break;
        default: return fail(c, MFE_EINVAL, "unknown strategy");
    }
    if (!strategy_supported(c->model, strategy))
        return fail(c, MFE_EUNSUPPORTED, "this strategy is written for the neo-Hookean law of eq. hypref");
    if (!c->has_state) return fail(c, MFE_ESTATE, "no state set");
    const int slot = cache_slot(strategy);
    if (slot == 0 || (slot > 0 && !fp32)) {
        if (!c->cache_valid[slot] || (slot > 0 && c->cache_version[slot] != c->state_version))
            return fail(c, MFE_ESTATE, "cache not built for the current state");
    } else if (slot > 0) {
        if (!c->cache32_valid[slot] || c->cache32_version[slot] != c->state_version)
            return fail(c, MFE_ESTATE, "FP32 cache not built for the current state");
    }
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    KParams p = base_params(c);
    if (slot >= 0) {
        p.cache = c->d_cache[slot];
        p.cache32 = c->d_cache32[slot];
    }
    const bool mask = constrained && c->n_con > 0;
    // the Q2 box kernel reads the constraint bitmap and writes v = w at the
    // constrained dofs itself; the others read a masked copy of w and get the
    // constrained entries of v copied afterwards
    // (the coloured mode always runs it)
    const bool wave = mfe::wave_apply(c->tab.n, mode, c->hex, sweep, fp32, c->deterministic);
    if (c->deterministic && !wave)
        return fail(c, MFE_EUNSUPPORTED, "the coloured apply is built for Q2 structured boxes with vector-ALU sweeps");
    if (fp32) {
        p.w32 = static_cast<const float*>(w);
        p.v32 = static_cast<float*>(v);
        if (mask && !wave) {  // the kernel reads w with the constrained entries zeroed
            float* wm = reinterpret_cast<float*>(c->d_wmask);
            MFE_HIP(c, hipMemcpyAsync(wm, w, c->n_dofs * sizeof(float), hipMemcpyDeviceToDevice, s));
            MFE_HIP(c, mfe::launch_set_indexed(c->d_cidx, c->n_con, 0.0f, wm, s));
            p.w32 = wm;
        }
        MFE_HIP(c, mfe::launch_fill(p.v32, c->n_dofs, 0.0f, s));
    } else {
        p.w = static_cast<const double*>(w);
        p.v = static_cast<double*>(v);
        if (mask && !wave) {
            MFE_HIP(c, hipMemcpyAsync(c->d_wmask, w, c->n_dofs * sizeof(double), hipMemcpyDeviceToDevice, s));
            MFE_HIP(c, mfe::launch_set_indexed(c->d_cidx, c->n_con, 0.0, c->d_wmask, s));
            p.w = c->d_wmask;
        }
        MFE_HIP(c, mfe::launch_fill(p.v, c->n_dofs, 0.0, s));
    }
    if (mask && wave) p.cmask = c->d_cmask;
    // timed applies: the dispatch itself records the kernel's start and end
    // (in the coloured mode the first and the last of the eight launches)
    mfe::LaunchTiming tm;
    const bool timed = c->timing > 0 && c->timing_seq++ % c->timing == 0;
    if (timed) {
        if (c->ev_used == (int)c->ev_start.size()) {
            hipEvent_t a, b;
            MFE_HIP(c, hipEventCreate(&a));
            MFE_HIP(c, hipEventCreate(&b));
            c->ev_start.push_back(a);
            c->ev_stop.push_back(b);
        }
        if (c->deterministic && !c->ev_scratch) MFE_HIP(c, hipEventCreate(&c->ev_scratch));
        tm.start = c->ev_start[c->ev_used];
        tm.stop = c->ev_stop[c->ev_used];
    }
    if (c->deterministic) {
        // the eight parity classes of bricks in a fixed order; bricks of one
        // class share no node, so each launch adds with plain read-add-writes
        int first = 0, last = 0;
        for (int col = 1; col <= 8; ++col)
            if (mfe::colour_bricks(c->nbx, c->nby, c->nbz, col) > 0) {
                if (!first) first = col;
                last = col;
            }
        for (int col = 1; col <= 8; ++col) {
            if (mfe::colour_bricks(c->nbx, c->nby, c->nbz, col) == 0) continue;
            p.colour = col;
            mfe::LaunchTiming tc;
            if (timed && first == last) tc = tm;
            else if (timed && col == first) tc.start = tm.start, tc.stop = c->ev_scratch;
            else if (timed && col == last) tc.start = c->ev_scratch, tc.stop = tm.stop;
            MFE_HIP(c, mfe::launch_cell_kernel(mode, c->tab, p, s, fp32, sweep, tc));
        }
    } else {
        MFE_HIP(c, mfe::launch_cell_kernel(mode, c->tab, p, s, fp32, sweep, tm));
    }
    if (timed) c->ev_used++;
    if (mask && !wave) {
        if (fp32)
            MFE_HIP(c, mfe::launch_copy_indexed(c->d_cidx, c->n_con, static_cast<const float*>(w), p.v32, s));
        else
            MFE_HIP(c, mfe::launch_copy_indexed(c->d_cidx, c->n_con, static_cast<const double*>(w), p.v, s));
    }
    return MFE_OK;
}

int mfe_apply_tangent(mfe_ctx* c, const void* w, void* v, int strategy, int precision, void* stream) {
    return apply_impl(c, w, v, strategy, precision, true, stream);
}

int mfe_energy(mfe_ctx* c, const double* u, double* energy, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!u || !energy) return fail(c, MFE_EINVAL, "null pointer");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nb = (int64_t)c->nbx * c->nby * c->nbz;
    if (!c->d_energy) MFE_HIP(c, hipMalloc(&c->d_energy, (nb + 1) * sizeof(double)));
    if (!c->h_scalars) MFE_HIP(c, hipHostMalloc(&c->h_scalars, 16 * sizeof(double), hipHostMallocDefault));
    KParams p = base_params(c);
    p.u = u;
    p.v = c->d_energy;
    MFE_HIP(c, mfe::launch_cell_kernel(c->model == MFE_MODEL_SPLIT ? mfe::MODE_ENERGY_SPLIT : mfe::MODE_ENERGY,
                                       c->tab, p, s));
    MFE_HIP(c, mfe::launch_sum(c->d_energy, nb, c->d_energy + nb, s));
    MFE_HIP(c, hipMemcpyAsync(c->h_scalars + 3, c->d_energy + nb, sizeof(double), hipMemcpyDeviceToHost, s));
    MFE_HIP(c, hipStreamSynchronize(s));
    *energy = c->h_scalars[3];
    return MFE_OK;
}

int mfe_energy_noalloc(mfe_ctx* c, const double* u, double* energy, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!u || !energy) return fail(c, MFE_EINVAL, "null pointer");
    const int64_t nb = (int64_t)c->nbx * c->nby * c->nbz;
    if (nb > kNoAllocDoubles)
        return fail(c, MFE_EINVAL, "mesh has " + std::to_string(nb) + " bricks of cells; the allocation-free energy "
                                   "holds at most " + std::to_string(kNoAllocDoubles) + " partial sums");
    if (overlaps(u, energy, c->n_dofs * (int64_t)sizeof(double))) return fail(c, MFE_EINVAL, "u and energy overlap");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    KParams p = base_params(c);
    p.u = u;
    p.v = c->d_scratch;  // every partial is written before the sum reads it
    MFE_HIP(c, mfe::launch_cell_kernel(c->model == MFE_MODEL_SPLIT ? mfe::MODE_ENERGY_SPLIT : mfe::MODE_ENERGY,
                                       c->tab, p, s));
    MFE_HIP(c, mfe::launch_sum(c->d_scratch, nb, energy, s));
    return MFE_OK;
}

int mfe_residual(mfe_ctx* c, const double* u, double* r, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!u || !r) return fail(c, MFE_EINVAL, "null vector");
    if (overlaps(u, r, c->n_dofs * (int64_t)sizeof(double))) return fail(c, MFE_EINVAL, "u and r overlap");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    KParams p = base_params(c);
    p.u = u;
    p.v = r;
    MFE_HIP(c, mfe::launch_fill(r, c->n_dofs, 0.0, s));
    MFE_HIP(c, mfe::launch_cell_kernel(c->model == MFE_MODEL_SPLIT ? mfe::MODE_RESIDUAL_SPLIT : mfe::MODE_RESIDUAL,
                                       c->tab, p, s));
    if (c->n_con > 0) MFE_HIP(c, mfe::launch_set_indexed(c->d_cidx, c->n_con, 0.0, r, s));
    return MFE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ solvers
namespace {

int ensure_work(mfe_ctx* c) {
    // 11 vectors: CG r, z, p, Kp, 1/diag; Newton R, du, dg; learned
    // preconditioner N, K z (then K N), r - K z
    if (!c->d_work) MFE_HIP(c, hipMalloc(&c->d_work, 11 * c->n_dofs * sizeof(double)));
    if (!c->d_partials) MFE_HIP(c, hipMalloc(&c->d_partials, (2 * mfe::kDotBlocks + 16) * sizeof(double)));
    if (!c->d_bad) MFE_HIP(c, hipMalloc(&c->d_bad, sizeof(int)));
    if (!c->h_scalars) MFE_HIP(c, hipHostMalloc(&c->h_scalars, 16 * sizeof(double), hipHostMallocDefault));
    return MFE_OK;
}

// two dot products (a.b, x.y) of length n read back to the host
int dotn(mfe_ctx* c, int64_t n, const double* a, const double* b, const double* x, const double* y, hipStream_t s,
         double& ab, double& xy) {
    double* out = c->d_partials + 2 * mfe::kDotBlocks;
    MFE_HIP(c, mfe::launch_dot2(a, b, x, y, n, c->d_partials, out, s));
    MFE_HIP(c, hipMemcpyAsync(c->h_scalars, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    MFE_HIP(c, hipStreamSynchronize(s));
    ab = c->h_scalars[0];
    xy = c->h_scalars[1];
    return MFE_OK;
}

int dot2(mfe_ctx* c, const double* a, const double* b, const double* x, const double* y, hipStream_t s,
         double& ab, double& xy) {
    return dotn(c, c->n_dofs, a, b, x, y, s, ab, xy);
}

int check_opts(mfe_ctx* c, const mfe_solve_opts* o) {
    if (!o) return fail(c, MFE_EINVAL, "null options");
    if (c->model != MFE_MODEL_NH)
        return fail(c, MFE_EUNSUPPORTED, "the solver (diagonal, smoothers) is built for the law of eq. hypref");
    if (o->strategy < MFE_OTF || o->strategy > MFE_OTF_AD) return fail(c, MFE_EINVAL, "unknown strategy");
    if (o->preconditioner < MFE_PC_NONE || o->preconditioner > MFE_PC_GMG_NET)
        return fail(c, MFE_EINVAL, "unknown preconditioner");
    if (o->preconditioner == MFE_PC_GMG || o->preconditioner == MFE_PC_GMG_NET) {
        if (c->hex)
            return fail(c, MFE_EUNSUPPORTED, "geometric multigrid coarsens structured boxes only (mfe_mesh_box)");
        if (o->mg_levels < 0) return fail(c, MFE_EINVAL, "mg_levels must be >= 0");
        if (o->cheb_degree < 1 || o->coarse_degree < 1) return fail(c, MFE_EINVAL, "Chebyshev degrees must be >= 1");
        if (!(o->cheb_range > 1.0) || !(o->coarse_range > 1.0) || !std::isfinite(o->cheb_range) ||
            !std::isfinite(o->coarse_range))
            return fail(c, MFE_EINVAL, "Chebyshev ranges must be finite and > 1");
        if (o->mg_precision != MFE_FP64 && o->mg_precision != MFE_SF_FP32)
            return fail(c, MFE_EINVAL, "mg_precision must be MFE_FP64 or MFE_SF_FP32");
        if (o->mg_graph != 0 && o->mg_graph != 1) return fail(c, MFE_EINVAL, "mg_graph must be 0 or 1");
        if (o->coarse_direct != 0 && o->coarse_direct != 1) return fail(c, MFE_EINVAL, "coarse_direct must be 0 or 1");
        if (o->mg_lag < 0) return fail(c, MFE_EINVAL, "mg_lag must be >= 0");
    }
    if (o->max_cg < 1 || o->max_newton < 1) return fail(c, MFE_EINVAL, "iteration limits must be >= 1");
    if (!(o->cg_rtol > 0.0) || !(o->newton_atol >= 0.0)) return fail(c, MFE_EINVAL, "bad tolerances");
    if (!(o->forcing >= 0.0 && o->forcing < 1.0)) return fail(c, MFE_EINVAL, "forcing must be 0 or in (0, 1)");
    return MFE_OK;
}

// diagonal of K at the current state into d (identity rows at constrained dofs)
int diagonal_into(mfe_ctx* c, double* d, hipStream_t s) {
    if (!c->cache_valid[1] || c->cache_version[1] != c->state_version) {
        const int rc = mfe_build_cache(c, MFE_T2, s);
        if (rc != MFE_OK) return rc;
    }
    MFE_HIP(c, mfe::launch_fill(d, c->n_dofs, 0.0, s));
    KParams p = base_params(c);
    p.cache = c->d_cache[1];
    MFE_HIP(c, mfe::launch_diagonal(c->tab, p, d, s));
    if (c->n_con > 0) MFE_HIP(c, mfe::launch_set_indexed(c->d_cidx, c->n_con, 1.0, d, s));  // identity rows
    return MFE_OK;
}

// ---------------------------------------------------------- multigrid (Sec. 2.3)

// Lagrange basis of the Gauss-Lobatto support points x[0..p] evaluated at t
void lagrange_at(int p, const double* x, double t, double* l) {
    for (int k = 0; k <= p; ++k) {
        double v = 1.0;
        for (int m = 0; m <= p; ++m)
            if (m != k) v *= (t - x[m]) / (x[k] - x[m]);
        l[k] = v;
    }
}

// 1D interpolation between the nodes of two Q_p lines, one with twice the
// cells of the other: row i holds the weights of the `from` nodes that give
// the value at `to` node i (nodal interpolation in the logical coordinate).
void line_interp(int p, int from_cells, int to_cells, std::vector<int>& rowptr, std::vector<int>& col,
                 std::vector<double>& val) {
    double x[8], l[8];
    gll_points(p, x);
    const int rows = p * to_cells + 1;
    rowptr.assign(1, 0);
    col.clear();
    val.clear();
    const double scale = (double)from_cells / to_cells;  // 2 or 1/2: exact
    for (int i = 0; i < rows; ++i) {
        const int ct = std::min(i / p, to_cells - 1);
        const double pos = (ct + x[i - p * ct]) * scale;  // in units of `from` cells
        const int cs = std::min((int)std::floor(pos), from_cells - 1);
        lagrange_at(p, x, pos - cs, l);
        for (int j = 0; j <= p; ++j) {
            double w = l[j];
            if (std::fabs(w) < 1e-14) continue;
            if (std::fabs(w - 1.0) < 1e-14) w = 1.0;
            col.push_back(p * cs + j);
            val.push_back(w);
        }
        rowptr.push_back((int)col.size());
    }
}

int upload_csr(mfe_ctx* c, DevCSR& m, int rows, int cols, const std::vector<int>& rp, const std::vector<int>& ci,
               const std::vector<double>& v) {
    m.rows = rows;
    m.cols = cols;
    MFE_HIP(c, hipMalloc(&m.rowptr, rp.size() * sizeof(int)));
    MFE_HIP(c, hipMalloc(&m.col, std::max<size_t>(ci.size(), 1) * sizeof(int)));
    MFE_HIP(c, hipMalloc(&m.val, std::max<size_t>(v.size(), 1) * sizeof(double)));
    MFE_HIP(c, hipMalloc(&m.valf, std::max<size_t>(v.size(), 1) * sizeof(float)));
    MFE_HIP(c, hipMemcpy(m.rowptr, rp.data(), rp.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!ci.empty()) {
        const std::vector<float> vf(v.begin(), v.end());
        MFE_HIP(c, hipMemcpy(m.col, ci.data(), ci.size() * sizeof(int), hipMemcpyHostToDevice));
        MFE_HIP(c, hipMemcpy(m.val, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
        MFE_HIP(c, hipMemcpy(m.valf, vf.data(), vf.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    return MFE_OK;
}

// transpose of a CSR matrix with `cols` columns
void csr_transpose(int cols, const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<double>& v,
                   std::vector<int>& trp, std::vector<int>& tci, std::vector<double>& tv) {
    const int rows = (int)rp.size() - 1;
    trp.assign(cols + 1, 0);
    for (int e : ci) trp[e + 1]++;
    for (int j = 0; j < cols; ++j) trp[j + 1] += trp[j];
    tci.assign(ci.size(), 0);
    tv.assign(v.size(), 0.0);
    std::vector<int> fill(trp.begin(), trp.end() - 1);
    for (int i = 0; i < rows; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int k = fill[ci[e]]++;
            tci[k] = i;
            tv[k] = v[e];
        }
}

int child_fail(mfe_ctx* c, mfe_ctx* child, int rc, const char* what) {
    return fail(c, rc, std::string("multigrid level setup (") + what + "): " + (child ? child->err : ""));
}

// Nested hierarchy: every coarser level halves the cell counts of the finer
// one (vertices of the coarse box are the even-indexed fine vertices), keeps
// the degree, averages (mu, lambda) over the 8 children, and constrains a
// coarse dof when every fine dof its value is interpolated from is constrained.
int mg_build(mfe_ctx* c, int max_levels) {
    if (!c->mg.empty() && c->mg_request == max_levels) return MFE_OK;
    mg_free(c);
    c->mg_request = max_levels;
    const int p = c->degree;
    std::vector<mfe_ctx*> ctxs{c};
    for (;;) {
        mfe_ctx* f = ctxs.back();
        if (max_levels > 0 && (int)ctxs.size() >= max_levels) break;
        if (f->nx % 2 || f->ny % 2 || f->nz % 2) break;
        const int nx = f->nx / 2, ny = f->ny / 2, nz = f->nz / 2;
        std::vector<double> verts((size_t)(nx + 1) * (ny + 1) * (nz + 1) * 3);
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    const int64_t cv = i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
                    const int64_t fv = 2 * i + (int64_t)(f->nx + 1) * (2 * j + (int64_t)(f->ny + 1) * 2 * k);
                    for (int d = 0; d < 3; ++d) verts[3 * cv + d] = f->h_verts[3 * fv + d];
                }
        mfe_ctx* child = nullptr;
        int rc = mfe_create(&child, c->device);
        if (rc != MFE_OK) return fail(c, rc, "multigrid level setup: mfe_create failed");
        MGLevel L;
        L.ctx = child;
        L.own = true;
        c->mg.push_back(L);  // owned from here on: freed by mg_free on any error
        rc = mfe_mesh_box(child, nx, ny, nz, p, verts.data());
        if (rc != MFE_OK) return child_fail(c, child, rc, "mesh");
        std::vector<double> mat;
        if (!f->h_cellmat.empty()) {
            mat.assign((size_t)2 * child->ne, 0.0);
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        const int64_t ce = i + (int64_t)nx * (j + (int64_t)ny * k);
                        for (int s = 0; s < 8; ++s) {
                            const int64_t fe = (2 * i + (s & 1)) +
                                               (int64_t)f->nx * ((2 * j + ((s >> 1) & 1)) + (int64_t)f->ny * (2 * k + (s >> 2)));
                            mat[2 * ce] += 0.125 * f->h_cellmat[2 * fe];
                            mat[2 * ce + 1] += 0.125 * f->h_cellmat[2 * fe + 1];
                        }
                    }
        }
        rc = mfe_set_material(child, f->mu, f->lam, mat.empty() ? nullptr : mat.data());
        if (rc != MFE_OK) return child_fail(c, child, rc, "material");
        ctxs.push_back(child);
    }
    // level 0 is the context itself
    MGLevel top;
    top.ctx = c;
    top.own = false;
    c->mg.insert(c->mg.begin(), top);
    std::mt19937_64 gen(12345);
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    for (size_t l = 0; l < c->mg.size(); ++l) {
        MGLevel& L = c->mg[l];
        mfe_ctx* f = L.ctx;
        const int64_t n = f->n_dofs;
        MFE_HIP(c, hipMalloc(&L.vec, 8 * n * sizeof(double)));
        double* const v[8] = {L.vec, L.vec + n, L.vec + 2 * n, L.vec + 3 * n,
                              L.vec + 4 * n, L.vec + 5 * n, L.vec + 6 * n, L.vec + 7 * n};
        L.v64.b = v[0];
        L.v64.x = v[1];
        L.v64.r = v[2];
        L.v64.d = v[3];
        L.v64.dinv = v[4];
        L.v64.tmp1 = v[5];
        L.v64.tmp2 = v[6];
        L.rnd = v[7];
        std::vector<double> rnd(n);
        for (auto& v : rnd) v = uni(gen);
        MFE_HIP(c, hipMemcpy(L.rnd, rnd.data(), n * sizeof(double), hipMemcpyHostToDevice));
        if (l + 1 == c->mg.size()) break;
        mfe_ctx* co = c->mg[l + 1].ctx;
        const int fc[3] = {f->nx, f->ny, f->nz}, cc[3] = {co->nx, co->ny, co->nz};
        const int fn[3] = {f->Nx, f->Ny, f->Nz}, cn[3] = {co->Nx, co->Ny, co->Nz};
        std::vector<std::vector<int>> irp(3), ici(3);
        std::vector<std::vector<double>> iv(3);
        for (int a = 0; a < 3; ++a) {
            std::vector<int> rp, ci, trp, tci;
            std::vector<double> v, tv;
            line_interp(p, cc[a], fc[a], rp, ci, v);  // coarse -> fine nodes
            int rc = upload_csr(c, L.P[a], fn[a], cn[a], rp, ci, v);
            if (rc != MFE_OK) return rc;
            csr_transpose(cn[a], rp, ci, v, trp, tci, tv);
            rc = upload_csr(c, L.R[a], cn[a], fn[a], trp, tci, tv);
            if (rc != MFE_OK) return rc;
            line_interp(p, fc[a], cc[a], irp[a], ici[a], iv[a]);  // fine -> coarse nodes
            rc = upload_csr(c, L.I[a], cn[a], fn[a], irp[a], ici[a], iv[a]);
            if (rc != MFE_OK) return rc;
        }
        // coarse constraints
        std::vector<unsigned char> fmask(f->n_dofs, 0);
        for (int64_t d : f->h_cidx) fmask[d] = 1;
        std::vector<int64_t> ccon;
        for (int k = 0; k < cn[2]; ++k)
            for (int j = 0; j < cn[1]; ++j)
                for (int i = 0; i < cn[0]; ++i)
                    for (int comp = 0; comp < 3; ++comp) {
                        bool all = true;
                        for (int ez = irp[2][k]; all && ez < irp[2][k + 1]; ++ez)
                            for (int ey = irp[1][j]; all && ey < irp[1][j + 1]; ++ey)
                                for (int ex = irp[0][i]; all && ex < irp[0][i + 1]; ++ex) {
                                    const int64_t fnode = ici[0][ex] + (int64_t)fn[0] * (ici[1][ey] + (int64_t)fn[1] * ici[2][ez]);
                                    all = fmask[3 * fnode + comp] != 0;
                                }
                        if (all) ccon.push_back(3 * (i + (int64_t)cn[0] * (j + (int64_t)cn[1] * k)) + comp);
                    }
        const int rc = mfe_set_constraints(co, (int64_t)ccon.size(), ccon.data());
        if (rc != MFE_OK) return child_fail(c, co, rc, "constraints");
    }
    return MFE_OK;
}

// FP32 work vectors of every level (first FP32 V-cycle)
int ensure_mg32(mfe_ctx* c) {
    for (auto& L : c->mg) {
        if (L.vec32) continue;
        const int64_t n = L.ctx->n_dofs;
        MFE_HIP(c, hipMalloc(&L.vec32, 7 * n * sizeof(float)));
        float* const v[7] = {L.vec32, L.vec32 + n, L.vec32 + 2 * n, L.vec32 + 3 * n,
                             L.vec32 + 4 * n, L.vec32 + 5 * n, L.vec32 + 6 * n};
        L.v32.b = v[0];
        L.v32.x = v[1];
        L.v32.r = v[2];
        L.v32.d = v[3];
        L.v32.dinv = v[4];
        L.v32.tmp1 = v[5];
        L.v32.tmp2 = v[6];
    }
    return MFE_OK;
}

// out = M_z M_y M_x in for per-axis matrices M (out nodes m[], in nodes n[]),
// through the two scratch arrays t1, t2 (each at least m_x n_y n_z, m_x m_y n_z)
// Fused forms (V-cycle): with rb, the input is read as the free residual
// (dinv != 0) ? rb - in : 0; with x_add, the result is added to x_add where
// dinv_out != 0 and `clear` is zeroed (out is not written).
template <typename T>
int tensor_apply(mfe_ctx* c, const DevCSR* M, const T* in, T* t1, T* t2, T* out, hipStream_t s,
                 const T* rb = nullptr, const T* dinv_in = nullptr, T* x_add = nullptr, const T* dinv_out = nullptr,
                 T* clear = nullptr) {
    const int mx = M[0].rows, my = M[1].rows, mz = M[2].rows;
    const int nx = M[0].cols, ny = M[1].cols, nz = M[2].cols;
    T* tag = nullptr;
    MFE_HIP(c, mfe::launch_axis_csr(M[0].rowptr, M[0].col, M[0].vals(tag), 0, mx, ny, nz, nx, ny, in, t1, s, rb,
                                    dinv_in));
    MFE_HIP(c, mfe::launch_axis_csr(M[1].rowptr, M[1].col, M[1].vals(tag), 1, mx, my, nz, mx, ny, t1, t2, s));
    MFE_HIP(c, mfe::launch_axis_csr(M[2].rowptr, M[2].col, M[2].vals(tag), 2, mx, my, mz, mx, my, t2, out, s,
                                    nullptr, dinv_out, x_add, clear));
    return MFE_OK;
}

template <typename T>
constexpr int precision_of() {
    return std::is_same<T, float>::value ? MFE_SF_FP32 : MFE_FP64;
}

int apply_mode(int strategy) {
    switch (strategy) {
        case MFE_OTF: return mfe::MODE_APPLY_OTF;
        case MFE_OTF_GEOM: return mfe::MODE_APPLY_OTF_GEOM;
        case MFE_T2: return mfe::MODE_APPLY_T2;
        case MFE_T4: return mfe::MODE_APPLY_T4;
        case MFE_OTF_AD: return mfe::MODE_APPLY_OTF_AD;
        default: return -1;
    }
}

// v += K_l w on level l in the V-cycle's precision and the solve's strategy,
// a bare kernel launch: v must hold zeros (or a partial sum), w must vanish
// at the level's constrained dofs, and the rows of v there are not fixed up.
// The level's caches are built by mg_update.
template <typename T>
int level_apply(mfe_ctx* c, const mfe_solve_opts* o, MGLevel& L, const T* w, T* v, hipStream_t s) {
    mfe_ctx* lc = L.ctx;
    KParams p = base_params(lc);
    const int slot = cache_slot(o->strategy);
    if (slot >= 0) {
        p.cache = lc->d_cache[slot];
        p.cache32 = lc->d_cache32[slot];
    }
    constexpr bool fp32 = std::is_same<T, float>::value;
    if constexpr (fp32) {
        p.w32 = w;
        p.v32 = v;
    } else {
        p.w = w;
        p.v = v;
    }
    MFE_HIP(c, mfe::launch_cell_kernel(apply_mode(o->strategy), lc->tab, p, s, fp32));
    return MFE_OK;
}

// Largest eigenvalue of the symmetric tridiagonal matrix (a, b) by bisection
// on the Sturm sequence count.
double tridiag_lmax(const std::vector<double>& a, const std::vector<double>& b) {
    const int m = (int)a.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    // count of eigenvalues < x
    auto below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-12 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) >= m) hi = mid; else lo = mid;
    }
    return hi;
}

// Estimates of lambda_max(D^-1 K) on several levels at once: kLanczosSteps
// steps of Jacobi-preconditioned CG (FP64, second-order cache) from each
// level's fixed random right-hand side; the CG coefficients give the Lanczos
// tridiagonal matrix of D^-1 K, whose largest eigenvalue approaches
// lambda_max from below (the smoothers use 1.2 times it).  Each level's
// steps run on a stream of its own (the levels are independent, and their
// short kernels overlap), with alpha and beta formed on the device; the dot
// products stay in a device history per level (hp + 2k: p.Ap of step k;
// hr + 2k: (r.r, r.z) before step k), which the host reads once, for all
// levels, and replays with the same arithmetic.  A level whose CG finds an
// invariant subspace stops there (later steps only do discarded work).
constexpr int kLanczosSteps = 8;
constexpr int kLzHist = 2 * (kLanczosSteps + 1);

int lanczos_levels(mfe_ctx* c, const std::vector<MGLevel*>& levels, hipStream_t s) {
    const size_t nlev = levels.size();
    if (nlev == 0) return MFE_OK;
    if (nlev > c->lz_levels) {
        dfree(c->d_lz);
        dfree(c->d_lz_part);
        if (c->h_lz) (void)hipHostFree(c->h_lz);
        c->h_lz = nullptr;
        c->lz_levels = 0;
        MFE_HIP(c, hipMalloc(&c->d_lz, nlev * 2 * kLzHist * sizeof(double)));
        MFE_HIP(c, hipMalloc(&c->d_lz_part, nlev * 2 * mfe::kDotBlocks * sizeof(double)));
        MFE_HIP(c, hipHostMalloc(&c->h_lz, nlev * 2 * kLzHist * sizeof(double), hipHostMallocDefault));
        c->lz_levels = nlev;
    }
    while (c->lz_streams.size() < nlev) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        MFE_HIP(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        c->lz_streams.push_back(st);
        MFE_HIP(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        c->lz_join.push_back(ev);
    }
    if (!c->lz_fork) MFE_HIP(c, hipEventCreateWithFlags(&c->lz_fork, hipEventDisableTiming));
    // the levels are independent: each runs its steps on a stream of its own
    // (forked from s, joined back into s), with its own partial-sum scratch
    struct Join {
        mfe_ctx* c;
        size_t n = 0;
        ~Join() {  // an early return leaves no level work behind
            for (size_t i = 0; i < n; ++i) (void)hipStreamSynchronize(c->lz_streams[i]);
        }
    } join{c};
    MFE_HIP(c, hipEventRecord(c->lz_fork, s));
    for (size_t i = 0; i < nlev; ++i) {
        MGLevel& L = *levels[i];
        const hipStream_t ls = c->lz_streams[i];
        MFE_HIP(c, hipStreamWaitEvent(ls, c->lz_fork, 0));
        join.n = i + 1;
        const int64_t n = L.ctx->n_dofs;
        double* part = c->d_lz_part + i * 2 * mfe::kDotBlocks;
        double* x = L.v64.x;
        double* r = L.v64.b;
        double* z = L.v64.tmp1;
        double* pv = L.v64.d;
        double* Ap = L.v64.r;
        double* hp = c->d_lz + i * 2 * kLzHist;
        double* hr = hp + kLzHist;
        MFE_HIP(c, mfe::launch_fill(x, n, 0.0, ls));
        MFE_HIP(c, mfe::launch_scale_mul(1.0, nullptr, L.rnd, r, n, ls));
        MFE_HIP(c, mfe::launch_scale_mul(1.0, L.v64.dinv, r, z, n, ls));
        MFE_HIP(c, mfe::launch_scale_mul(1.0, nullptr, z, pv, n, ls));
        MFE_HIP(c, mfe::launch_dot2(r, r, r, z, n, part, hr, ls));
        for (int k = 0; k < kLanczosSteps && k < n; ++k) {
            int rc = mfe_apply_tangent(L.ctx, pv, Ap, MFE_T2, MFE_FP64, ls);
            if (rc != MFE_OK) return L.ctx != c ? child_fail(c, L.ctx, rc, "apply") : rc;
            MFE_HIP(c, mfe::launch_dot2(pv, Ap, nullptr, nullptr, n, part, hp + 2 * k, ls));
            MFE_HIP(c, mfe::launch_cg_update_dev(x, r, z, pv, Ap, L.v64.dinv, hr + 2 * k + 1, hp + 2 * k, n, part,
                                                 hr + 2 * (k + 1), ls));
            MFE_HIP(c, mfe::launch_p_update_dev(z, hr + 2 * (k + 1) + 1, hr + 2 * k + 1, pv, n, ls));
        }
        MFE_HIP(c, hipEventRecord(c->lz_join[i], ls));
        MFE_HIP(c, hipStreamWaitEvent(s, c->lz_join[i], 0));
    }
    MFE_HIP(c, hipMemcpyAsync(c->h_lz, c->d_lz, nlev * 2 * kLzHist * sizeof(double), hipMemcpyDeviceToHost, s));
    MFE_HIP(c, hipStreamSynchronize(s));
    for (size_t i = 0; i < nlev; ++i) {
        MGLevel& L = *levels[i];
        const int m = (int)std::min<int64_t>(kLanczosSteps, L.ctx->n_dofs);
        const double* Hp = c->h_lz + i * 2 * kLzHist;
        const double* Hr = Hp + kLzHist;
        std::vector<double> diag, off;
        double alpha_prev = 0.0, beta_prev = 0.0;
        for (int j = 0; j < m; ++j) {
            const double rz = Hr[2 * j + 1], pAp = Hp[2 * j], rz_new = Hr[2 * (j + 1) + 1];
            if (!(pAp > 0.0) || !std::isfinite(pAp))
                return fail(c, MFE_ENOTCONV, "eigenvalue estimate: level tangent is not positive definite");
            const double alpha = rz / pAp;
            diag.push_back(1.0 / alpha + (j > 0 ? beta_prev / alpha_prev : 0.0));
            if (!(rz_new > 1e-30 * rz)) break;  // invariant subspace found
            const double beta = rz_new / rz;
            if (j + 1 < m) off.push_back(std::sqrt(beta) / alpha);
            alpha_prev = alpha;
            beta_prev = beta;
        }
        off.resize(diag.size() > 0 ? diag.size() - 1 : 0);
        const double lmax = tridiag_lmax(diag, off);
        if (!(lmax > 0.0) || !std::isfinite(lmax)) return fail(c, MFE_ENOTCONV, "eigenvalue estimate failed");
        L.lmax = lmax;
    }
    return MFE_OK;
}

// Per linearisation point: interpolate the state to every coarser level,
// build the level caches (in the V-cycle's precision), the inverse diagonals
// and an estimate of the largest eigenvalue of D^-1 K.
// Inverse of the coarsest level's tangent on its free dofs, from its
// second-order cache, which must be current.  ok = false when there are
// more than kDenseMax free dofs or the tangent is not positive definite
// (then the level is smoothed instead).
// Launch half (on stream s): assembly and sweep inversion, the pivot check
// into c->d_bad_dense; returns with launched = false when the level has no
// or too many free dofs.  The finish half reads the check.
int dense_launch(mfe_ctx* c, MGLevel& L, hipStream_t s, bool& launched) {
    launched = false;
    mfe_ctx* lc = L.ctx;
    const int n = (int)lc->n_dofs;
    if (!L.dense) {  // the constraints of a level are fixed for the life of the hierarchy
        std::vector<int> pos(n, 0), free_idx;
        for (int64_t d : lc->h_cidx) pos[d] = -1;
        for (int d = 0; d < n; ++d)
            if (pos[d] == 0) {
                pos[d] = (int)free_idx.size();
                free_idx.push_back(d);
            }
        L.dense_nf = (int)free_idx.size();
        if (L.dense_nf == 0 || L.dense_nf > mfe::kDenseMax) return MFE_OK;
        const size_t nf2 = (size_t)L.dense_nf * L.dense_nf;
        MFE_HIP(c, hipMalloc(&L.dense, (nf2 + (size_t)n * n) * sizeof(double)));
        MFE_HIP(c, hipMalloc(&L.dense_pos, n * sizeof(int)));
        MFE_HIP(c, hipMalloc(&L.dense_free, L.dense_nf * sizeof(int)));
        MFE_HIP(c, hipMemcpy(L.dense_pos, pos.data(), n * sizeof(int), hipMemcpyHostToDevice));
        MFE_HIP(c, hipMemcpy(L.dense_free, free_idx.data(), L.dense_nf * sizeof(int), hipMemcpyHostToDevice));
    }
    const int nf = L.dense_nf;
    const size_t nf2 = (size_t)nf * nf;
    double* A = L.dense + nf2;
    MFE_HIP(c, mfe::launch_fill(A, (int64_t)n * n, 0.0, s));
    KParams p = base_params(lc);
    p.cache = lc->d_cache[1];
    MFE_HIP(c, mfe::launch_dense_tangent(lc->tab, p, A, n, s));
    if (!c->d_bad_dense) MFE_HIP(c, hipMalloc(&c->d_bad_dense, sizeof(int)));
    MFE_HIP(c, mfe::launch_sweep_inverse(A, n, L.dense_free, nf, L.dense, c->d_bad_dense, s));
    launched = true;
    return MFE_OK;
}

int dense_finish(mfe_ctx* c, MGLevel& L, bool fp32, hipStream_t s, bool& ok) {
    const size_t nf2 = (size_t)L.dense_nf * L.dense_nf;
    int bad = 1;
    MFE_HIP(c, hipMemcpyAsync(&bad, c->d_bad_dense, sizeof(int), hipMemcpyDeviceToHost, s));
    MFE_HIP(c, hipStreamSynchronize(s));
    ok = bad == 0;
    if (ok && fp32) {
        if (!L.dense32) MFE_HIP(c, hipMalloc(&L.dense32, nf2 * sizeof(float)));
        MFE_HIP(c, mfe::launch_convert(L.dense, L.dense32, (int64_t)nf2, s));
    }
    return MFE_OK;
}

const double* dense_of(const MGLevel& L, double*) { return L.dense; }
const float* dense_of(const MGLevel& L, float*) { return L.dense32; }

// The coarsest level's direct-solve set-up (one workgroup, ~0.6 ms) runs on
// the side stream while the other levels' eigenvalue estimates run on s; a
// failed pivot check falls back to smoothing that level.
int mg_spectra(mfe_ctx* c, const mfe_solve_opts* o, bool fp32, hipStream_t s) {
    const size_t nl = c->mg.size();
    MGLevel& Lc = c->mg[nl - 1];
    for (MGLevel& L : c->mg) L.dense_ok = false;
    bool dense = false;
    // an early return leaves no side-stream work behind
    struct SideGuard {
        hipStream_t side = nullptr;
        ~SideGuard() {
            if (side) (void)hipStreamSynchronize(side);
        }
    } guard;
    {
        const int64_t n_free = Lc.ctx->n_dofs - Lc.ctx->n_con;
        if (o->coarse_direct && Lc.ctx->n_dofs <= 1024 && n_free > 0 && n_free <= mfe::kDenseMax) {
            if (!c->side_stream) MFE_HIP(c, hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
            if (!c->side_fork) MFE_HIP(c, hipEventCreateWithFlags(&c->side_fork, hipEventDisableTiming));
            if (!c->side_join) MFE_HIP(c, hipEventCreateWithFlags(&c->side_join, hipEventDisableTiming));
            MFE_HIP(c, hipEventRecord(c->side_fork, s));
            MFE_HIP(c, hipStreamWaitEvent(c->side_stream, c->side_fork, 0));
            guard.side = c->side_stream;
            const int rc = dense_launch(c, Lc, c->side_stream, dense);
            if (rc != MFE_OK) return rc;
            MFE_HIP(c, hipEventRecord(c->side_join, c->side_stream));
        }
    }
    {
        // spectrum estimates of the smoothed levels, all at once (the
        // coarsest one too unless its direct solve is being set up)
        std::vector<MGLevel*> est;
        for (size_t l = 0; l + 1 < nl; ++l) est.push_back(&c->mg[l]);
        if (!dense) est.push_back(&Lc);
        int rc = lanczos_levels(c, est, s);
        if (rc != MFE_OK) return rc;
        if (dense) {
            MFE_HIP(c, hipStreamWaitEvent(s, c->side_join, 0));
            rc = dense_finish(c, Lc, fp32, s, Lc.dense_ok);
            if (rc != MFE_OK) return rc;
            guard.side = nullptr;  // joined: dense_finish waited for it
            if (Lc.dense_ok) {
                Lc.lmax = 0.0;  // solved, not smoothed: no spectrum estimate needed
            } else {
                rc = lanczos_levels(c, std::vector<MGLevel*>{&Lc}, s);
                if (rc != MFE_OK) return rc;
            }
        }
    }
    return MFE_OK;
}

int mg_update(mfe_ctx* c, const mfe_solve_opts* o, hipStream_t s) {
    const bool cached = o->strategy != MFE_OTF && o->strategy != MFE_OTF_AD;
    const bool fp32 = o->mg_precision == MFE_SF_FP32;
    if (fp32) {
        const int rc = ensure_mg32(c);
        if (rc != MFE_OK) return rc;
    }
    for (size_t l = 0; l < c->mg.size(); ++l) {
        MGLevel& L = c->mg[l];
        mfe_ctx* lc = L.ctx;
        int rc;
        if (l > 0) {
            MGLevel& F = c->mg[l - 1];
            rc = tensor_apply(c, F.I, static_cast<const double*>(F.ctx->d_u), F.v64.tmp1, F.v64.tmp2, L.v64.x, s);
            if (rc != MFE_OK) return rc;
            // the coarse states' det F checks are read with the diagonals' below
            rc = set_state_queued(lc, L.v64.x, s);
            if (rc != MFE_OK) return child_fail(c, lc, rc, "state");
        }
        if (cached) {
            const int slot = cache_slot(o->strategy);
            if (fp32) {
                rc = mfe_build_cache_fp32(lc, o->strategy, s);
            } else if (l > 0 || !lc->cache_valid[slot] || (slot > 0 && lc->cache_version[slot] != lc->state_version)) {
                rc = mfe_build_cache(lc, o->strategy, s);
            } else {
                rc = MFE_OK;
            }
            if (rc != MFE_OK) return l ? child_fail(c, lc, rc, "cache") : rc;
        }
        rc = diagonal_into(lc, L.v64.dinv, s);
        if (rc != MFE_OK) return l ? child_fail(c, lc, rc, "diagonal") : rc;
        if (l == 0) MFE_HIP(c, hipMemsetAsync(c->d_bad, 0, sizeof(int), s));
        MFE_HIP(c, mfe::launch_invert(L.v64.dinv, lc->n_dofs, c->d_bad, s));  // every level flags into d_bad
    }
    {
        // one host wait for every level: the coarse states' det F flags, then
        // the diagonals' flag
        const size_t nlv = c->mg.size();
        std::vector<int> flags(nlv + 1, 0);
        for (size_t l = 1; l < nlv; ++l)
            MFE_HIP(c, hipMemcpyAsync(&flags[l], c->mg[l].ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        MFE_HIP(c, hipMemcpyAsync(&flags[nlv], c->d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
        MFE_HIP(c, hipStreamSynchronize(s));
        for (size_t l = 1; l < nlv; ++l)
            if (flags[l]) {
                mfe_ctx* lc = c->mg[l].ctx;
                lc->has_state = false;
                fail(lc, MFE_EJACOBIAN, "det F <= 0 at some quadrature point");
                return child_fail(c, lc, MFE_EJACOBIAN, "state");
            }
        if (flags[nlv]) return fail(c, MFE_EJACOBIAN, "level tangent diagonal is not positive: no Chebyshev-Jacobi smoother");
    }
    // A lagged set-up keeps the spectrum estimates and the coarse inverse of
    // the last full one (same V-cycle precision and coarse mode); the level
    // operators, caches and diagonals above are always the current ones.
    const size_t nl = c->mg.size();
    const bool lag = o->mg_lag > 0 && c->mg_lag_left > 0 && c->mg_lag_prec == o->mg_precision &&
                     c->mg_lag_direct == o->coarse_direct;
    if (lag) {
        --c->mg_lag_left;
    } else {
        c->mg_lag_left = 0;
        const int rc = mg_spectra(c, o, fp32, s);
        if (rc != MFE_OK) return rc;
        c->mg_lag_left = o->mg_lag;
        c->mg_lag_prec = o->mg_precision;
        c->mg_lag_direct = o->coarse_direct;
    }
    for (size_t l = 0; l < nl; ++l) {
        MGLevel& L = c->mg[l];
        mfe_ctx* lc = L.ctx;
        // the V-cycle works on the free dofs: the smoother never moves a
        // constrained entry, and its operator-output buffer starts cleared
        if (lc->n_con > 0) MFE_HIP(c, mfe::launch_set_indexed(lc->d_cidx, lc->n_con, 0.0, L.v64.dinv, s));
        MFE_HIP(c, mfe::launch_fill(L.v64.r, lc->n_dofs, 0.0, s));
        if (fp32) {
            MFE_HIP(c, mfe::launch_convert(L.v64.dinv, L.v32.dinv, lc->n_dofs, s));
            MFE_HIP(c, mfe::launch_fill(L.v32.r, lc->n_dofs, 0.0f, s));
        }
    }
    c->mg_graph_valid = false;  // smoother coefficients changed
    c->mg_ready_version = c->state_version;
    c->mg_ready_strategy = o->strategy;
    c->mg_ready_prec = o->mg_precision;
    c->mg_ready_opts = *o;
    return MFE_OK;
}

int net_smooth(mfe_ctx* c, const mfe_solve_opts* o, MGLevel& L, const double* b, double* x, hipStream_t s);

// x = x + p(D^-1 K) D^-1 (b - K x): `degree` Chebyshev-Jacobi steps on
// [lmax / range, lmax] with lmax 1.2 times the estimate (x = 0 on entry when
// zero_start, which saves one operator application).  On the free dofs only:
// dinv is 0 at constrained dofs, so x stays 0 there.  The operator output V.r
// is zero on entry and on exit (each step clears it after use).
template <typename T>
int chebyshev(mfe_ctx* c, const mfe_solve_opts* o, MGLevel& L, const T* b, T* x, int degree, double range,
              bool zero_start, hipStream_t s) {
    MGVec<T>& V = L.vecs(static_cast<T*>(nullptr));
    const int64_t n = L.ctx->n_dofs;
    const double hi = 1.2 * L.lmax, lo = hi / range;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    int rc;
    if (zero_start) {  // x = d: no separate clearing of x
        MFE_HIP(c, mfe::launch_cheb(V.d, x, b, static_cast<T*>(nullptr), V.dinv, T(0), T(1.0 / theta), n, s, true));
    } else {
        rc = level_apply(c, o, L, static_cast<const T*>(x), V.r, s);
        if (rc != MFE_OK) return rc;
        MFE_HIP(c, mfe::launch_cheb(V.d, x, b, V.r, V.dinv, T(0), T(1.0 / theta), n, s));
    }
    for (int k = 1; k < degree; ++k) {
        rc = level_apply(c, o, L, static_cast<const T*>(x), V.r, s);
        if (rc != MFE_OK) return rc;
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        MFE_HIP(c, mfe::launch_cheb(V.d, x, b, V.r, V.dinv, T(rho_new * rho), T(2.0 * rho_new / delta), n, s));
        rho = rho_new;
    }
    return MFE_OK;
}

// one V-cycle x = V_l b on the free dofs of level l (x need not be
// initialised; b is not read at constrained dofs; x is 0 there on exit)
template <typename T>
int vcycle(mfe_ctx* c, const mfe_solve_opts* o, size_t l, const T* b, T* x, hipStream_t s) {
    MGLevel& L = c->mg[l];
    MGVec<T>& V = L.vecs(static_cast<T*>(nullptr));
    if (l + 1 == c->mg.size()) {
        if (L.dense_ok) {
            MFE_HIP(c, mfe::launch_dense_matvec(dense_of(L, static_cast<T*>(nullptr)), L.dense_pos, L.dense_free,
                                                L.dense_nf, b, x, (int)L.ctx->n_dofs, s));
            return MFE_OK;
        }
        return chebyshev(c, o, L, b, x, o->coarse_degree, o->coarse_range, true, s);
    }
    int rc = chebyshev(c, o, L, b, x, o->cheb_degree, o->cheb_range, true, s);
    if (rc != MFE_OK) return rc;
    // K x into V.r; the restriction forms the free residual b - K x on the fly
    rc = level_apply(c, o, L, static_cast<const T*>(x), V.r, s);
    if (rc != MFE_OK) return rc;
    MGLevel& C = c->mg[l + 1];
    MGVec<T>& CV = C.vecs(static_cast<T*>(nullptr));
    rc = tensor_apply(c, L.R, static_cast<const T*>(V.r), V.tmp1, V.tmp2, CV.b, s, b,
                      static_cast<const T*>(V.dinv));
    if (rc != MFE_OK) return rc;
    rc = vcycle(c, o, l + 1, static_cast<const T*>(CV.b), CV.x, s);
    if (rc != MFE_OK) return rc;
    // x += prolongated correction on the free dofs; V.r cleared for the smoother
    rc = tensor_apply(c, L.P, static_cast<const T*>(CV.x), V.tmp1, V.tmp2, static_cast<T*>(nullptr), s,
                      static_cast<const T*>(nullptr), static_cast<const T*>(nullptr), x,
                      static_cast<const T*>(V.dinv), V.r);
    if (rc != MFE_OK) return rc;
    if constexpr (std::is_same<T, double>::value) {
        if (l == 0 && c->net_in_cycle) {  // the learned step takes the last post-smoothing step's place
            if (o->cheb_degree > 1) {
                rc = chebyshev(c, o, L, b, x, o->cheb_degree - 1, o->cheb_range, false, s);
                if (rc != MFE_OK) return rc;
            }
            return net_smooth(c, o, L, b, x, s);
        }
    }
    return chebyshev(c, o, L, b, x, o->cheb_degree, o->cheb_range, false, s);
}

// The whole preconditioner application z = B r as one kernel sequence (no
// host synchronisation): B is the V-cycle on the free dofs and the identity
// on the constrained ones (exact for the identity rows of K).
int gmg_body(mfe_ctx* c, const mfe_solve_opts* o, const double* r, double* z, hipStream_t s) {
    MGLevel& L = c->mg[0];
    const int64_t n = c->n_dofs;
    int rc;
    if (o->mg_precision == MFE_SF_FP32) {
        MFE_HIP(c, mfe::launch_convert(r, L.v32.b, n, s));
        rc = vcycle(c, o, 0, static_cast<const float*>(L.v32.b), L.v32.x, s);
        if (rc != MFE_OK) return rc;
        MFE_HIP(c, mfe::launch_convert(static_cast<const float*>(L.v32.x), z, n, s));
    } else {
        rc = vcycle(c, o, 0, r, z, s);
        if (rc != MFE_OK) return rc;
    }
    if (c->n_con > 0) MFE_HIP(c, mfe::launch_copy_indexed(c->d_cidx, c->n_con, r, z, s));
    return MFE_OK;
}

// z = B r, replayed from a HIP graph of gmg_body when opts->mg_graph is set
// (captured once per hierarchy update and (r, z, precision)), else launched
// kernel by kernel.  The graph holds kernel nodes only.
int gmg_apply(mfe_ctx* c, const mfe_solve_opts* o, const double* r, double* z, hipStream_t s) {
    if (!o->mg_graph) return gmg_body(c, o, r, z, s);
    const mfe_solve_opts& go = c->mg_graph_opts;
    const bool same = go.cheb_degree == o->cheb_degree && go.cheb_range == o->cheb_range &&
                      go.coarse_degree == o->coarse_degree && go.coarse_range == o->coarse_range &&
                      go.coarse_direct == o->coarse_direct && go.strategy == o->strategy &&
                      c->mg_graph_net == c->net_in_cycle;
    if (!c->mg_graph_valid || !same || c->mg_graph_r != r || c->mg_graph_z != z ||
        c->mg_graph_prec != o->mg_precision) {
        if (c->mg_exec) {
            (void)hipGraphExecDestroy(c->mg_exec);
            c->mg_exec = nullptr;
        }
        if (!c->mg_stream) MFE_HIP(c, hipStreamCreateWithFlags(&c->mg_stream, hipStreamNonBlocking));
        MFE_HIP(c, hipStreamBeginCapture(c->mg_stream, hipStreamCaptureModeThreadLocal));
        const int rc = gmg_body(c, o, r, z, c->mg_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(c->mg_stream, &graph);
        if (rc != MFE_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        const hipError_t ei = hipGraphInstantiate(&c->mg_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            c->mg_exec = nullptr;
            return hip_fail(c, ei, "hipGraphInstantiate");
        }
        c->mg_graph_valid = true;
        c->mg_graph_r = r;
        c->mg_graph_z = z;
        c->mg_graph_prec = o->mg_precision;
        c->mg_graph_opts = *o;
        c->mg_graph_net = c->net_in_cycle;
    }
    MFE_HIP(c, hipGraphLaunch(c->mg_exec, s));
    return MFE_OK;
}


// ------------------------------------------------------- learned correction
// Network layout: conv 6->32 (ReLU), conv 32->32 (ReLU), conv 32->3, 3x3x3
// kernels on the 9^3 nodes of a patch of 4^3 Q2 cells; W[co][ci][27] then
// bias[co] per layer.
constexpr int kNetW1 = 0, kNetB1 = 5184, kNetW2 = 5216, kNetB2 = 32864, kNetW3 = 32896, kNetB3 = 35488;
constexpr int kNetParams = 35491;
constexpr int64_t kPatchVox = 729;

int patch_dims(const mfe_ctx* c, int& npx, int& npy, int& npz) {
    npx = npy = npz = 0;
    if (!c->has_mesh || c->hex || c->degree != 2 || c->nx % 4 || c->ny % 4 || c->nz % 4) return 0;
    npx = c->nx / 4;
    npy = c->ny / 4;
    npz = c->nz / 4;
    return npx * npy * npz;
}

// variant MFE_NET_RELU: ReLU after layers 1 and 2, biases; MFE_NET_LINEAR:
// neither (the biases are not read), so y is a linear function of x
hipError_t net_forward(const float* prm, const float* x, int P, int variant, float* act, float* y, hipStream_t s) {
    const bool nl = variant == MFE_NET_RELU;
    float* a1 = act;
    float* a2 = act + (int64_t)P * 32 * kPatchVox;
    hipError_t e = mfe::launch_conv3d(x, prm + kNetW1, nl ? prm + kNetB1 : nullptr, P, 6, 32, false, nl, nullptr, a1, s);
    if (e == hipSuccess)
        e = mfe::launch_conv3d(a1, prm + kNetW2, nl ? prm + kNetB2 : nullptr, P, 32, 32, false, nl, nullptr, a2, s);
    if (e == hipSuccess)
        e = mfe::launch_conv3d(a2, prm + kNetW3, nl ? prm + kNetB3 : nullptr, P, 32, 3, false, false, nullptr, y, s);
    return e;
}

hipError_t net_backward(const float* prm, const float* x, const float* act, const float* dy, int P, int variant,
                        float* work, float* grad, hipStream_t s) {
    const bool nl = variant == MFE_NET_RELU;
    const float* a1 = act;
    const float* a2 = act + (int64_t)P * 32 * kPatchVox;
    float* d1 = work;
    float* d2 = work + (int64_t)P * 32 * kPatchVox;
    hipError_t e = mfe::launch_conv3d_wgrad(a2, dy, P, 32, 3, grad + kNetW3, grad + kNetB3, s);
    if (e == hipSuccess) e = mfe::launch_conv3d(dy, prm + kNetW3, nullptr, P, 3, 32, true, false, nl ? a2 : nullptr, d2, s);
    if (e == hipSuccess) e = mfe::launch_conv3d_wgrad(a1, d2, P, 32, 32, grad + kNetW2, grad + kNetB2, s);
    if (e == hipSuccess) e = mfe::launch_conv3d(d2, prm + kNetW2, nullptr, P, 32, 32, true, false, nl ? a1 : nullptr, d1, s);
    if (e == hipSuccess) e = mfe::launch_conv3d_wgrad(x, d1, P, 6, 32, grad + kNetW1, grad + kNetB1, s);
    if (e == hipSuccess && !nl) {  // biases are not part of the linear variant
        e = mfe::launch_fill(grad + kNetB1, 32, 0.0f, s);
        if (e == hipSuccess) e = mfe::launch_fill(grad + kNetB2, 32, 0.0f, s);
        if (e == hipSuccess) e = mfe::launch_fill(grad + kNetB3, 3, 0.0f, s);
    }
    return e;
}

// node invariants (I1, I2, J of C = F^T F) of the current state
int ensure_node_invariants(mfe_ctx* c, hipStream_t s) {
    if (c->ninv_valid && c->ninv_version == c->state_version) return MFE_OK;
    if (!c->has_state) return fail(c, MFE_ESTATE, "no state set");
    if (!c->d_ninv) MFE_HIP(c, hipMalloc(&c->d_ninv, 3 * c->n_nodes * sizeof(float)));
    if (!c->d_cinv) MFE_HIP(c, hipMalloc(&c->d_cinv, 3 * c->ne * sizeof(float)));
    MFE_HIP(c, mfe::launch_node_invariants(c->d_u, c->d_verts, c->nx, c->ny, c->nz, c->Nx, c->Ny, c->Nz, c->d_cinv,
                                           c->d_ninv, s));
    c->ninv_valid = true;
    c->ninv_version = c->state_version;
    return MFE_OK;
}

// Buffers and state data of the learned step, set up outside the V-cycle
// (which may be captured in a graph): the node invariants of the current
// state, the per-patch buffers and the device slots of its two dots.
int net_prepare(mfe_ctx* c, hipStream_t s) {
    int npx, npy, npz;
    const int P = patch_dims(c, npx, npy, npz);
    if (!c->d_net) return fail(c, MFE_EINVAL, "no network set (mfe_set_network)");
    if (P == 0) return fail(c, MFE_EUNSUPPORTED, "the learned correction needs Q2 and cell counts divisible by 4");
    int rc = ensure_node_invariants(c, s);
    if (rc != MFE_OK) return rc;
    const int64_t per = (int64_t)P * kPatchVox;
    if (!c->d_nbuf) MFE_HIP(c, hipMalloc(&c->d_nbuf, ((6 + 64 + 3) * per + P) * sizeof(float)));
    if (!c->d_netdot) MFE_HIP(c, hipMalloc(&c->d_netdot, 2 * sizeof(double)));
    return MFE_OK;
}

// The learned step of the finest level's post-smoother (in place of its last
// Chebyshev step): r1 = b - K x, the residual the earlier smoothing left on
// the free dofs; N = the network's correction of r1 (features of every
// patch, the network, the patch-averaged scatter, 0 at constrained dofs);
// x += alpha N with alpha = N.r1 / N.K N, the step that minimises the energy
// norm of the error along N (no step unless both dots are positive).  The
// dots stay on the device and alpha is formed there, so the V-cycle remains
// one kernel sequence without host synchronisation.
int net_smooth(mfe_ctx* c, const mfe_solve_opts* o, MGLevel& L, const double* b, double* x, hipStream_t s) {
    int npx, npy, npz;
    const int P = patch_dims(c, npx, npy, npz);
    const int64_t n = c->n_dofs;
    double* N = c->d_work + 8 * n;    // the correction
    double* Kv = c->d_work + 9 * n;   // K x, then K N
    double* r1 = c->d_work + 10 * n;  // b - K x
    const int64_t per = (int64_t)P * kPatchVox;
    float* feat = c->d_nbuf;
    float* act = feat + 6 * per;
    float* y = act + 64 * per;
    float* scale = y + 3 * per;
    MFE_HIP(c, mfe::launch_fill(Kv, n, 0.0, s));
    int rc = level_apply(c, o, L, static_cast<const double*>(x), Kv, s);
    if (rc != MFE_OK) return rc;
    MFE_HIP(c, mfe::launch_copy(b, r1, n, s));
    MFE_HIP(c, mfe::launch_axpby(-1.0, Kv, 1.0, r1, n, s));
    if (c->n_con > 0) MFE_HIP(c, mfe::launch_set_indexed(c->d_cidx, c->n_con, 0.0, r1, s));
    const bool linear = c->net_variant == MFE_NET_LINEAR;
    MFE_HIP(c, mfe::launch_patch_features(r1, c->d_ninv, c->Nx, c->Ny, npx, npy, P, linear, feat, scale, s));
    MFE_HIP(c, net_forward(c->d_net, feat, P, c->net_variant, act, y, s));
    MFE_HIP(c, mfe::launch_fill(N, n, 0.0, s));
    MFE_HIP(c, mfe::launch_patch_scatter(y, scale, c->Nx, c->Ny, c->Nz, npx, npy, npz, 1.0, N, s));
    if (c->n_con > 0) MFE_HIP(c, mfe::launch_set_indexed(c->d_cidx, c->n_con, 0.0, N, s));
    MFE_HIP(c, mfe::launch_fill(Kv, n, 0.0, s));
    rc = level_apply(c, o, L, static_cast<const double*>(N), Kv, s);
    if (rc != MFE_OK) return rc;
    MFE_HIP(c, mfe::launch_dot2(N, r1, N, Kv, n, c->d_partials, c->d_netdot, s));
    MFE_HIP(c, mfe::launch_axpy_ratio(c->d_netdot, N, x, n, s));
    return MFE_OK;
}

// z = B r (GMG V-cycle, with the learned step in its finest post-smoother
// when `net`), then r.z > 0
int precondition(mfe_ctx* c, const mfe_solve_opts* o, bool net, const double* r, double* z, hipStream_t s,
                 double& rz) {
    c->net_in_cycle = net;
    int rc = gmg_apply(c, o, r, z, s);
    c->net_in_cycle = false;
    if (rc != MFE_OK) return rc;
    double unused;
    rc = dot2(c, r, z, nullptr, nullptr, s, rz, unused);
    if (rc != MFE_OK) return rc;
    if (!(rz > 0.0)) return fail(c, MFE_ENOTCONV, "preconditioner is not positive definite");
    return MFE_OK;
}

// Flexible CG (truncated, the last kMaxDirs directions kept K-orthogonal)
// for the preconditioner with the learned correction, which is not a fixed
// linear operator: z = B r, p = z - sum_j (z.K p_j / p_j.K p_j) p_j,
// alpha = p.r / p.K p.  x starts at 0, r = b, z = B b on entry.  The learned
// part is dropped (net = false) when the residual stagnates.
int fcg(mfe_ctx* c, const mfe_solve_opts* o, bool net, double* x, double* r, double* z, double bnorm,
        hipStream_t s, int& iters, double& rel, int* net_fallbacks) {
    const int64_t n = c->n_dofs;
    constexpr int M = mfe::kMaxDirs;
    if (!c->d_fcg) MFE_HIP(c, hipMalloc(&c->d_fcg, 2 * (int64_t)M * n * sizeof(double)));
    double* Pd = c->d_fcg;             // directions, M rows
    double* KPd = c->d_fcg + M * n;    // their images under K
    double pkp[M];
    double* out = c->d_partials + 2 * mfe::kDotBlocks;
    std::vector<double> rel_hist;
    int have = 0, head = 0;  // ring buffer of directions
    int rc;
    for (int it = 1; it <= o->max_cg; ++it) {
        // p = z orthogonalised against the stored directions (in ring order)
        const int slot = head;
        double* p = Pd + (int64_t)slot * n;
        double* Kp = KPd + (int64_t)slot * n;
        mfe::DirCoeffs cf{};
        if (have > 0) {
            // only the `have` rows written so far are read (rows 0..have-1)
            MFE_HIP(c, mfe::launch_multidot(z, KPd, have, n, c->d_partials, out, s));
            MFE_HIP(c, hipMemcpyAsync(c->h_scalars, out, have * sizeof(double), hipMemcpyDeviceToHost, s));
            MFE_HIP(c, hipStreamSynchronize(s));
            for (int j = 0; j < M; ++j) {
                const bool used = j < have && j != slot;
                cf.c[j] = used ? c->h_scalars[j] / pkp[j] : 0.0;
            }
        }
        MFE_HIP(c, mfe::launch_multi_axpy(z, Pd, cf, have, n, p, s));
        rc = mfe_apply_tangent(c, p, Kp, o->strategy, MFE_FP64, s);
        if (rc != MFE_OK) return rc;
        double pr, pKp;
        rc = dot2(c, p, r, p, Kp, s, pr, pKp);
        if (rc != MFE_OK) return rc;
        if (!(pKp > 0.0)) return fail(c, MFE_ENOTCONV, "CG breakdown: p.Kp <= 0 (tangent not positive definite)");
        pkp[slot] = pKp;
        head = (head + 1) % M;
        have = std::min(have + 1, M);
        const double alpha = pr / pKp;
        double* out2 = c->d_partials + 2 * mfe::kDotBlocks;
        MFE_HIP(c, mfe::launch_cg_update(x, r, z, p, Kp, nullptr, alpha, n, c->d_partials, out2, s));
        MFE_HIP(c, hipMemcpyAsync(c->h_scalars, out2, sizeof(double), hipMemcpyDeviceToHost, s));
        MFE_HIP(c, hipStreamSynchronize(s));
        iters = it;
        rel = std::sqrt(c->h_scalars[0]) / bnorm;
        if (rel <= o->cg_rtol) return MFE_OK;
        if (net) {  // stagnation: less than 10% residual reduction over the last 3 iterations
            rel_hist.push_back(rel);
            const size_t k = rel_hist.size();
            if (k >= 4 && rel_hist[k - 1] > 0.9 * rel_hist[k - 4]) {
                net = false;
                c->net_off = true;
                if (net_fallbacks) ++*net_fallbacks;
            }
        }
        double rz;
        rc = precondition(c, o, net, r, z, s, rz);
        if (rc == MFE_ENOTCONV && net) {
            net = false;
            c->net_off = true;
            if (net_fallbacks) ++*net_fallbacks;
            c->err.clear();
            rc = precondition(c, o, false, r, z, s, rz);
        }
        if (rc != MFE_OK) return rc;
    }
    return fail(c, MFE_ENOTCONV, "CG did not reach its tolerance");
}

// preconditioned CG on K(u) x = b, x starts at 0.  Work vectors: r, z, p, Ap, dinv.
int cg(mfe_ctx* c, const mfe_solve_opts* o, const double* b, double* x, hipStream_t s, int& iters, double& rel,
       int* fallbacks = nullptr, int* net_fallbacks = nullptr) {
    const int64_t n = c->n_dofs;
    double* r = c->d_work + 0 * n;
    double* z = c->d_work + 1 * n;
    double* pv = c->d_work + 2 * n;
    double* Ap = c->d_work + 3 * n;
    double* dinv = c->d_work + 4 * n;
    iters = 0;
    rel = 0.0;
    bool jac = o->preconditioner == MFE_PC_JACOBI;
    bool gmg = o->preconditioner == MFE_PC_GMG || o->preconditioner == MFE_PC_GMG_NET;
    // learned correction on top of the V-cycle: flexible CG (the preconditioner
    // is not linear), dropped for the rest of the solve when it stops helping
    // once a solve on this context had to drop the correction, later solves
    // use the plain V-cycle until a network is set again
    bool net = o->preconditioner == MFE_PC_GMG_NET && !c->net_off;
    const bool flexible = net;
    int rc;
    if (net) {
        int npx, npy, npz;
        if (!c->d_net) return fail(c, MFE_EINVAL, "no network set (mfe_set_network)");
        if (patch_dims(c, npx, npy, npz) == 0)
            return fail(c, MFE_EUNSUPPORTED, "the learned correction needs Q2 and cell counts divisible by 4");
        if (o->mg_precision != MFE_FP64)
            return fail(c, MFE_EUNSUPPORTED, "the learned correction runs in the FP64 V-cycle");
    }
    MFE_HIP(c, mfe::launch_fill(x, n, 0.0, s));
    MFE_HIP(c, mfe::launch_scale_mul(1.0, nullptr, b, r, n, s));
    if (gmg) {
        // The V-cycle needs positive level tangents (eigenvalue estimates,
        // smoothers).  Far from equilibrium K(u) can be indefinite; then this
        // solve falls back to Jacobi-PCG, which stops at negative curvature
        // with a descent direction.
        rc = mg_build(c, o->mg_levels);
        if (rc != MFE_OK) return rc;
        rc = mg_update(c, o, s);
        if (rc == MFE_OK && net) rc = net_prepare(c, s);
        if (rc == MFE_OK) {
            double unused;
            rc = precondition(c, o, net, r, z, s, unused);
            if (rc == MFE_ENOTCONV && net) {  // try without the learned part
                net = false;
                c->net_off = true;
                if (net_fallbacks) ++*net_fallbacks;
                c->err.clear();
                rc = precondition(c, o, false, r, z, s, unused);
            }
        }
        if (rc == MFE_ENOTCONV || rc == MFE_EJACOBIAN) {
            gmg = net = false;
            jac = true;
            if (fallbacks) ++*fallbacks;
            c->err.clear();
        } else if (rc != MFE_OK) {
            return rc;
        }
    }
    if (jac) {
        // Jacobi with |diag K|: positive (so CG stays well defined) also where
        // a strongly compressed state makes diagonal entries negative
        rc = diagonal_into(c, dinv, s);
        if (rc != MFE_OK) return rc;
        MFE_HIP(c, hipMemsetAsync(c->d_bad, 0, sizeof(int), s));
        MFE_HIP(c, mfe::launch_invert(dinv, n, c->d_bad, s, true));
        int bad = 0;
        MFE_HIP(c, hipMemcpyAsync(&bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
        MFE_HIP(c, hipStreamSynchronize(s));
        if (bad) return fail(c, MFE_EJACOBIAN, "tangent diagonal has zero or non-finite entries: no Jacobi preconditioner");
    }
    if (!gmg) MFE_HIP(c, mfe::launch_scale_mul(1.0, jac ? dinv : nullptr, r, z, n, s));
    MFE_HIP(c, mfe::launch_scale_mul(1.0, nullptr, z, pv, n, s));
    double rr, rz;
    rc = dot2(c, r, r, r, z, s, rr, rz);
    if (rc != MFE_OK) return rc;
    const double bnorm = std::sqrt(rr);
    if (bnorm == 0.0) return MFE_OK;
    if (flexible && gmg) return fcg(c, o, net, x, r, z, bnorm, s, iters, rel, net_fallbacks);
    double* out = c->d_partials + 2 * mfe::kDotBlocks;
    if (gmg) {
        // The same iteration with alpha and beta formed on the device from
        // device-resident dot products, so each iteration waits for the host
        // once (for the stopping test) instead of three times.  S[0] = p.Ap,
        // S[2] = r.r after the update, S[4] and S[6] = r.z of the current and
        // the next iterate.  A non-positive r.z (preconditioner) or p.Ap
        // (curvature) zeroes the next update on the device and is reported at
        // the following wait, with x, r and the iteration count as the
        // host-side loop leaves them.
        double* S = out + 8;
        c->h_scalars[8] = rz;
        MFE_HIP(c, hipMemcpyAsync(S + 4, c->h_scalars + 8, sizeof(double), hipMemcpyHostToDevice, s));
        int cur = 0;
        for (int it = 1; it <= o->max_cg; ++it) {
            rc = mfe_apply_tangent(c, pv, Ap, o->strategy, MFE_FP64, s);
            if (rc != MFE_OK) return rc;
            double* rzc = S + 4 + 2 * cur;
            MFE_HIP(c, mfe::launch_dot2(pv, Ap, nullptr, nullptr, n, c->d_partials, S, s));
            MFE_HIP(c, mfe::launch_cg_update_dev(x, r, z, pv, Ap, nullptr, rzc, S, n, c->d_partials, S + 2, s));
            MFE_HIP(c, hipMemcpyAsync(c->h_scalars, S, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
            MFE_HIP(c, hipStreamSynchronize(s));
            const double pAp = c->h_scalars[0], rzh = c->h_scalars[4 + 2 * cur];
            if (!(rzh > 0.0)) return fail(c, MFE_ENOTCONV, "preconditioner is not positive definite");
            if (!(pAp > 0.0)) {
                if (it == 1 && pAp < 0.0) MFE_HIP(c, mfe::launch_axpby(rzh / -pAp, pv, 0.0, x, n, s));
                return fail(c, MFE_ENOTCONV, "CG breakdown: p.Kp <= 0 (tangent not positive definite)");
            }
            iters = it;
            rel = std::sqrt(c->h_scalars[2]) / bnorm;
            if (rel <= o->cg_rtol) return MFE_OK;
            rc = gmg_apply(c, o, r, z, s);
            if (rc != MFE_OK) return rc;
            double* rzn = S + 4 + 2 * (1 - cur);
            MFE_HIP(c, mfe::launch_dot2(r, z, nullptr, nullptr, n, c->d_partials, rzn, s));
            MFE_HIP(c, mfe::launch_p_update_dev(z, rzn, rzc, pv, n, s));
            cur = 1 - cur;
        }
        return fail(c, MFE_ENOTCONV, "CG did not reach its tolerance");
    }
    for (int it = 1; it <= o->max_cg; ++it) {
        rc = mfe_apply_tangent(c, pv, Ap, o->strategy, MFE_FP64, s);
        if (rc != MFE_OK) return rc;
        double pAp, unused;
        rc = dot2(c, pv, Ap, nullptr, nullptr, s, pAp, unused);
        if (rc != MFE_OK) return rc;
        if (!(pAp > 0.0)) {
            // negative curvature: keep the iterate so far; on the first
            // iteration take the preconditioned residual scaled by |p.Kp|
            if (it == 1 && pAp < 0.0) MFE_HIP(c, mfe::launch_axpby(rz / -pAp, pv, 0.0, x, n, s));
            return fail(c, MFE_ENOTCONV, "CG breakdown: p.Kp <= 0 (tangent not positive definite)");
        }
        const double alpha = rz / pAp;
        MFE_HIP(c, mfe::launch_cg_update(x, r, z, pv, Ap, jac ? dinv : nullptr, alpha, n, c->d_partials, out, s));
        MFE_HIP(c, hipMemcpyAsync(c->h_scalars, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        MFE_HIP(c, hipStreamSynchronize(s));
        rr = c->h_scalars[0];
        double rz_new = c->h_scalars[1];
        iters = it;
        rel = std::sqrt(rr) / bnorm;
        if (rel <= o->cg_rtol) return MFE_OK;
        if (gmg) {
            rc = precondition(c, o, false, r, z, s, rz_new);
            if (rc != MFE_OK) return rc;
        }
        MFE_HIP(c, mfe::launch_axpby(1.0, z, rz_new / rz, pv, n, s));
        rz = rz_new;
    }
    return fail(c, MFE_ENOTCONV, "CG did not reach its tolerance");
}

}  // namespace

extern "C" {

int mfe_axpby(mfe_ctx* c, double a, const double* x, double b, double* y, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!x || !y) return fail(c, MFE_EINVAL, "null vector");
    DeviceGuard g(c->device);
    MFE_HIP(c, mfe::launch_axpby(a, x, b, y, c->n_dofs, static_cast<hipStream_t>(stream)));
    return MFE_OK;
}

int mfe_dot(mfe_ctx* c, const double* x, const double* y, double* result, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!x || !y || !result) return fail(c, MFE_EINVAL, "null pointer");
    DeviceGuard g(c->device);
    int rc = ensure_work(c);
    if (rc != MFE_OK) return rc;
    double unused;
    return dotn(c, c->n_dofs, x, y, nullptr, nullptr, static_cast<hipStream_t>(stream), *result, unused);
}

int mfe_zero_constrained(mfe_ctx* c, double* v, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!v) return fail(c, MFE_EINVAL, "null vector");
    DeviceGuard g(c->device);
    if (c->n_con > 0) MFE_HIP(c, mfe::launch_set_indexed(c->d_cidx, c->n_con, 0.0, v, static_cast<hipStream_t>(stream)));
    return MFE_OK;
}

int mfe_diagonal(mfe_ctx* c, double* d, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!c->has_state) return fail(c, MFE_ESTATE, "no state set");
    if (!d) return fail(c, MFE_EINVAL, "null vector");
    if (c->model != MFE_MODEL_NH)
        return fail(c, MFE_EUNSUPPORTED, "the diagonal is built from the second-order cache of eq. hypref");
    DeviceGuard g(c->device);
    int rc = ensure_work(c);
    if (rc != MFE_OK) return rc;
    return diagonal_into(c, d, static_cast<hipStream_t>(stream));
}

// shared checks of the standalone GMG entry points; o2 gets the options with
// the preconditioner set to GMG
static int gmg_entry(mfe_ctx* c, const mfe_solve_opts* o, mfe_solve_opts& o2) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    if (!o) return fail(c, MFE_EINVAL, "null options");
    o2 = *o;
    o2.preconditioner = MFE_PC_GMG;
    int rc = check_opts(c, &o2);
    if (rc != MFE_OK) return rc;
    if (!c->has_state) return fail(c, MFE_ESTATE, "no state set");
    return ensure_work(c);
}

int mfe_gmg_setup(mfe_ctx* c, const mfe_solve_opts* o, void* stream) {
    mfe_solve_opts o2;
    int rc = gmg_entry(c, o, o2);
    if (rc != MFE_OK) return rc;
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (o2.strategy != MFE_OTF && o2.strategy != MFE_OTF_AD) {
        const int slot = cache_slot(o2.strategy);
        if (!c->cache_valid[slot] || (slot > 0 && c->cache_version[slot] != c->state_version)) {
            rc = mfe_build_cache(c, o2.strategy, s);
            if (rc != MFE_OK) return rc;
        }
    }
    rc = mg_build(c, o2.mg_levels);
    if (rc != MFE_OK) return rc;
    c->mg_lag_left = 0;  // a set-up on request is a full one
    return mg_update(c, &o2, s);
}

int mfe_gmg_apply(mfe_ctx* c, const mfe_solve_opts* o, const double* r, double* z, void* stream) {
    mfe_solve_opts o2;
    int rc = gmg_entry(c, o, o2);
    if (rc != MFE_OK) return rc;
    if (!r || !z) return fail(c, MFE_EINVAL, "null vector");
    if (overlaps(r, z, c->n_dofs * (int64_t)sizeof(double))) return fail(c, MFE_EINVAL, "r and z overlap");
    const mfe_solve_opts& m = c->mg_ready_opts;
    if (c->mg.empty() || c->mg_request != o2.mg_levels || c->mg_ready_version != c->state_version ||
        c->mg_ready_strategy != o2.strategy || c->mg_ready_prec != o2.mg_precision ||
        m.cheb_degree != o2.cheb_degree || m.cheb_range != o2.cheb_range || m.coarse_degree != o2.coarse_degree ||
        m.coarse_range != o2.coarse_range || m.coarse_direct != o2.coarse_direct)
        return fail(c, MFE_ESTATE, "multigrid level data not set up for this state and these options");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = c->n_dofs;
    double* rw = c->d_work;      // the CG residual and preconditioned residual slots:
    double* zw = c->d_work + n;  // the same buffers as inside CG, so one graph serves both
    const bool net = o->preconditioner == MFE_PC_GMG_NET;
    if (net) {
        if (o2.mg_precision != MFE_FP64)
            return fail(c, MFE_EUNSUPPORTED, "the learned correction runs in the FP64 V-cycle");
        rc = net_prepare(c, s);
        if (rc != MFE_OK) return rc;
    }
    MFE_HIP(c, mfe::launch_copy(r, rw, n, s));
    c->net_in_cycle = net;
    rc = gmg_apply(c, &o2, rw, zw, s);
    c->net_in_cycle = false;
    if (rc != MFE_OK) return rc;
    MFE_HIP(c, mfe::launch_copy(static_cast<const double*>(zw), z, n, s));
    return MFE_OK;
}

int mfe_cg_solve(mfe_ctx* c, const mfe_solve_opts* o, const double* b, double* x, int* iterations_out,
                 double* rel_out, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    int rc = check_opts(c, o);
    if (rc != MFE_OK) return rc;
    if (!b || !x) return fail(c, MFE_EINVAL, "null vector");
    if (overlaps(b, x, c->n_dofs * (int64_t)sizeof(double))) return fail(c, MFE_EINVAL, "b and x overlap");
    if (!c->has_state) return fail(c, MFE_ESTATE, "no state set");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = ensure_work(c);
    if (rc != MFE_OK) return rc;
    c->mg_lag_left = 0;  // a CG solve on its own sets the multigrid up in full
    if (o->strategy != MFE_OTF && o->strategy != MFE_OTF_AD) {
        const int slot = cache_slot(o->strategy);
        if (!c->cache_valid[slot] || (slot > 0 && c->cache_version[slot] != c->state_version)) {
            rc = mfe_build_cache(c, o->strategy, s);
            if (rc != MFE_OK) return rc;
        }
    }
    int iters = 0;
    double rel = 0.0;
    rc = cg(c, o, b, x, s, iters, rel);
    if (iterations_out) *iterations_out = iters;
    if (rel_out) *rel_out = rel;
    return rc;
}

int mfe_newton_solve(mfe_ctx* c, const mfe_solve_opts* o, double* u, const double* g, mfe_solve_report* rep,
                     void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    mfe_solve_report local;
    std::memset(&local, 0, sizeof(local));
    if (rep) *rep = local;
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    int rc = check_opts(c, o);
    if (rc != MFE_OK) return rc;
    if (!u) return fail(c, MFE_EINVAL, "null vector");
    DeviceGuard dg_guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = ensure_work(c);
    if (rc != MFE_OK) return rc;
    c->mg_lag_left = 0;  // the first CG solve sets the multigrid up in full
    const int64_t n = c->n_dofs;
    double* res = c->d_work + 5 * n;   // residual, then the right-hand side
    double* du = c->d_work + 6 * n;    // Newton correction
    double* dg = c->d_work + 7 * n;    // increment of the Dirichlet values
    const bool has_dg = g != nullptr && c->n_con > 0;
    if (has_dg) {
        MFE_HIP(c, mfe::launch_fill(dg, n, 0.0, s));
        MFE_HIP(c, mfe::launch_diff_indexed(c->d_cidx, c->n_con, g, u, dg, s));
    }
    const bool cached = o->strategy != MFE_OTF && o->strategy != MFE_OTF_AD;
    int status = MFE_ENOTCONV;
    double rn = 0.0;
    bool have_res = false;
    // Eisenstat-Walker forcing: the previous residual norm and tolerance
    double rn_prev = 0.0, eta_prev = o->forcing;
    bool boundary_left = has_dg;  // dg holds the part of the Dirichlet increment not yet applied
    for (int it = 0;; ++it) {
        if (!have_res) {
            rc = mfe_residual(c, u, res, s);
            if (rc != MFE_OK) { status = rc; break; }
            double rr, unused;
            rc = dot2(c, res, res, nullptr, nullptr, s, rr, unused);
            if (rc != MFE_OK) { status = rc; break; }
            rn = std::sqrt(rr);
        }
        have_res = false;
        if (it == 0) local.initial_residual = rn;
        local.final_residual = rn;
        if (it < MFE_HISTORY) local.residual_history[it] = rn;
        if (!std::isfinite(rn)) { status = fail(c, MFE_ENOTCONV, "residual is not finite"); break; }
        const bool boundary_step = boundary_left;
        if (!boundary_step && rn <= o->newton_atol) { local.converged = 1; status = MFE_OK; break; }
        if (it == o->max_newton) { status = fail(c, MFE_ENOTCONV, "Newton did not converge"); break; }
        rc = mfe_set_state(c, u, s);
        if (rc != MFE_OK) { status = rc; break; }
        if (cached) {
            rc = mfe_build_cache(c, o->strategy, s);
            if (rc != MFE_OK) { status = rc; break; }
        }
        MFE_HIP(c, mfe::launch_scale_mul(-1.0, nullptr, res, res, n, s));
        if (boundary_step) {
            // rhs_f = -R_f - (K dg)_f with the unconstrained operator, rhs_c = dg_c
            rc = apply_impl(c, dg, du, o->strategy, MFE_FP64, false, s);
            if (rc != MFE_OK) { status = rc; break; }
            MFE_HIP(c, mfe::launch_axpby(-1.0, du, 1.0, res, n, s));
            MFE_HIP(c, mfe::launch_copy_indexed(c->d_cidx, c->n_con, dg, res, s));
        }
        mfe_solve_opts oc = *o;
        if (o->forcing > 0.0 && !boundary_step) {
            double eta = o->forcing;
            if (rn_prev > 0.0) {
                const double q = rn / rn_prev;
                eta = 0.9 * q * q;
                const double safe = 0.9 * eta_prev * eta_prev;
                if (safe > 0.1) eta = std::max(eta, safe);
            }
            eta = std::min(eta, o->forcing);
            eta = std::max(eta, 0.5 * o->newton_atol / rn);
            eta = std::max(eta, o->cg_rtol);
            oc.cg_rtol = eta;
            eta_prev = eta;
            rn_prev = rn;
        }
        int iters = 0;
        double rel = 0.0;
        rc = cg(c, &oc, res, du, s, iters, rel, &local.pc_fallbacks, &local.net_fallbacks);
        local.cg_iterations += iters;
        // no lagged set-up after a solve that stopped early, nor after the
        // boundary increment, which moves the state furthest
        if (rc != MFE_OK || boundary_step) c->mg_lag_left = 0;
        if (rc != MFE_OK && rc != MFE_ENOTCONV) { status = rc; break; }
        c->err.clear();
        local.newton_iterations = it + 1;
        if (boundary_step) {
            // the linearised response to the increment is applied in full;
            // a state it inverts shows as a non-finite residual next
            MFE_HIP(c, mfe::launch_axpby(1.0, du, 1.0, u, n, s));
            MFE_HIP(c, mfe::launch_copy_indexed(c->d_cidx, c->n_con, g, u, s));  // exact Dirichlet values
            boundary_left = false;
            continue;
        }
        // backtracking line search, det F > 0 required: accept when ||R|| or
        // the stored energy decreases (Armijo, slope R.du); the energy test
        // carries the iteration through regions where ||R|| grows on the way
        // to the minimiser, the residual test the last steps where energy
        // differences drown in rounding
        double e0 = 0.0, slope = 0.0, unused0;
        rc = mfe_energy(c, u, &e0, s);
        if (rc != MFE_OK) { status = rc; break; }
        rc = dot2(c, res, du, nullptr, nullptr, s, slope, unused0);  // res holds -R
        if (rc != MFE_OK) { status = rc; break; }
        slope = -slope;
        double a = 1.0;
        MFE_HIP(c, mfe::launch_axpby(1.0, du, 1.0, u, n, s));
        bool accepted = false;
        for (int k = 0; k <= 12; ++k) {
            rc = mfe_set_state(c, u, s);
            if (rc == MFE_OK) {
                rc = mfe_residual(c, u, res, s);
                if (rc != MFE_OK) break;
                double rr, unused;
                rc = dot2(c, res, res, nullptr, nullptr, s, rr, unused);
                if (rc != MFE_OK) break;
                const double rt = std::sqrt(rr);
                double et = 0.0;
                bool armijo = false;
                if (slope < 0.0 && std::isfinite(rt)) {
                    rc = mfe_energy(c, u, &et, s);
                    if (rc != MFE_OK) break;
                    armijo = et <= e0 + 1e-4 * a * slope;
                }
                if (rt < rn || (armijo && std::isfinite(rt))) {
                    rn = rt;
                    have_res = true;
                    accepted = true;
                    break;
                }
            } else if (rc != MFE_EJACOBIAN) {
                break;
            }
            rc = MFE_OK;
            if (k == 12) break;
            a *= 0.5;  // u = u_old + a du
            MFE_HIP(c, mfe::launch_axpby(-a, du, 1.0, u, n, s));
            local.backtracks++;
        }
        if (rc != MFE_OK) { status = rc; break; }
        if (!accepted) {
            c->err.clear();
            status = fail(c, MFE_ENOTCONV, "line search failed");
            break;
        }
    }
    (void)hipStreamSynchronize(s);
    if (rep) *rep = local;
    return status;
}

int mfe_solve_load_path(mfe_ctx* c, const mfe_solve_opts* o, double* u, double* prev, int n_steps,
                        double min_fraction, int extrapolate, mfe_path_state* state, mfe_load_fn load,
                        void* load_user, mfe_step_fn on_step, void* step_user, mfe_path_report* reports,
                        int max_reports, int* n_reports, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (n_reports) *n_reports = 0;
    if (!c->has_mesh) return fail(c, MFE_EINVAL, "no mesh");
    int rc = check_opts(c, o);
    if (rc != MFE_OK) return rc;
    if (!u) return fail(c, MFE_EINVAL, "null state vector");
    if (extrapolate && !prev) return fail(c, MFE_EINVAL, "extrapolation needs the previous-state vector");
    if (prev == u) return fail(c, MFE_EINVAL, "the state and previous-state vectors alias");
    if (n_steps < 1) return fail(c, MFE_EINVAL, "n_steps must be >= 1");
    if (!(min_fraction > 0.0 && min_fraction <= 1.0)) return fail(c, MFE_EINVAL, "min_fraction must be in (0, 1]");
    if (c->n_con > 0 && !load) return fail(c, MFE_EINVAL, "constrained dofs need a load callback");
    if (max_reports < 0 || (max_reports > 0 && !reports)) return fail(c, MFE_EINVAL, "bad report buffer");
    mfe_path_state st{0.0, 0.0, 0.0, 0.0};
    if (state) st = *state;
    const double h0 = 1.0 / n_steps;
    if (!(st.t >= 0.0 && st.t <= 1.0)) return fail(c, MFE_EINVAL, "path position outside [0, 1]");
    if (!(st.h > 0.0)) st.h = h0;
    if (!(st.h_cap > 0.0)) st.h_cap = h0;
    if (!(st.prev_h > 0.0)) st.prev_h = 0.0;
    DeviceGuard dg_guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = c->n_dofs;
    if (!c->d_path) MFE_HIP(c, hipMalloc(&c->d_path, 3 * n * sizeof(double)));
    double* trial = c->d_path;
    double* g = c->d_path + n;          // prescribed values at the constrained dofs, other entries unused
    double* gc = c->d_path + 2 * n;     // the same values, compact
    std::vector<double> vals(c->n_con);
    int nrep = 0;
    auto record = [&](double t, double h, bool failed, int status, const mfe_solve_report& r) {
        if (nrep < max_reports) reports[nrep] = mfe_path_report{t, h, failed ? 1 : 0, status, r};
        if (nrep < max_reports) ++nrep;
        if (n_reports) *n_reports = nrep;
    };
    // a Newton solve ends the path only for errors other than convergence
    auto hard = [](int r) { return r != MFE_OK && r != MFE_ENOTCONV && r != MFE_EJACOBIAN; };
    int status = MFE_OK;
    while (st.t < 1.0 - 1e-12) {
        const double h = std::min(st.h, 1.0 - st.t);
        st.h = h;
        if (c->n_con > 0) {
            if (load(st.t + h, vals.data(), c->n_con, load_user) != 0) {
                status = fail(c, MFE_EINVAL, "the load callback failed");
                break;
            }
            MFE_HIP(c, hipMemcpyAsync(gc, vals.data(), c->n_con * sizeof(double), hipMemcpyHostToDevice, s));
            MFE_HIP(c, mfe::launch_scatter_indexed(c->d_cidx, c->n_con, gc, g, s));
            // the host buffer is reused by the next step's callback
            MFE_HIP(c, hipStreamSynchronize(s));
        }
        const bool extra = extrapolate && st.prev_h > 0.0;
        if (extra) {  // trial = u + (h / prev_h) (u - prev)
            MFE_HIP(c, mfe::launch_axpby(1.0 + h / st.prev_h, u, 0.0, trial, n, s));
            MFE_HIP(c, mfe::launch_axpby(-h / st.prev_h, prev, 1.0, trial, n, s));
        } else {
            MFE_HIP(c, hipMemcpyAsync(trial, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        const double* gp = c->n_con > 0 ? g : nullptr;
        mfe_solve_report r;
        int nr = mfe_newton_solve(c, o, trial, gp, &r, s);
        if (hard(nr)) { status = nr; break; }
        if (nr != MFE_OK && extra) {
            // the extrapolated start can be worse than the last converged
            // state (cells it distorts): retry the step from there
            record(st.t + h, h, true, nr, r);
            MFE_HIP(c, hipMemcpyAsync(trial, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            nr = mfe_newton_solve(c, o, trial, gp, &r, s);
            if (hard(nr)) { status = nr; break; }
        }
        if (nr == MFE_OK) {
            if (prev) MFE_HIP(c, hipMemcpyAsync(prev, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            MFE_HIP(c, hipMemcpyAsync(u, trial, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            st.prev_h = h;
            st.t += h;
            record(st.t, h, false, nr, r);
            st.h = std::min(st.h_cap, 1.25 * h);
            c->err.clear();
            if (on_step) {
                MFE_HIP(c, hipStreamSynchronize(s));
                if (on_step(&st, u, prev, step_user) != 0) break;
            }
        } else {
            record(st.t + h, h, true, nr, r);
            st.h_cap = std::min(st.h_cap, 0.9 * h);
            st.h = 0.5 * h;
            if (st.h < min_fraction) {
                c->err.clear();
                status = fail(c, MFE_ENOTCONV, "load step below min_fraction of the path at t = " + std::to_string(st.t));
                break;
            }
        }
    }
    (void)hipStreamSynchronize(s);
    if (state) *state = st;
    return status;
}

}  // extern "C"

extern "C" {

int mfe_set_deterministic(mfe_ctx* c, int on) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    c->deterministic = on != 0;
    return MFE_OK;
}

int mfe_set_timing(mfe_ctx* c, int every) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (every < 0) return fail(c, MFE_EINVAL, "timing interval must be >= 0");
    c->timing = every;
    c->timing_seq = 0;
    c->ev_used = 0;
    return MFE_OK;
}

double mfe_apply_kernel_ms(mfe_ctx* c, int* count_out) {
    if (count_out) *count_out = 0;
    if (!c || c->ev_used == 0) return -1.0;
    DeviceGuard g(c->device);
    double total = 0.0;
    for (int i = 0; i < c->ev_used; ++i) {
        if (hipEventSynchronize(c->ev_stop[i]) != hipSuccess) return -1.0;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]) != hipSuccess) return -1.0;
        total += ms;
    }
    if (count_out) *count_out = c->ev_used;
    return total / c->ev_used;
}

}  // extern "C"

// ---------------------------------------------------------------- learned correction
extern "C" {

int mfe_set_network(mfe_ctx* c, const float* params_host, int variant) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    if (variant != MFE_NET_RELU && variant != MFE_NET_LINEAR) return fail(c, MFE_EINVAL, "unknown network variant");
    c->net_variant = variant;
    c->net_off = false;
    c->mg_graph_valid = false;  // a captured cycle holds the parameter pointer and the variant
    DeviceGuard g(c->device);
    if (!params_host) {
        dfree(c->d_net);
        return MFE_OK;
    }
    for (int i = 0; i < kNetParams; ++i)
        if (!std::isfinite(params_host[i])) return fail(c, MFE_EINVAL, "non-finite network parameter");
    if (!c->d_net) MFE_HIP(c, hipMalloc(&c->d_net, kNetParams * sizeof(float)));
    MFE_HIP(c, hipMemcpy(c->d_net, params_host, kNetParams * sizeof(float), hipMemcpyHostToDevice));
    return MFE_OK;
}

int64_t mfe_patch_count(const mfe_ctx* c) {
    if (!c) return 0;
    int npx, npy, npz;
    return patch_dims(c, npx, npy, npz);
}

int mfe_patch_features(mfe_ctx* c, const double* r, float* feat, float* scale, int variant, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    int npx, npy, npz;
    const int P = patch_dims(c, npx, npy, npz);
    if (P == 0) return fail(c, MFE_EUNSUPPORTED, "patches need Q2 and cell counts divisible by 4");
    if (!r || !feat || !scale) return fail(c, MFE_EINVAL, "null pointer");
    DeviceGuard g(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_node_invariants(c, s);
    if (rc != MFE_OK) return rc;
    MFE_HIP(c, mfe::launch_patch_features(r, c->d_ninv, c->Nx, c->Ny, npx, npy, P, variant == MFE_NET_LINEAR, feat,
                                          scale, s));
    return MFE_OK;
}

int mfe_patch_targets(mfe_ctx* c, const double* e, const float* scale, float* t, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    int npx, npy, npz;
    const int P = patch_dims(c, npx, npy, npz);
    if (P == 0) return fail(c, MFE_EUNSUPPORTED, "patches need Q2 and cell counts divisible by 4");
    if (!e || !scale || !t) return fail(c, MFE_EINVAL, "null pointer");
    DeviceGuard g(c->device);
    MFE_HIP(c, mfe::launch_patch_targets(e, scale, c->Nx, c->Ny, npx, npy, P, t, static_cast<hipStream_t>(stream)));
    return MFE_OK;
}

int mfe_patch_scatter(mfe_ctx* c, const float* y, const float* scale, double alpha, double* z, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    int npx, npy, npz;
    const int P = patch_dims(c, npx, npy, npz);
    if (P == 0) return fail(c, MFE_EUNSUPPORTED, "patches need Q2 and cell counts divisible by 4");
    if (!y || !scale || !z) return fail(c, MFE_EINVAL, "null pointer");
    DeviceGuard g(c->device);
    MFE_HIP(c, mfe::launch_patch_scatter(y, scale, c->Nx, c->Ny, c->Nz, npx, npy, npz, alpha, z,
                                         static_cast<hipStream_t>(stream)));
    return MFE_OK;
}

int mfe_patch_adjoint(mfe_ctx* c, const double* g, const float* scale, double alpha, float* dy, void* stream) {
    if (!c) return MFE_EINVAL;
    c->err.clear();
    int npx, npy, npz;
    const int P = patch_dims(c, npx, npy, npz);
    if (P == 0) return fail(c, MFE_EUNSUPPORTED, "patches need Q2 and cell counts divisible by 4");
    if (!g || !scale || !dy) return fail(c, MFE_EINVAL, "null pointer");
    DeviceGuard gd(c->device);
    MFE_HIP(c, mfe::launch_patch_adjoint(g, scale, c->Nx, c->Ny, npx, npy, npz, P, (float)alpha, dy,
                                         static_cast<hipStream_t>(stream)));
    return MFE_OK;
}

int mfe_net_forward(const float* params, const float* x, int n_patches, int variant, float* act, float* y,
                    void* stream) {
    if (!params || !x || !act || !y || n_patches < 0) return MFE_EINVAL;
    if (variant != MFE_NET_RELU && variant != MFE_NET_LINEAR) return MFE_EINVAL;
    return net_forward(params, x, n_patches, variant, act, y, static_cast<hipStream_t>(stream)) == hipSuccess
               ? MFE_OK
               : MFE_EHIP;
}

int mfe_net_backward(const float* params, const float* x, const float* act, const float* dy, int n_patches,
                     int variant, float* work, float* grad, void* stream) {
    if (!params || !x || !act || !dy || !work || !grad || n_patches < 1) return MFE_EINVAL;
    if (variant != MFE_NET_RELU && variant != MFE_NET_LINEAR) return MFE_EINVAL;
    return net_backward(params, x, act, dy, n_patches, variant, work, grad, static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? MFE_OK
               : MFE_EHIP;
}

int mfe_net_loss(const float* y, const float* t, int64_t n, float* dy, double* scratch, double* loss, void* stream) {
    if (!y || !t || !scratch || !loss || n < 1) return MFE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = mfe::mse_blocks(n);
    if (mfe::launch_mse(y, t, n, dy, scratch, s) != hipSuccess) return MFE_EHIP;
    if (mfe::launch_sum(scratch, nb, scratch + 1024, s) != hipSuccess) return MFE_EHIP;
    double h = 0.0;
    if (hipMemcpyAsync(&h, scratch + 1024, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return MFE_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MFE_EHIP;
    *loss = h / (double)n;
    return MFE_OK;
}

int mfe_net_adam(float* params, const float* grad, float* m, float* v, int step, float lr, void* stream) {
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f)) return MFE_EINVAL;
    return mfe::launch_adam(params, grad, m, v, kNetParams, lr, 0.9f, 0.999f, 1e-8f, step,
                            static_cast<hipStream_t>(stream)) == hipSuccess
               ? MFE_OK
               : MFE_EHIP;
}

}  // extern "C"
