/*
 * mfe.h -- C ABI of the matrix-free finite-strain tangent library (libmfe.so).
 *
 * The library applies the tangent operator of a compressible neo-Hookean
 * hyperelastic body discretised with hexahedral Q_p elements,
 *
 *     v_i = K(u; w, phi_i) = sum_cells sum_q JxW_q  Grad phi_i : L(F_q) : Grad w
 *
 * (Wichrowski et al., "Matrix-free methods for finite-strain elasticity",
 * Sec. 2.1 eqs. DF and L for the tangent, Sec. 2.4 Alg. 1 for the cell-wise
 * matrix-free evaluation, Sec. 2.5 Alg. 2 for the cached variant, Sec. 3.2
 * eq. hypref for the energy), without ever forming a matrix.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh     a structured nx*ny*nz box of hexahedra whose corner vertices are
 *          given by the caller (any positions giving positive Jacobians); the
 *          geometry map of each cell is trilinear through its 8 vertices.
 * Nodes    a degree-p mesh has (p*nx+1)*(p*ny+1)*(p*nz+1) nodes numbered
 *          I + Nx*(J + Ny*K), x fastest; the Lagrange support points are
 *          Gauss-Lobatto-Legendre points; quadrature is the (p+1)^3 Gauss rule.
 * DoFs     node n carries dofs 3n, 3n+1, 3n+2 (x, y, z displacement).
 * Vectors  u, w, v, r are contiguous float64 arrays of n_dofs entries in
 *          device memory of the context's GPU, owned by the caller; they
 *          must stay valid until the work queued on the given stream ends.
 *          The library never frees or retains them (set_state copies u).
 * Streams  every `stream` argument is a hipStream_t passed as void*; NULL
 *          means the null stream.  Work is queued on that stream; only
 *          mfe_set_state (once, to read the det F check) and the solvers
 *          (to read dot products) wait for it.
 * Errors   every call returns an mfe_status; nothing throws across the ABI.
 *          mfe_last_error() returns a message for the last failed call on
 *          that context (valid until the next call on it).
 * Threads  a context is not thread-safe; use one context per host thread.
 */
#ifndef MFE_H
#define MFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfe_ctx mfe_ctx;

typedef enum mfe_status {
    MFE_OK = 0,
    MFE_EINVAL = -1,        /* bad argument: sizes, degree, aliasing, null pointer */
    MFE_EHIP = -2,          /* a HIP runtime call failed */
    MFE_ENOMEM = -3,        /* device allocation failed */
    MFE_EJACOBIAN = -4,     /* det F <= 0 or det J_g <= 0 at some quadrature point */
    MFE_ESTATE = -5,        /* apply before set_state, or cache older than the state */
    MFE_ENOTCONV = -6,      /* an iterative solver did not reach its tolerance */
    MFE_EUNSUPPORTED = -7   /* valid request that this build does not implement */
} mfe_status;

/* Point-wise strategies of the quadrature loop (Sec. 2.5).
 *   MFE_OTF       on the fly, reference configuration: G = L : Grad w in
 *                 closed form (Sec. 2.5.1), F recomputed from u and the cell
 *                 geometry recomputed from its 8 vertices at every apply.
 *   MFE_OTF_GEOM  as MFE_OTF but with the inverse geometry Jacobian and
 *                 JxW stored per quadrature point (10 doubles), the layout of
 *                 the paper's matrix-free data structures (Sec. 2.4).
 *   MFE_T2        cached second-order data of the current configuration:
 *                 M = J_g^-1 F^-1 (9), tau*JxW (6) and two scalars (17 doubles).
 *   MFE_T4        cached fourth-order spatial tangent J c * JxW (21, Voigt),
 *                 tau*JxW (6) and M (9): 36 doubles (Alg. 2; storage count of
 *                 Sec. 3.2.2).
 *   MFE_OTF_AD    on the fly like MFE_OTF, but G is obtained as the
 *                 directional derivative of P along the seed dF = Grad w by
 *                 forward-mode dual numbers (Sec. 2.5.1, eq. LG).            */
typedef enum mfe_strategy {
    MFE_OTF = 0,
    MFE_OTF_GEOM = 1,
    MFE_T2 = 2,
    MFE_T4 = 3,
    MFE_OTF_AD = 4
} mfe_strategy;

/* Arithmetic of the tangent apply (the precision direction of the method's
 * growth: the sweeps inside a preconditioner need not be FP64).
 *   MFE_FP64     w, v double; everything FP64.
 *   MFE_SF_FP32  w, v float, FP32 atomics; T2/T4 applies read the FP32
 *                cache (mfe_build_cache_fp32: values computed in FP64 from
 *                F, J, log J and rounded once) and run the sweeps of w, the
 *                point-wise products and the test contraction in FP32; the
 *                on-the-fly strategies keep u, F, J, log J, the point-wise
 *                response and the sweeps of w in FP64 (FP32 sweeps only for
 *                MFE_OTF_GEOM on Q2 boxes and in the coloured mode), since
 *                they are bound by arithmetic that FP32 does not make
 *                cheaper without packed instructions.
 *   MFE_SF_BF16  as MFE_SF_FP32 (float w and v, the FP32 cache of
 *                mfe_build_cache_fp32), but the sum-factorization sweeps of w
 *                and the test contraction run on the matrix cores: 16x16x16
 *                bf16 products with FP32 accumulation, both operands rounded
 *                to bf16 (relative error of v about 5e-3 .. 1e-2).
 *   MFE_SF_BF16X3  the same products with both operands split into three
 *                bf16 pieces and the six piece products of order <= 2
 *                accumulated: the accuracy of the FP32 sweeps.
 *   The two matrix-core precisions are built for structured boxes
 *   (mfe_mesh_box); on a general mesh they return MFE_EUNSUPPORTED. */
typedef enum mfe_precision {
    MFE_FP64 = 0,
    MFE_SF_FP32 = 1,
    MFE_SF_BF16 = 2,
    MFE_SF_BF16X3 = 3
} mfe_precision;

/* Create a context bound to HIP device `hip_device`.  *out receives the
 * context (NULL on failure).  Returns MFE_EINVAL for a bad device index. */
int mfe_create(mfe_ctx** out, int hip_device);

/* Free every device buffer of the context and the context itself.  Waits for
 * the device to finish the context's work first.  NULL is ignored. */
void mfe_destroy(mfe_ctx* ctx);

/* Message of the last failed call on ctx ("" if none; a static message if
 * ctx is NULL).  The pointer stays valid until the next call on ctx. */
const char* mfe_last_error(const mfe_ctx* ctx);

/* Define the mesh: an nx*ny*nz box of degree-`degree` hexahedra
 * (1 <= degree <= 6, each n >= 1).  vertex_xyz_host: host array of
 * (nx+1)*(ny+1)*(nz+1)*3 doubles, vertex (ix,iy,iz) at index
 * ix + (nx+1)*(iy + (ny+1)*iz), coordinates interleaved (x,y,z); copied.
 * Checks det J_g > 0 at every quadrature point (MFE_EJACOBIAN otherwise).
 * Resets material (mu = 1, lambda = 1), constraints, state and caches.
 * Synchronous. */
int mfe_mesh_box(mfe_ctx* ctx, int nx, int ny, int nz, int degree,
                 const double* vertex_xyz_host);

/* Define a general mesh of n_cells degree-`degree` hexahedra (1 <= degree <=
 * 6) over n_vertices vertices (Sec. 2.2 discretises with Q_p hexahedra; the
 * cell integrals of Sec. 2.4 run over any such cells, mapped trilinearly from
 * their 8 vertices).
 *   vertex_xyz_host      n_vertices*3 doubles (x,y,z interleaved), copied.
 *   cell_vertices_host   n_cells*8 int32 vertex ids per cell in lexicographic
 *                        local order: local vertex bx + 2 by + 4 bz sits at
 *                        reference corner (bx, by, bz); copied.
 * Nodes follow the canonical numbering, which depends only on vertex ids:
 *   1. node v < n_vertices is vertex v;
 *   2. (degree >= 2) each edge, edges sorted by their (lower, higher) vertex
 *      ids, owns degree-1 nodes, counted from its lower-id end;
 *   3. each face, faces sorted by their ascending 4-tuple of vertex ids, owns
 *      (degree-1)^2 nodes, node (s-1) + (degree-1)(t-1), where s counts support
 *      points from the face's lowest-id vertex o towards the lower-id of o's
 *      two edge neighbours on the face and t towards the other;
 *   4. each cell owns (degree-1)^3 interior nodes in its local lexicographic
 *      order, cells in order.
 * Node n carries dofs 3n, 3n+1, 3n+2; support points are Gauss-Lobatto.
 * Errors: MFE_EINVAL for ids out of range, a cell repeating a vertex, a face
 * shared by more than two cells or by two cells that disagree on its edges,
 * or a mesh beyond 32-bit indices; MFE_EJACOBIAN if det J_g <= 0 at a
 * quadrature point.  Every call except the geometric multigrid and the
 * learned correction (MFE_EUNSUPPORTED: they need a structured box) works on
 * such a mesh; per-cell material is indexed by the cell's position in
 * cell_vertices_host.  Cells are processed in the given order, so an order
 * with neighbours close together keeps the gathers local.  Resets material,
 * constraints, state and caches.  Synchronous. */
int mfe_mesh_hex(mfe_ctx* ctx, int64_t n_vertices, const double* vertex_xyz_host, int64_t n_cells,
                 const int32_t* cell_vertices_host, int degree);

/* The canonical numbering of mfe_mesh_hex without a context or a device
 * (host only): n_nodes_out receives the node count and, unless it is NULL,
 * cell_nodes_host (n_cells*(degree+1)^3 int32, caller-owned) the node of
 * every (cell, local node a = i + (degree+1)(j + (degree+1)k)).  Returns
 * MFE_EINVAL for the mesh errors listed at mfe_mesh_hex (except the
 * geometry, which is not looked at) or null arguments. */
int mfe_hex_numbering(int64_t n_vertices, int64_t n_cells, const int32_t* cell_vertices_host, int degree,
                      int32_t* cell_nodes_host, int64_t* n_nodes_out);

/* Reference coordinates of every node of the current mesh (box or general):
 * xyz_host receives n_dofs doubles, node n at (3n, 3n+1, 3n+2): the trilinear
 * image of the Gauss-Lobatto support point.  Host memory owned by the
 * caller.  Synchronous; MFE_EINVAL without a mesh. */
int mfe_node_coordinates(mfe_ctx* ctx, double* xyz_host);

/* Number of dofs of the current mesh, 3 * n_nodes (0 without a mesh). */
int64_t mfe_n_dofs(const mfe_ctx* ctx);

/* Number of cells and of quadrature points of the current mesh. */
int64_t mfe_n_cells(const mfe_ctx* ctx);
int64_t mfe_n_qpoints(const mfe_ctx* ctx);

/* Material of eq. hypref, Psi = mu/2 (tr C - 3 - 2 log J) + lambda log^2 J.
 * per_cell_mu_lambda_host: NULL for the uniform (mu, lambda), else a host
 * array of n_cells*2 doubles (mu, lambda per cell, cell index
 * ex + nx*(ey + ny*ez) on a box, the cell's position on a general mesh),
 * copied.  Invalidates state-derived caches. */
int mfe_set_material(mfe_ctx* ctx, double mu, double lambda,
                     const double* per_cell_mu_lambda_host);

/* Stored-energy function: MFE_MODEL_NH, the compressible neo-Hookean law of
 * eq. hypref with (mu, lambda) (the default), or MFE_MODEL_SPLIT, the
 * isochoric-volumetric split law of eq. hypcomplex,
 * Psi = mu/2 (J^-2/3 tr C - 3) + kappa/2 ((J^2 - 1)/2 - log J),
 * whose (mu, kappa) are passed as the (mu, lambda) of mfe_set_material.  The
 * split law is supported by the strategies that do not depend on the law or
 * differentiate it with dual numbers -- MFE_OTF_AD and MFE_T4 (whose cache is
 * filled from dual-number derivatives of P) -- and by mfe_residual and
 * mfe_energy; MFE_OTF, MFE_OTF_GEOM, MFE_T2, the diagonal and the solver
 * return MFE_EUNSUPPORTED.  A change of law invalidates the T2/T4 caches. */
#define MFE_MODEL_NH 0
#define MFE_MODEL_SPLIT 1
int mfe_set_model(mfe_ctx* ctx, int model);

/* Homogeneous Dirichlet constraints for the tangent: the listed dofs become
 * identity rows and columns (apply reads w as 0 there and returns v_c = w_c;
 * residual entries there are 0).  dofs_host: host array of n dof indices in
 * [0, n_dofs), duplicates allowed; n = 0 clears the constraints. */
int mfe_set_constraints(mfe_ctx* ctx, int64_t n, const int64_t* dofs_host);

/* Set the linearisation point u (device array of n_dofs doubles, copied on
 * `stream`).  Evaluates F = I + Grad u at every quadrature point and waits
 * for the stream once to read the result: MFE_EJACOBIAN if det F <= 0
 * anywhere (the state is then not set).  Marks every cache stale. */
int mfe_set_state(mfe_ctx* ctx, const double* u_dev, void* stream);

/* Build the per-quadrature-point data of `strategy` from the current state
 * (Alg. 2 inputs): MFE_OTF_GEOM 10, MFE_T2 17, MFE_T4 36 doubles per point,
 * stored brick by brick (all fields of a brick's points contiguous), owned
 * by the context.  No-op for MFE_OTF and
 * MFE_OTF_AD.  MFE_ESTATE without a state.  Asynchronous on `stream`. */
int mfe_build_cache(mfe_ctx* ctx, int strategy, void* stream);

/* FP32 copy of the T2 (17 floats per point) or T4 (36) cache for
 * MFE_SF_FP32 applies, computed in FP64 from the current state and rounded
 * once; same layout as the FP64 cache.  MFE_OTF_GEOM: builds the FP64
 * geometry cache (its FP32 applies read it); MFE_OTF, MFE_OTF_AD: no-op.
 * MFE_ESTATE without a state.  Asynchronous on `stream`. */
int mfe_build_cache_fp32(mfe_ctx* ctx, int strategy, void* stream);

/* Bytes of device memory held for `strategy`'s cache (0 if not built). */
int64_t mfe_cache_bytes(const mfe_ctx* ctx, int strategy);

/* v = K(u) w with u the current state (Alg. 1 for MFE_OTF/MFE_OTF_GEOM/
 * MFE_OTF_AD, Alg. 2 for MFE_T2/MFE_T4).  w_dev, v_dev: device arrays of
 * n_dofs doubles (MFE_FP64) or floats (MFE_SF_FP32); v is overwritten; w and
 * v must not overlap (MFE_EINVAL).  MFE_ESTATE before set_state or when the
 * strategy's cache (FP32 cache for MFE_SF_FP32 with T2/T4) was not built for
 * the current state.  Asynchronous. */
int mfe_apply_tangent(mfe_ctx* ctx, const void* w_dev, void* v_dev,
                      int strategy, int precision, void* stream);

/* Allocation-free variant of mfe_energy, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): *energy_dev (a device double) = the stored energy at the
 * displacement u_dev (device array of n_dofs doubles), written on `stream`;
 * asynchronous, no host synchronisation.  The per-brick partial sums go to a
 * fixed device array of 2^18 doubles (2 MiB) that each GPU holds for the
 * life of the process; a mesh with more bricks of cells (workgroups) than
 * that returns MFE_EINVAL.  Calls no hipMalloc/hipFree.  Calls on one GPU
 * share the array: calls that overlap in time (other streams, other threads,
 * other contexts on that GPU) race and must be serialised by the caller. */
int mfe_energy_noalloc(mfe_ctx* ctx, const double* u_dev, double* energy_dev, void* stream);

/* r = residual of the weak form at displacement u (eq. F without traction):
 * r_(a,i) = sum_cells sum_q JxW_q P_iA(F_q) Grad_A N_a, zero at constrained
 * dofs.  u_dev, r_dev: device arrays of n_dofs doubles, must not overlap.
 * Does not change the state.  Asynchronous (det F is not checked). */
int mfe_residual(mfe_ctx* ctx, const double* u_dev, double* r_dev, void* stream);

/* *energy_host = stored energy sum_cells sum_q JxW_q Psi(F_q) of the law of
 * eq. hypref at displacement u (u_dev: device array of n_dofs doubles);
 * per-brick partial sums in a fixed order, so the result is reproducible.
 * Not finite if det F <= 0 somewhere.  Synchronises the stream. */
int mfe_energy(mfe_ctx* ctx, const double* u_dev, double* energy_host, void* stream);

/* ---------------------------------------------------------------------------
 * Newton-CG solver (Sec. 2.2-2.3): Newton's method on the weak form with the
 * tangent applied matrix-free inside a preconditioned (Jacobi or geometric
 * multigrid) conjugate gradient method.  Dirichlet data live on the
 * constrained dofs (mfe_set_constraints): the residual vanishes there, and a
 * load step that moves the prescribed values is entered through the
 * linearised response to the increment (K_ff du_f = -R_f - K_fc dg,
 * du_c = dg).
 * ------------------------------------------------------------------------- */
typedef enum mfe_preconditioner {
    MFE_PC_NONE = 0,      /* plain CG */
    MFE_PC_JACOBI = 1,    /* inverse of |diagonal of K(u)| (matrix-free diagonal) */
    MFE_PC_GMG = 2,       /* one geometric multigrid V-cycle (Sec. 2.3): nested
                             boxes, each coarser one halving the cell counts
                             while all three are even; level operators K(u_l)
                             at the nodal interpolant u_l of the state;
                             Chebyshev-Jacobi pre- and post-smoothing;
                             Chebyshev-Jacobi on the coarsest level */
    MFE_PC_GMG_NET = 3    /* the V-cycle with the learned correction
                             (mfe_set_network) inside the finest level's
                             post-smoother: its last Chebyshev step is replaced
                             by x += alpha N, N the network's correction of the
                             residual r1 = r - K x left by the earlier steps,
                             alpha = N.r1 / N.K N (the step that minimises the
                             error's energy norm along N; no step when either
                             dot is <= 0), formed on the device, so the cycle
                             stays one kernel sequence (one graph); FP64 V-cycle
                             only (MFE_EUNSUPPORTED otherwise); inside flexible
                             CG; the correction is dropped when the residual
                             stagnates (< 10% reduction over 3 iterations) or
                             r.Br <= 0, for the rest of that solve and for later
                             solves on the context until mfe_set_network is
                             called */
} mfe_preconditioner;

typedef struct mfe_solve_opts {
    int strategy;         /* apply strategy used inside CG (mfe_strategy) */
    int preconditioner;   /* mfe_preconditioner */
    int max_newton;       /* Newton iterations allowed (>= 1) */
    int max_cg;           /* CG iterations allowed per linear solve (>= 1) */
    double newton_atol;   /* converged when ||R(u)||_2 <= newton_atol (free dofs) */
    double cg_rtol;       /* CG stops when ||r||_2 <= cg_rtol * ||b||_2 */
    int mg_levels;        /* GMG: most levels, the finest included (0: as many
                             as the cell counts allow) */
    int cheb_degree;      /* GMG: Chebyshev degree of pre- and post-smoothing (>= 1) */
    double cheb_range;    /* GMG: lambda_max / lambda_min of the smoothed spectrum (> 1) */
    int coarse_degree;    /* GMG: Chebyshev degree on the coarsest level (>= 1) */
    double coarse_range;  /* GMG: lambda_max / lambda_min on the coarsest level (> 1) */
    int mg_precision;     /* GMG: MFE_FP64, or MFE_SF_FP32 for an FP32 V-cycle (FP32
                             vectors, transfers, smoother and MFE_SF_FP32 level
                             applies) inside the FP64 CG, whose residual, dot
                             products and update stay FP64 (defect correction) */
    int mg_graph;         /* GMG: 1 = replay each V-cycle from a HIP graph
                             (captured on a private stream after every level
                             update; kernel nodes only), 0 = launch eagerly */
    int coarse_direct;    /* GMG: 1 = solve the coarsest level exactly when it has
                             at most 196 free dofs and 1024 dofs in all (its
                             dense tangent, assembled from the second-order
                             cache, is inverted on the device once per
                             linearisation point; if it is not positive
                             definite, or larger, the level is smoothed as
                             with 0), 0 = Chebyshev smoothing with
                             coarse_degree and coarse_range */
    double forcing;       /* Newton: 0 = every CG solve stops at cg_rtol; in (0, 1) =
                             inexact Newton with the Eisenstat-Walker forcing term
                             (choice 2, gamma 0.9, exponent 2): the k-th
                             correction's CG stops at
                             eta_k = 0.9 (||R_k|| / ||R_k-1||)^2, at least
                             0.9 eta_(k-1)^2 when that exceeds 0.1, at most
                             `forcing` (also eta_0), at least cg_rtol and at least
                             0.5 newton_atol / ||R_k||; the first correction of a
                             load step (the boundary increment) uses cg_rtol */
    int mg_lag;           /* GMG inside mfe_newton_solve: 0 = every CG solve
                             re-estimates the smoothed levels' spectra and
                             refactors the coarsest level; k > 0 = after such a
                             full set-up the next k CG solves of the same Newton
                             solve keep those estimates and that inverse (a
                             lagged preconditioner: the level states, caches,
                             diagonals and operators are always the current
                             ones); a CG solve that stops early and the
                             boundary increment's solve make the next set-up a
                             full one.  mfe_cg_solve and mfe_gmg_setup always
                             set up in full */
} mfe_solve_opts;

#define MFE_HISTORY 64
typedef struct mfe_solve_report {
    int converged;             /* 1 if ||R|| <= newton_atol was reached */
    int newton_iterations;     /* Newton corrections applied */
    int cg_iterations;         /* CG iterations summed over the Newton steps */
    int backtracks;            /* step halvings (line search and boundary steps) */
    int pc_fallbacks;          /* CG solves in which GMG was replaced by Jacobi
                                  (a level tangent was not positive definite) */
    int net_fallbacks;         /* CG solves in which the learned correction was
                                  dropped (stagnation or r.Br <= 0) */
    double initial_residual;   /* ||R(u_in)||_2 */
    double final_residual;     /* ||R(u_out)||_2 */
    double residual_history[MFE_HISTORY];  /* ||R|| before each correction, then the final one */
} mfe_solve_report;

/* Solve R(u) = 0 in place: u_dev (device, n_dofs doubles) holds the initial
 * guess on entry and the last iterate on return.  g_dev (device, n_dofs
 * doubles, or NULL) holds the new prescribed values at the constrained dofs
 * (other entries are ignored); with NULL the constrained values of u are
 * kept.  Each Newton step sets the state to u, builds the strategy's cache
 * (and the second-order cache for the Jacobi diagonal), solves
 * K(u) du = -R(u) by CG to cg_rtol, and updates u += a du, halving a (at
 * most 12 times) until det F > 0 everywhere and either ||R|| decreases or
 * the stored energy satisfies E(u + a du) <= E(u) + 1e-4 a R.du.  New
 * Dirichlet values enter through the first correction, K du = -R with
 * du_c = g_c - u_c, applied in full; the prescribed values are then copied
 * exactly.
 * Synchronises the stream for every dot product.  Returns MFE_OK when
 * converged, MFE_ENOTCONV when max_newton is exhausted, the line search
 * fails or the residual is not finite (the first correction inverted a
 * cell); `report` (may be NULL) is filled in every case.  CG solves that stop early (iteration limit, negative
 * curvature: the iterate so far is used) do not end the Newton iteration. */
int mfe_newton_solve(mfe_ctx* ctx, const mfe_solve_opts* opts, double* u_dev, const double* g_dev,
                     mfe_solve_report* report, void* stream);

/* Load stepping (Sec. 2.2; the twisted-beam runs of Sec. 3.1 follow a load
 * path t in (0, 1] in steps).
 *
 * Position of the driver on the path.  t: load reached by the state;
 * h: next increment (<= 0: 1 / n_steps); h_cap: largest increment allowed
 * from now on (<= 0: 1 / n_steps); prev_h: increment that led to t (<= 0:
 * none, so no extrapolation). */
typedef struct mfe_path_state {
    double t, h, h_cap, prev_h;
} mfe_path_state;

/* One Newton solve the driver attempted: the load it aimed at, its increment,
 * failed = 1 when the attempt did not converge (then retried or halved),
 * status = the mfe_newton_solve return code, and its report. */
typedef struct mfe_path_report {
    double t, h;
    int failed, status;
    mfe_solve_report solve;
} mfe_path_report;

/* Prescribed values at load t: fill values_host[n] (n = number of
 * constrained dofs, in ascending dof order) and return 0; a nonzero return
 * ends the path with MFE_EINVAL. */
typedef int (*mfe_load_fn)(double t, double* values_host, int64_t n, void* user);

/* Called after every converged step, with the stream synchronised: the new
 * position, the state u_dev at state->t and the state before it, prev_dev
 * (device arrays of n_dofs doubles, valid during the call).  A nonzero return
 * stops the path there (the driver then returns MFE_OK with state->t < 1). */
typedef int (*mfe_step_fn)(const mfe_path_state* state, const double* u_dev, const double* prev_dev, void* user);

/* Follow the load path from state->t to t = 1 with mfe_newton_solve.
 * u_dev (device, n_dofs doubles) holds the converged state at state->t on
 * entry and at the last converged load on return; prev_dev (device, n_dofs
 * doubles) holds the converged state before it when state->prev_h > 0 and is
 * kept up to date (needed only with extrapolate; may be NULL otherwise).
 * state (in/out) may be NULL: start at t = 0 with steps of 1 / n_steps.
 * Each step aims at t + h (at most 1), takes the values load(t + h), and
 * starts Newton from the linear extrapolation u + (h / prev_h) (u - prev)
 * when extrapolate != 0 and a previous step exists, else from u.  An
 * extrapolated start that does not converge is retried once from u; a step
 * that still fails sets h_cap = min(h_cap, 0.9 h) and halves h, down to
 * min_fraction.  After a converged step h grows to min(h_cap, 1.25 h).
 * reports (host, may be NULL) receives up to max_reports attempts in order;
 * *n_reports (may be NULL) their count.  The driver's two work vectors are
 * allocated with the context's other solver vectors.  Synchronises the
 * stream.  Returns MFE_OK at t = 1 (or when on_step stopped it), MFE_ENOTCONV
 * when the increment falls below min_fraction (state keeps the last converged
 * position), MFE_EINVAL for bad arguments or a failed load callback, and the
 * error of a Newton solve that fails for a reason other than convergence
 * (device errors, unsupported options). */
int mfe_solve_load_path(mfe_ctx* ctx, const mfe_solve_opts* opts, double* u_dev, double* prev_dev, int n_steps,
                        double min_fraction, int extrapolate, mfe_path_state* state, mfe_load_fn load,
                        void* load_user, mfe_step_fn on_step, void* step_user, mfe_path_report* reports,
                        int max_reports, int* n_reports, void* stream);

/* x = K(u)^-1 b by (preconditioned) CG at the current state, starting from
 * x = 0; b_dev, x_dev device arrays of n_dofs doubles (b must vanish at
 * constrained dofs).  Uses opts->strategy, preconditioner, max_cg, cg_rtol.
 * iterations_out / rel_residual_out (may be NULL) receive the iteration count
 * and ||b - K x|| / ||b|| as tracked by CG.  MFE_ENOTCONV if max_cg is
 * reached before cg_rtol.  Synchronises the stream.
 * With MFE_PC_GMG the hierarchy (one child context per coarser level, the
 * 1D transfer matrices, 8 vectors per level) is built by the first such solve
 * and kept until the mesh, material or constraints change; every solve then
 * interpolates the state to the coarser levels, builds their caches and
 * inverse diagonals, and estimates lambda_max(D^-1 K) per level from 8
 * Lanczos steps (Jacobi-CG on a fixed random right-hand side); the smoothers
 * use 1.2 times that estimate.  The V-cycle acts on the free dofs (the
 * smoother never moves a constrained entry) and the preconditioner is the
 * identity on the constrained ones.  When a level tangent is not positive
 * definite (or an interpolated state inverts a cell) the solve uses Jacobi
 * instead (counted in mfe_solve_report.pc_fallbacks by Newton). */
int mfe_cg_solve(mfe_ctx* ctx, const mfe_solve_opts* opts, const double* b_dev, double* x_dev,
                 int* iterations_out, double* rel_residual_out, void* stream);

/* The GMG preconditioner on its own, at the current state: mfe_gmg_setup
 * builds the hierarchy if needed and the level data (states, caches,
 * diagonals, eigenvalue estimates) as a CG solve with MFE_PC_GMG does;
 * mfe_gmg_apply then computes z = B r (r_dev, z_dev: device arrays of n_dofs
 * doubles, not overlapping) with the V-cycle of `opts` (precision, graph),
 * including the learned step when opts->preconditioner is MFE_PC_GMG_NET
 * (network set, FP64 V-cycle).
 * MFE_ESTATE if the level data were not set up for the current state and
 * options.  Setup synchronises the stream; apply is asynchronous. */
int mfe_gmg_setup(mfe_ctx* ctx, const mfe_solve_opts* opts, void* stream);
int mfe_gmg_apply(mfe_ctx* ctx, const mfe_solve_opts* opts, const double* r_dev, double* z_dev, void* stream);

/* y = a x + b y on device arrays of n_dofs doubles (vector helper for load
 * stepping drivers: predictors, copies with a = 1, b = 0).  Asynchronous. */
int mfe_axpby(mfe_ctx* ctx, double a, const double* x_dev, double b, double* y_dev, void* stream);

/* *result_host = x . y over the n_dofs entries of two device arrays, summed in
 * a fixed order (per-block partial sums, then one ordered sum): the same
 * inputs give the same bits.  Waits for `stream`. */
int mfe_dot(mfe_ctx* ctx, const double* x_dev, const double* y_dev, double* result_host, void* stream);

/* v = 0 at the constrained dofs (mfe_set_constraints) of a device array of
 * n_dofs doubles; no-op without constraints.  Asynchronous. */
int mfe_zero_constrained(mfe_ctx* ctx, double* v_dev, void* stream);

/* d = diagonal of K(u) at the current state (identity rows: 1 at
 * constrained dofs), from the second-order cache, which this call builds if
 * it is stale.  d_dev: device array of n_dofs doubles.  Asynchronous. */
int mfe_diagonal(mfe_ctx* ctx, double* d_dev, void* stream);

/* Summation order of mfe_apply_tangent (Alg. 1/Alg. 2 "scatter"): on = 0
 * (default), every brick of cells adds the nodes it shares with a
 * neighbouring brick with atomics, so the order of the additions at such a
 * node (and the last bits of v) can change from call to call; on != 0, the
 * bricks run as eight launches in a fixed order, one per parity class of the
 * brick position (bx & 1, by & 1, bz & 1), whose bricks share no node, and
 * shared nodes are added with plain read-add-writes: v is bitwise
 * reproducible.  Within a brick the cells' contributions are summed in a
 * fixed order in either mode.  The coloured mode is built for Q2 structured
 * boxes with the vector-ALU sweeps (MFE_FP64, MFE_SF_FP32); other meshes,
 * degrees and precisions then return MFE_EUNSUPPORTED from the apply.
 * Timing (below) covers the first to the last of the eight launches. */
int mfe_set_deterministic(mfe_ctx* ctx, int on);

/* Kernel timing of mfe_apply_tangent.  mfe_set_timing(ctx, every) records
 * the apply kernel of every `every`-th call from now on (1: every call, 0:
 * off; < 0: MFE_EINVAL) and forgets earlier records.  A recorded launch
 * carries a start and a stop HIP event that its dispatch packet records on the
 * launch stream (no extra commands between the kernels); a timestamped
 * dispatch still costs a few microseconds of stream time, hence the interval.
 * mfe_apply_kernel_ms returns the average duration in milliseconds of the
 * recorded launches and their number in *count_out (may be NULL); -1 and 0 if
 * none.  Synchronizes with the recorded events. */
int mfe_set_timing(mfe_ctx* ctx, int every);
double mfe_apply_kernel_ms(mfe_ctx* ctx, int* count_out);

/* ---------------------------------------------------------------------------
 * Learned smoother correction (the method's "learned parts" growth direction):
 * a 3D convolutional network on patches of 4x4x4 Q2 cells (9x9x9 nodes;
 * patch (px,py,pz) holds nodes (8px+i, 8py+j, 8pz+k), i,j,k = 0..8, so
 * neighbouring patches share face nodes).  Input channels per node: the
 * residual (3 components) divided by the patch RMS s_p of the residual, and
 * I1 - 3, I2 - 3, J - 1 of C = F^T F (F at the centres of the node's cells,
 * averaged); output: 3 channels, the correction divided by s_p.  Layers:
 * conv 6->32 + ReLU, conv 32->32 + ReLU, conv 32->3, 3x3x3 kernels, zero
 * padding.  Parameters (FP32, MFE_NET_PARAMS): per layer W[co][ci][tap]
 * (tap = a + 3b + 9c for the offset (a-1, b-1, c-1)) then bias[co].
 * Activations are [patch][channel][729] floats with node v = i + 9j + 81k.
 * All of it FP32; every pointer below is a device pointer unless named _host.
 * ------------------------------------------------------------------------- */
#define MFE_NET_PARAMS 35491
/* Network variants: MFE_NET_RELU as above; MFE_NET_LINEAR drops the ReLUs,
 * the biases, the patch scaling (s_p = 1) and the invariant channels (0), so
 * that the correction N is a fixed linear map of the residual (the step
 * alpha is still chosen per application). */
#define MFE_NET_RELU 0
#define MFE_NET_LINEAR 1

/* Copy the network parameters (host, MFE_NET_PARAMS floats) and its variant
 * into the context for MFE_PC_GMG_NET; NULL clears them.  MFE_EINVAL for
 * non-finite values or an unknown variant.  Synchronous. */
int mfe_set_network(mfe_ctx* ctx, const float* params_host, int variant);

/* Number of patches of the mesh (0 unless degree 2 with nx, ny, nz
 * divisible by 4). */
int64_t mfe_patch_count(const mfe_ctx* ctx);

/* feat[P][6][729] and scale[P] (s_p) from a residual r (n_dofs doubles) at
 * the current state, for the network `variant`.  MFE_ESTATE without a state, MFE_EUNSUPPORTED without
 * patches.  Asynchronous. */
int mfe_patch_features(mfe_ctx* ctx, const double* r_dev, float* feat_dev, float* scale_dev, int variant,
                       void* stream);

/* t[P][3][729] = e at the patch nodes / s_p (0 where s_p = 0). */
int mfe_patch_targets(mfe_ctx* ctx, const double* e_dev, const float* scale_dev, float* t_dev, void* stream);

/* z += alpha * (patch outputs y[P][3][729] times s_p, averaged over the
 * patches that hold each node).  Constrained dofs are not special here. */
int mfe_patch_scatter(mfe_ctx* ctx, const float* y_dev, const float* scale_dev, double alpha, double* z_dev,
                      void* stream);

/* Adjoint of mfe_patch_scatter: dy[P][3][729] = alpha * s_p * g(node) / (number
 * of patches holding the node), i.e. d L / d y for d L / d z = g (g: n_dofs
 * doubles).  Used to train the network on a loss of the assembled z. */
int mfe_patch_adjoint(mfe_ctx* ctx, const double* g_dev, const float* scale_dev, double alpha, float* dy_dev,
                      void* stream);

/* y[P][3][729] = network(x[P][6][729]); act[2][P][32][729] receives the
 * hidden activations (needed by the backward pass).  Asynchronous. */
int mfe_net_forward(const float* params_dev, const float* x_dev, int n_patches, int variant, float* act_dev,
                    float* y_dev, void* stream);

/* grad[MFE_NET_PARAMS] = d loss / d params given dy = d loss / d y, with x
 * and act from the forward pass; work: [2][P][32][729] floats of scratch.
 * Weight gradients are per-workgroup sums in a fixed order (deterministic).
 * Asynchronous. */
int mfe_net_backward(const float* params_dev, const float* x_dev, const float* act_dev, const float* dy_dev,
                     int n_patches, int variant, float* work_dev, float* grad_dev, void* stream);

/* *loss_host = mean of (y - t)^2 over n entries (accumulated in FP64); dy
 * (may be NULL) = 2 (y - t) / n.  scratch: 1025 doubles.  Synchronises. */
int mfe_net_loss(const float* y_dev, const float* t_dev, int64_t n, float* dy_dev, double* scratch_dev,
                 double* loss_host, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected for
 * step >= 1) on MFE_NET_PARAMS parameters; m, v: moment buffers (start at 0).
 * Asynchronous. */
int mfe_net_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int step, float lr,
                 void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MFE_H */
