/* The oracle's tangent K(u) of a structured Q_p box assembled into CSR on all
 * host cores: the "classical" assembled-matrix baseline the paper sets the
 * matrix-free operators against (Sec. 3.2.2), sized for the benchmark's
 * 48^3 Q2 box (2.7M rows, about 5e8 stored entries), where the numpy
 * assembly would take hours.
 *
 * TEST AND BASELINE INFRASTRUCTURE ONLY (see the oracle package docstring).
 * It computes the same definition as the numpy oracle, term by term:
 *   K_(a,i),(b,j) = sum_cells sum_q w_q det J_g  dN_a/dX_A  L_iAjB(F_q)  dN_b/dX_B
 * with the explicit 81-entry tangent of eq. L for the energy of eq. hypref,
 *   L_iAjB = mu d_ij d_AB + 2 lam Finv_Ai Finv_Bj + (mu - 2 lam log J) Finv_Aj Finv_Bi,
 * F = I + sum_a u_a (x) Grad N_a, Grad N_a = J_g^-T grad_xi N_a, and J_g the
 * trilinear map of the cell's 8 vertices.  The 1D tables (Gauss weights,
 * gradients of the tensor-product basis and of the trilinear vertex functions
 * at the quadrature points) come from the numpy oracle.  No constraints.
 *
 * Numbering: node (I, J, K) -> I + Nx (J + Ny K), dof = 3 node + c; cell
 * (ex, ey, ez) -> ex + nx (ey + ny ez); vertices likewise with nx + 1, ny + 1;
 * local node a = i + n (j + n k), n = p + 1; local vertex v = vx + 2 vy + 4 vz.
 *
 * Row pattern: a dof couples with every dof of the nodes of the cells that
 * hold its node, i.e. in each direction with the node range
 * [p cmin, p (cmax + 1)] of those cells; columns are stored sorted.  Cells are
 * added in eight passes by the parity of (ex, ey, ez): cells of one pass share
 * no node, so the threads of a pass write disjoint entries. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static void node_range(int I, int p, int ncell, int* lo, int* hi) {
    int cmin = (I + p - 1) / p - 1, cmax = I / p;
    if (cmin < 0) cmin = 0;
    if (cmax > ncell - 1) cmax = ncell - 1;
    *lo = p * cmin;
    *hi = p * (cmax + 1);
}

/* indptr[0..n_dofs]: row starts.  Returns the number of stored entries. */
int64_t csr_pattern_box(int nx, int ny, int nz, int p, int64_t* indptr) {
    const int64_t Nx = (int64_t)p * nx + 1, Ny = (int64_t)p * ny + 1, Nz = (int64_t)p * nz + 1;
    const int64_t nn = Nx * Ny * Nz;
    indptr[0] = 0;
#pragma omp parallel for schedule(static)
    for (int64_t node = 0; node < nn; ++node) {
        const int I = (int)(node % Nx), J = (int)((node / Nx) % Ny), K = (int)(node / (Nx * Ny));
        int lx, hx, ly, hy, lz, hz;
        node_range(I, p, nx, &lx, &hx);
        node_range(J, p, ny, &ly, &hy);
        node_range(K, p, nz, &lz, &hz);
        const int64_t cnt = 3 * (int64_t)(hx - lx + 1) * (hy - ly + 1) * (hz - lz + 1);
        for (int c = 0; c < 3; ++c) indptr[3 * node + c + 1] = cnt;
    }
    for (int64_t r = 0; r < 3 * nn; ++r) indptr[r + 1] += indptr[r];
    return indptr[3 * nn];
}

static double inv3(const double a[3][3], double b[3][3]) {
    const double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
    const double c01 = a[0][2] * a[2][1] - a[0][1] * a[2][2];
    const double c02 = a[0][1] * a[1][2] - a[0][2] * a[1][1];
    const double c10 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
    const double c11 = a[0][0] * a[2][2] - a[0][2] * a[2][0];
    const double c12 = a[0][2] * a[1][0] - a[0][0] * a[1][2];
    const double c20 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
    const double c21 = a[0][1] * a[2][0] - a[0][0] * a[2][1];
    const double c22 = a[0][0] * a[1][1] - a[0][1] * a[1][0];
    const double det = a[0][0] * c00 + a[0][1] * c10 + a[0][2] * c20;
    const double r = 1.0 / det;
    b[0][0] = c00 * r; b[0][1] = c01 * r; b[0][2] = c02 * r;
    b[1][0] = c10 * r; b[1][1] = c11 * r; b[1][2] = c12 * r;
    b[2][0] = c20 * r; b[2][1] = c21 * r; b[2][2] = c22 * r;
    return det;
}

/* Fills indices and data (indptr from csr_pattern_box).  qw[nq3], tri_grads
 * [nq3][8][3] (dN1_v/dxi_A), basis_grads [nq3][n3][3] (dN_a/dxi_B).  Returns
 * the number of threads used, or -1 if det J_g <= 0 or det F <= 0 somewhere. */
int csr_assemble_box(int nx, int ny, int nz, int p, int nq3, const double* verts, const double* u, double mu,
                     double lam, const double* qw, const double* tri_grads, const double* basis_grads,
                     const int64_t* indptr, int32_t* indices, double* data) {
    const int n = p + 1, n3 = n * n * n, nd = 3 * n3;
    const int64_t Nx = (int64_t)p * nx + 1, Ny = (int64_t)p * ny + 1, Nz = (int64_t)p * nz + 1;
    const int64_t nn = Nx * Ny * Nz;
    int threads = 1, bad = 0;
    /* column indices, row by row, in the sorted order of the pattern */
#pragma omp parallel for schedule(static)
    for (int64_t node = 0; node < nn; ++node) {
        const int I = (int)(node % Nx), J = (int)((node / Nx) % Ny), K = (int)(node / (Nx * Ny));
        int lx, hx, ly, hy, lz, hz;
        node_range(I, p, nx, &lx, &hx);
        node_range(J, p, ny, &ly, &hy);
        node_range(K, p, nz, &lz, &hz);
        for (int c = 0; c < 3; ++c) {
            int64_t pos = indptr[3 * node + c];
            for (int kk = lz; kk <= hz; ++kk)
                for (int jj = ly; jj <= hy; ++jj)
                    for (int ii = lx; ii <= hx; ++ii)
                        for (int cc = 0; cc < 3; ++cc) {
                            indices[pos] = (int32_t)(3 * (ii + Nx * (jj + Ny * kk)) + cc);
                            data[pos++] = 0.0;
                        }
        }
    }
#pragma omp parallel
    {
#pragma omp single
        threads = omp_get_num_threads();
        double* Ke = (double*)malloc(sizeof(double) * nd * nd);
        double* gN = (double*)malloc(sizeof(double) * n3 * 3);
        double* T = (double*)malloc(sizeof(double) * n3 * 27);
        int64_t* gnode = (int64_t*)malloc(sizeof(int64_t) * n3);
        for (int colour = 0; colour < 8; ++colour) {
            const int ox = colour & 1, oy = (colour >> 1) & 1, oz = colour >> 2;
            const int mx = (nx - ox + 1) / 2, my = (ny - oy + 1) / 2, mz = (nz - oz + 1) / 2;
            const int64_t ncol = (int64_t)mx * my * mz;
#pragma omp for schedule(dynamic, 8)
            for (int64_t t = 0; t < ncol; ++t) {
                const int ex = 2 * (int)(t % mx) + ox, ey = 2 * (int)((t / mx) % my) + oy, ez = 2 * (int)(t / ((int64_t)mx * my)) + oz;
                double X[8][3];
                for (int v = 0; v < 8; ++v) {
                    const int64_t vid = (ex + (v & 1)) + (int64_t)(nx + 1) * ((ey + ((v >> 1) & 1)) + (int64_t)(ny + 1) * (ez + (v >> 2)));
                    for (int d = 0; d < 3; ++d) X[v][d] = verts[3 * vid + d];
                }
                for (int a = 0; a < n3; ++a) {
                    const int i = a % n, j = (a / n) % n, k = a / (n * n);
                    gnode[a] = (p * ex + i) + Nx * ((p * ey + j) + Ny * (int64_t)(p * ez + k));
                }
                memset(Ke, 0, sizeof(double) * nd * nd);
                for (int q = 0; q < nq3; ++q) {
                    double Jg[3][3] = {{0}}, Ji[3][3];
                    for (int v = 0; v < 8; ++v)
                        for (int d = 0; d < 3; ++d)
                            for (int A = 0; A < 3; ++A) Jg[d][A] += X[v][d] * tri_grads[(q * 8 + v) * 3 + A];
                    const double detg = inv3(Jg, Ji); /* Ji[A][d] */
                    if (!(detg > 0.0)) {
#pragma omp atomic write
                        bad = 1;
                    }
                    for (int a = 0; a < n3; ++a)
                        for (int A = 0; A < 3; ++A) {
                            double s = 0.0;
                            for (int B = 0; B < 3; ++B) s += Ji[B][A] * basis_grads[(q * n3 + a) * 3 + B];
                            gN[3 * a + A] = s;
                        }
                    double F[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, Fi[3][3];
                    for (int a = 0; a < n3; ++a)
                        for (int i = 0; i < 3; ++i)
                            for (int A = 0; A < 3; ++A) F[i][A] += u[3 * gnode[a] + i] * gN[3 * a + A];
                    const double Jd = inv3(F, Fi); /* Fi[A][i] = (F^-1)_Ai */
                    if (!(Jd > 0.0)) {
#pragma omp atomic write
                        bad = 1;
                    }
                    const double lJ = log(Jd);
                    double L[3][3][3][3];
                    for (int i = 0; i < 3; ++i)
                        for (int A = 0; A < 3; ++A)
                            for (int j = 0; j < 3; ++j)
                                for (int B = 0; B < 3; ++B)
                                    L[i][A][j][B] = (i == j && A == B ? mu : 0.0) + 2.0 * lam * Fi[A][i] * Fi[B][j] +
                                                    (mu - 2.0 * lam * lJ) * Fi[A][j] * Fi[B][i];
                    const double JxW = qw[q] * detg;
                    /* T[a][i][j][B] = sum_A dN_a/dX_A L_iAjB */
                    for (int a = 0; a < n3; ++a)
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j)
                                for (int B = 0; B < 3; ++B) {
                                    double s = 0.0;
                                    for (int A = 0; A < 3; ++A) s += gN[3 * a + A] * L[i][A][j][B];
                                    T[((a * 3 + i) * 3 + j) * 3 + B] = s;
                                }
                    /* Ke[(a,i)][(b,j)] += JxW sum_B T[a][i][j][B] dN_b/dX_B */
                    for (int a = 0; a < n3; ++a)
                        for (int i = 0; i < 3; ++i) {
                            double* row = Ke + (size_t)(3 * a + i) * nd;
                            for (int b = 0; b < n3; ++b)
                                for (int j = 0; j < 3; ++j) {
                                    const double* t3 = T + ((a * 3 + i) * 3 + j) * 3;
                                    row[3 * b + j] += JxW * (t3[0] * gN[3 * b] + t3[1] * gN[3 * b + 1] + t3[2] * gN[3 * b + 2]);
                                }
                        }
                }
                /* add into the rows of the cell's dofs (no other cell of this pass touches them) */
                for (int a = 0; a < n3; ++a) {
                    const int64_t node = gnode[a];
                    const int I = (int)(node % Nx), J = (int)((node / Nx) % Ny), K = (int)(node / (Nx * Ny));
                    int lx, hx, ly, hy, lz, hz;
                    node_range(I, p, nx, &lx, &hx);
                    node_range(J, p, ny, &ly, &hy);
                    node_range(K, p, nz, &lz, &hz);
                    const int64_t rx = hx - lx + 1, ry = hy - ly + 1;
                    for (int i = 0; i < 3; ++i) {
                        const int64_t start = indptr[3 * node + i];
                        const double* row = Ke + (size_t)(3 * a + i) * nd;
                        for (int b = 0; b < n3; ++b) {
                            const int bi = b % n, bj = (b / n) % n, bk = b / (n * n);
                            const int64_t off = (((int64_t)(p * ez + bk - lz) * ry + (p * ey + bj - ly)) * rx + (p * ex + bi - lx)) * 3;
                            for (int j = 0; j < 3; ++j) data[start + off + j] += row[3 * b + j];
                        }
                    }
                }
            }
        }
        free(Ke);
        free(gN);
        free(T);
        free(gnode);
    }
    return bad ? -1 : threads;
}
