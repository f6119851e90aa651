// Device-side building blocks of the matrix-free tangent (gfx950).  The
// sum-factorization kernels and the cached-data point-wise products are
// templates over the arithmetic type R (double, or float for the mixed-precision
// sweeps); kinematics and everything that evaluates F, J and log J is FP64.
//
//  * 1D sum-factorization kernels with the even-odd split of centro-symmetric
//    and centro-antisymmetric matrices (the 1D kernels of Sec. 2.4).
//  * 3x3 tensor algebra.
//  * The point-wise operations of the quadrature loop (Sec. 2.5): on-the-fly
//    G = L : Grad w in closed form and by forward-mode dual numbers (the
//    "seed" formulation, eq. LG), the current-configuration products with
//    cached second-order (T2) and fourth-order (T4) data (Alg. 2), and the
//    per-point cache construction from F.
//
// Everything here is __host__ __device__ so that the arithmetic can also be
// exercised by a host build.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MFE_HD __host__ __device__ __forceinline__

namespace mfe {

MFE_HD double fmar(double a, double b, double c) { return fma(a, b, c); }
MFE_HD float fmar(float a, float b, float c) { return fmaf(a, b, c); }

// --------------------------------------------------------------------------
// 1D matrices in even-odd form.
//
// A matrix A (N x N) is centro-symmetric if A[N-1-q][N-1-i] = A[q][i] (the
// Lagrange interpolation matrix from symmetric support points to symmetric
// Gauss points) and centro-antisymmetric if A[N-1-q][N-1-i] = -A[q][i] (a
// derivative matrix).  With x_e[i] = x[i] + x[N-1-i], x_o[i] = x[i] - x[N-1-i]
// (i < N/2) and, for odd N, x_e[N/2] = x[N/2]:
//   symmetric:      y[q] = E[q].x_e + O[q].x_o,  y[N-1-q] = E[q].x_e - O[q].x_o
//   antisymmetric:  y[q] = O[q].x_o + E[q].x_e,  y[N-1-q] = O[q].x_o - E[q].x_e
// where for q < N/2:  E[q][i] = (A[q][i] + A[q][N-1-i]) / 2 (i < N/2),
//                     E[q][N/2] = A[q][N/2] (odd N),
//                     O[q][i] = (A[q][i] - A[q][N-1-i]) / 2,
// and the middle row of odd N is E[N/2][.] = A[N/2][.] (symmetric, acting on
// x_e) or O[N/2][i] = A[N/2][i] (antisymmetric, acting on x_o).
// --------------------------------------------------------------------------
template <int N, typename R = double>
struct EO {
    static constexpr int H = (N + 1) / 2;
    static constexpr int M = N / 2;
    R E[H][H];
    R O[H][M > 0 ? M : 1];
};

template <int N, typename R = double>
struct Tables {
    EO<N, R> S;     // y[q] = sum_i S[q][i] x[i]   nodal values -> Gauss points
    EO<N, R> St;    // y[i] = sum_q S[q][i] x[q]   transpose
    EO<N, R> D;     // y[q] = sum_l D[q][l] x[l]   derivative collocated on Gauss points
    EO<N, R> Dt;    // y[l] = sum_q D[q][l] x[q]   transpose
    double qp[N];   // Gauss points on [0, 1]
    double qw[N];   // Gauss weights on [0, 1]
};

template <int N, bool ANTI, typename R>
MFE_HD void apply_eo(const EO<N, R>& T, const R (&x)[N], R (&y)[N]) {
    constexpr int H = EO<N, R>::H;
    constexpr int M = EO<N, R>::M;
    R xe[H];
    R xo[M > 0 ? M : 1];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        xe[i] = x[i] + x[N - 1 - i];
        xo[i] = x[i] - x[N - 1 - i];
    }
    if constexpr (N % 2 == 1) xe[M] = x[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
        R a = 0, b = 0;
#pragma unroll
        for (int i = 0; i < H; ++i) a = fmar(T.E[q][i], xe[i], a);
#pragma unroll
        for (int i = 0; i < M; ++i) b = fmar(T.O[q][i], xo[i], b);
        if constexpr (ANTI) {
            y[q] = b + a;
            y[N - 1 - q] = b - a;
        } else {
            y[q] = a + b;
            y[N - 1 - q] = a - b;
        }
    }
    if constexpr (N % 2 == 1) {
        R m = 0;
        if constexpr (ANTI) {
#pragma unroll
            for (int i = 0; i < M; ++i) m = fmar(T.O[M][i], xo[i], m);
        } else {
#pragma unroll
            for (int i = 0; i < H; ++i) m = fmar(T.E[M][i], xe[i], m);
        }
        y[M] = m;
    }
}

// --------------------------------------------------------------------------
// 3x3 algebra (row-major a[i][j])
// --------------------------------------------------------------------------
template <typename R>
MFE_HD void matmul3(const R a[3][3], const R b[3][3], R c[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c[i][j] = fmar(a[i][0], b[0][j], fmar(a[i][1], b[1][j], a[i][2] * b[2][j]));
}

// c = a * b^T
template <typename R>
MFE_HD void matmul3_bt(const R a[3][3], const R b[3][3], R c[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c[i][j] = fmar(a[i][0], b[j][0], fmar(a[i][1], b[j][1], a[i][2] * b[j][2]));
}

// adjugate (transpose of the cofactor matrix) and determinant: a^-1 = adj / det
MFE_HD double adj_det3(const double a[3][3], double c[3][3]) {
    c[0][0] = fma(a[1][1], a[2][2], -a[1][2] * a[2][1]);
    c[0][1] = fma(a[0][2], a[2][1], -a[0][1] * a[2][2]);
    c[0][2] = fma(a[0][1], a[1][2], -a[0][2] * a[1][1]);
    c[1][0] = fma(a[1][2], a[2][0], -a[1][0] * a[2][2]);
    c[1][1] = fma(a[0][0], a[2][2], -a[0][2] * a[2][0]);
    c[1][2] = fma(a[0][2], a[1][0], -a[0][0] * a[1][2]);
    c[2][0] = fma(a[1][0], a[2][1], -a[1][1] * a[2][0]);
    c[2][1] = fma(a[0][1], a[2][0], -a[0][0] * a[2][1]);
    c[2][2] = fma(a[0][0], a[1][1], -a[0][1] * a[1][0]);
    return fma(a[0][0], c[0][0], fma(a[0][1], c[1][0], a[0][2] * c[2][0]));
}

// Voigt order (xx, yy, zz, yz, xz, xy); packed upper triangle of a 6x6
// symmetric matrix, row-major: index of (r, c), r <= c.
MFE_HD constexpr int voigt_packed(int r, int c) { return r * 6 - (r * (r - 1)) / 2 + (c - r); }

// --------------------------------------------------------------------------
// Trilinear geometry.  Edge vectors of a cell with vertices X_v,
// v = vx + 2 vy + 4 vz:  ex[a] = X_{1,a} - X_{0,a} for the 4 x-edges
// (a = (vy, vz) = 0..3), likewise ey (a = (vx, vz)) and ez (a = (vx, vy)).
// dX/dxi_0 = sum_a bilinear weight(xi_1, xi_2)_a ex[a], etc.
// --------------------------------------------------------------------------
struct CellEdges {
    double ex[4][3], ey[4][3], ez[4][3];
};

MFE_HD void edges_from_vertices(const double X[8][3], CellEdges& E) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        E.ex[0][d] = X[1][d] - X[0][d];
        E.ex[1][d] = X[3][d] - X[2][d];
        E.ex[2][d] = X[5][d] - X[4][d];
        E.ex[3][d] = X[7][d] - X[6][d];
        E.ey[0][d] = X[2][d] - X[0][d];
        E.ey[1][d] = X[3][d] - X[1][d];
        E.ey[2][d] = X[6][d] - X[4][d];
        E.ey[3][d] = X[7][d] - X[5][d];
        E.ez[0][d] = X[4][d] - X[0][d];
        E.ez[1][d] = X[5][d] - X[1][d];
        E.ez[2][d] = X[6][d] - X[2][d];
        E.ez[3][d] = X[7][d] - X[3][d];
    }
}

// Jg[d][A] = dX_d / dxi_A at reference point xi, from the 12 edge vectors
// stored contiguously as edges[12][3] (x-edges, y-edges, z-edges).
MFE_HD void jacobian_from_edges(const double* edges, double x0, double x1, double x2,
                                double Jg[3][3]) {
    const double m0 = 1.0 - x0, m1 = 1.0 - x1, m2 = 1.0 - x2;
    const double wx[4] = {m1 * m2, x1 * m2, m1 * x2, x1 * x2};
    const double wy[4] = {m0 * m2, x0 * m2, m0 * x2, x0 * x2};
    const double wz[4] = {m0 * m1, x0 * m1, m0 * x1, x0 * x1};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Jg[d][0] = fma(wx[0], edges[0 * 3 + d], fma(wx[1], edges[1 * 3 + d],
                   fma(wx[2], edges[2 * 3 + d], wx[3] * edges[3 * 3 + d])));
        Jg[d][1] = fma(wy[0], edges[4 * 3 + d], fma(wy[1], edges[5 * 3 + d],
                   fma(wy[2], edges[6 * 3 + d], wy[3] * edges[7 * 3 + d])));
        Jg[d][2] = fma(wz[0], edges[8 * 3 + d], fma(wz[1], edges[9 * 3 + d],
                   fma(wz[2], edges[10 * 3 + d], wz[3] * edges[11 * 3 + d])));
    }
}

// --------------------------------------------------------------------------
// Kinematics at a quadrature point: F = I + Grad u with Grad u = du_ref Jginv.
// --------------------------------------------------------------------------
struct Kin {
    double Finv[3][3];
    double lJ;     // log det F
    double J;      // det F
};

MFE_HD void kinematics(const double du[3][3], const double Jginv[3][3], double F[3][3], Kin& k) {
    matmul3(du, Jginv, F);
    F[0][0] += 1.0;
    F[1][1] += 1.0;
    F[2][2] += 1.0;
    double adj[3][3];
    k.J = adj_det3(F, adj);
    const double rJ = 1.0 / k.J;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) k.Finv[i][j] = adj[i][j] * rJ;
    k.lJ = log(k.J);
}

// --------------------------------------------------------------------------
// On the fly, closed form (reference configuration, Sec. 2.5.1):
//   G = L : Hw = mu Hw + 2 lam tr(F^-1 Hw) F^-T + (mu - 2 lam log J) F^-T Hw^T F^-T
// returned already multiplied by JxW and pulled back: Q = JxW G Jginv^T, so
// that the test contraction is sum_A Q[c][A] dN_a/dxi_A.
// --------------------------------------------------------------------------
MFE_HD void pointwise_otf(const double dw[3][3], const double Jginv[3][3], const Kin& k,
                          double mu, double lam, double JxW, double Q[3][3]) {
    double Hw[3][3], Y[3][3], Z[3][3], G[3][3];
    matmul3(dw, Jginv, Hw);           // Grad w
    matmul3(Hw, k.Finv, Y);           // Hw F^-1
    matmul3(k.Finv, Y, Z);            // F^-1 Hw F^-1
    const double tr = Y[0][0] + Y[1][1] + Y[2][2];
    const double a = mu * JxW;
    const double b = 2.0 * lam * tr * JxW;
    const double c = (mu - 2.0 * lam * k.lJ) * JxW;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A)
            G[i][A] = fma(a, Hw[i][A], fma(b, k.Finv[A][i], c * Z[A][i]));
    matmul3_bt(G, Jginv, Q);
}

// --------------------------------------------------------------------------
// Forward-mode dual numbers: the "seed" evaluation of Sec. 2.5.1.  P(F) is
// written once, generically; evaluating it on dual numbers whose derivative
// part is the seed dF/dxi = Grad w yields dP/dxi = L : Grad w without ever
// forming L (eq. LG).
// --------------------------------------------------------------------------
struct Dual {
    double v, d;
};
MFE_HD Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
MFE_HD Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
MFE_HD Dual operator*(Dual a, Dual b) { return {a.v * b.v, fma(a.v, b.d, a.d * b.v)}; }
MFE_HD Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
MFE_HD Dual dual_fms(Dual a, Dual b, Dual c, Dual e) {  // a*b - c*e
    return {fma(a.v, b.v, -c.v * e.v), fma(a.d, b.v, fma(a.v, b.d, -fma(c.d, e.v, c.v * e.d)))};
}
MFE_HD Dual dual_recip(Dual a) {
    const double r = 1.0 / a.v;
    return {r, -a.d * r * r};
}
MFE_HD Dual dual_log(Dual a) { return {log(a.v), a.d / a.v}; }

// First Piola-Kirchhoff stress of eq. hypref, P = mu F + (2 lam log J - mu) F^-T,
// for any scalar type with +, -, *, reciprocal and log.
MFE_HD void piola_dual(const Dual F[3][3], double mu, double lam, Dual P[3][3]) {
    Dual c[3][3];  // cofactor matrix: c[i][j] = (adj F)[j][i], F^-T = c / J
    c[0][0] = dual_fms(F[1][1], F[2][2], F[1][2], F[2][1]);
    c[1][0] = dual_fms(F[0][2], F[2][1], F[0][1], F[2][2]);
    c[2][0] = dual_fms(F[0][1], F[1][2], F[0][2], F[1][1]);
    c[0][1] = dual_fms(F[1][2], F[2][0], F[1][0], F[2][2]);
    c[1][1] = dual_fms(F[0][0], F[2][2], F[0][2], F[2][0]);
    c[2][1] = dual_fms(F[0][2], F[1][0], F[0][0], F[1][2]);
    c[0][2] = dual_fms(F[1][0], F[2][1], F[1][1], F[2][0]);
    c[1][2] = dual_fms(F[0][1], F[2][0], F[0][0], F[2][1]);
    c[2][2] = dual_fms(F[0][0], F[1][1], F[0][1], F[1][0]);
    const Dual J = F[0][0] * c[0][0] + F[0][1] * c[0][1] + F[0][2] * c[0][2];
    const Dual rJ = dual_recip(J);
    const Dual lJ = dual_log(J);
    const Dual coef = (2.0 * lam) * lJ - Dual{mu, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) P[i][A] = mu * F[i][A] + coef * (c[i][A] * rJ);
}

// G = dP/dxi with F(xi) = I + Hu + xi Hw; returns Q = JxW G Jginv^T.
MFE_HD void pointwise_otf_ad(const double du[3][3], const double dw[3][3], const double Jginv[3][3],
                             double mu, double lam, double JxW, double Q[3][3]) {
    double Hu[3][3], Hw[3][3];
    matmul3(du, Jginv, Hu);
    matmul3(dw, Jginv, Hw);
    Dual F[3][3], P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) F[i][A] = Dual{Hu[i][A] + (i == A ? 1.0 : 0.0), Hw[i][A]};
    piola_dual(F, mu, lam, P);
    double G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) G[i][A] = JxW * P[i][A].d;
    matmul3_bt(G, Jginv, Q);
}

// --------------------------------------------------------------------------
// Split neo-Hookean law (Sec. 3.3, eq. hypcomplex) with bulk modulus kappa:
//   Psi = mu/2 (J^-2/3 tr C - 3) + kappa/2 ((J^2 - 1)/2 - log J)
//   P   = a (F - I1/3 F^-T) + b F^-T,   a = mu J^-2/3, b = kappa/2 (J^2 - 1),
// I1 = tr C.  Its tangent is never written out here: the on-the-fly apply
// differentiates P with dual numbers (the same "seed" evaluation as for the
// other law) and the fourth-order cache is filled from nine such directional
// derivatives -- the model-independent strategies of the paper.
// --------------------------------------------------------------------------
MFE_HD Dual dual_pow(Dual a, double e) {
    const double v = pow(a.v, e);
    return {v, e * v / a.v * a.d};
}

MFE_HD void piola_split_dual(const Dual F[3][3], double mu, double kappa, Dual P[3][3]) {
    Dual c[3][3];  // cofactor matrix: F^-T = c / J
    c[0][0] = dual_fms(F[1][1], F[2][2], F[1][2], F[2][1]);
    c[1][0] = dual_fms(F[0][2], F[2][1], F[0][1], F[2][2]);
    c[2][0] = dual_fms(F[0][1], F[1][2], F[0][2], F[1][1]);
    c[0][1] = dual_fms(F[1][2], F[2][0], F[1][0], F[2][2]);
    c[1][1] = dual_fms(F[0][0], F[2][2], F[0][2], F[2][0]);
    c[2][1] = dual_fms(F[0][2], F[1][0], F[0][0], F[1][2]);
    c[0][2] = dual_fms(F[1][0], F[2][1], F[1][1], F[2][0]);
    c[1][2] = dual_fms(F[0][1], F[2][0], F[0][0], F[2][1]);
    c[2][2] = dual_fms(F[0][0], F[1][1], F[0][1], F[1][0]);
    const Dual J = F[0][0] * c[0][0] + F[0][1] * c[0][1] + F[0][2] * c[0][2];
    const Dual rJ = dual_recip(J);
    Dual I1{0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) I1 = I1 + F[i][A] * F[i][A];
    const Dual a = mu * dual_pow(J, -2.0 / 3.0);
    const Dual b = (0.5 * kappa) * (J * J - Dual{1.0, 0.0});
    const Dual third = (1.0 / 3.0) * I1;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) {
            const Dual G = c[i][A] * rJ;
            P[i][A] = a * (F[i][A] - third * G) + b * G;
        }
}

// dP/dxi along the seed Hw on the split law; returns Q = JxW G Jginv^T
MFE_HD void pointwise_otf_ad_split(const double du[3][3], const double dw[3][3], const double Jginv[3][3],
                                   double mu, double kappa, double JxW, double Q[3][3]) {
    double Hu[3][3], Hw[3][3];
    matmul3(du, Jginv, Hu);
    matmul3(dw, Jginv, Hw);
    Dual F[3][3], P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) F[i][A] = Dual{Hu[i][A] + (i == A ? 1.0 : 0.0), Hw[i][A]};
    piola_split_dual(F, mu, kappa, P);
    double G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) G[i][A] = JxW * P[i][A].d;
    matmul3_bt(G, Jginv, Q);
}

// residual integrand of the split law: Q = JxW P Jginv^T
MFE_HD void pointwise_piola_split(const double F[3][3], const Kin& k, double mu, double kappa,
                                  const double Jginv[3][3], double JxW, double Q[3][3]) {
    double I1 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) I1 = fma(F[i][A], F[i][A], I1);
    const double a = mu * pow(k.J, -2.0 / 3.0);
    const double b = 0.5 * kappa * (k.J * k.J - 1.0);
    double P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) {
            const double G = k.Finv[A][i];
            P[i][A] = (a * (F[i][A] - I1 / 3.0 * G) + b * G) * JxW;
        }
    matmul3_bt(P, Jginv, Q);
}

// tau = P F^T = a (b - I1/3 I) + b_vol I of the split law, Voigt, times s
MFE_HD void kirchhoff_split_voigt(const double F[3][3], const Kin& k, double mu, double kappa, double s,
                                  double tau[6]) {
    double bb[3][3];
    matmul3_bt(F, F, bb);
    const double I1 = bb[0][0] + bb[1][1] + bb[2][2];
    const double a = mu * pow(k.J, -2.0 / 3.0);
    const double bv = 0.5 * kappa * (k.J * k.J - 1.0);
    tau[0] = s * (a * (bb[0][0] - I1 / 3.0) + bv);
    tau[1] = s * (a * (bb[1][1] - I1 / 3.0) + bv);
    tau[2] = s * (a * (bb[2][2] - I1 / 3.0) + bv);
    tau[3] = s * a * bb[1][2];
    tau[4] = s * a * bb[0][2];
    tau[5] = s * a * bb[0][1];
}

// Voigt matrix of J c * s for the split law from nine dual-number directional
// derivatives of P: L_iAkB = dP_iA/dF_kB, J c_ijkl = F_jA F_lB L_iAkB - d_ik tau_jl,
// symmetrised over the minor index pairs and the Voigt transpose.
MFE_HD void spatial_tangent_split_voigt(const double F[3][3], double mu, double kappa, double s, double D21[21]) {
    double L[3][3][3][3];  // L[i][A][k][B]
    double P[3][3];
    for (int k = 0; k < 3; ++k)
        for (int B = 0; B < 3; ++B) {
            Dual Fd[3][3], Pd[3][3];
            for (int i = 0; i < 3; ++i)
                for (int A = 0; A < 3; ++A) Fd[i][A] = Dual{F[i][A], (i == k && A == B) ? 1.0 : 0.0};
            piola_split_dual(Fd, mu, kappa, Pd);
            for (int i = 0; i < 3; ++i)
                for (int A = 0; A < 3; ++A) {
                    L[i][A][k][B] = Pd[i][A].d;
                    P[i][A] = Pd[i][A].v;
                }
        }
    double T[3][3];  // tau = P F^T
    matmul3_bt(P, F, T);
    auto jc = [&](int i, int j, int k, int l) {
        double v = 0.0;
        for (int A = 0; A < 3; ++A)
            for (int B = 0; B < 3; ++B) v = fma(F[j][A] * F[l][B], L[i][A][k][B], v);
        return v - (i == k ? T[j][l] : 0.0);
    };
    const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
    double D[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            const int i = vi[r], j = vj[r], k = vi[c], l = vj[c];
            D[r][c] = 0.25 * (jc(i, j, k, l) + jc(j, i, k, l) + jc(i, j, l, k) + jc(j, i, l, k));
        }
    for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) D21[voigt_packed(r, c)] = 0.5 * (D[r][c] + D[c][r]) * s;
}

// stored energy density of the two laws
MFE_HD double energy_nh(const double F[3][3], const Kin& k, double mu, double lam) {
    double trC = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) trC = fma(F[i][j], F[i][j], trC);
    return 0.5 * mu * (trC - 3.0 - 2.0 * k.lJ) + lam * k.lJ * k.lJ;
}

MFE_HD double energy_split(const double F[3][3], const Kin& k, double mu, double kappa) {
    double I1 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) I1 = fma(F[i][j], F[i][j], I1);
    return 0.5 * mu * (pow(k.J, -2.0 / 3.0) * I1 - 3.0) + 0.5 * kappa * (0.5 * (k.J * k.J - 1.0) - k.lJ);
}

// --------------------------------------------------------------------------
// Residual integrand: Q = JxW P Jginv^T with P = mu F + (2 lam log J - mu) F^-T.
// --------------------------------------------------------------------------
MFE_HD void pointwise_piola(const double F[3][3], const Kin& k, double mu, double lam,
                            const double Jginv[3][3], double JxW, double Q[3][3]) {
    double P[3][3];
    const double a = mu * JxW;
    const double b = (2.0 * lam * k.lJ - mu) * JxW;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int A = 0; A < 3; ++A) P[i][A] = fma(a, F[i][A], b * k.Finv[A][i]);
    matmul3_bt(P, Jginv, Q);
}

// --------------------------------------------------------------------------
// Current-configuration data (Sec. 2.1 eqs. F:cur, DF:cur, Jc; Alg. 2).
//   M = Jginv F^-1 maps reference-cell gradients to spatial gradients:
//   grad w = dw M.  tau = P F^T = mu (F F^T - I) + 2 lam log J I.
//   J c = 2 lam I(x)I + 2 (mu - 2 lam log J) I^s.
// The tangent action tested with phi is  grad phi : (J c : sym h + h tau)
// with h = grad w, integrated over the reference cell (weights JxW).
// --------------------------------------------------------------------------
MFE_HD void spatial_map(const double Jginv[3][3], const Kin& k, double M[3][3]) {
    matmul3(Jginv, k.Finv, M);
}

MFE_HD void kirchhoff_voigt(const double F[3][3], const Kin& k, double mu, double lam, double s,
                            double tau[6]) {
    // tau_ij = mu ((F F^T)_ij - d_ij) + 2 lam log J d_ij, times s
    double b[3][3];
    matmul3_bt(F, F, b);
    const double iso = 2.0 * lam * k.lJ - mu;
    tau[0] = s * fma(mu, b[0][0], iso);
    tau[1] = s * fma(mu, b[1][1], iso);
    tau[2] = s * fma(mu, b[2][2], iso);
    tau[3] = s * mu * b[1][2];
    tau[4] = s * mu * b[0][2];
    tau[5] = s * mu * b[0][1];
}

template <typename R>
MFE_HD void tau_full(const R t[6], R T[3][3]) {
    T[0][0] = t[0]; T[1][1] = t[1]; T[2][2] = t[2];
    T[1][2] = T[2][1] = t[3];
    T[0][2] = T[2][0] = t[4];
    T[0][1] = T[1][0] = t[5];
}

// T2 point-wise product: h = dw M, g = c1 tr(h) I + c2 sym(h) + h tau, Q = g M^T
template <typename R>
MFE_HD void pointwise_t2(const R dw[3][3], const R M[3][3], const R tau6[6], R c1, R c2, R Q[3][3]) {
    R h[3][3], T[3][3], g[3][3];
    matmul3(dw, M, h);
    tau_full(tau6, T);
    matmul3(h, T, g);
    const R tr = c1 * (h[0][0] + h[1][1] + h[2][2]);
    const R hc = R(0.5) * c2;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) g[i][j] = fmar(hc, h[i][j] + h[j][i], g[i][j]);
    g[0][0] += tr;
    g[1][1] += tr;
    g[2][2] += tr;
    matmul3_bt(g, M, Q);
}

// T4 point-wise product with the general symmetric 6x6 (Voigt) tangent:
// s = D eps(h) (engineering shears), g = s + h tau, Q = g M^T.
template <typename R>
MFE_HD void pointwise_t4(const R dw[3][3], const R M[3][3], const R D21[21], const R tau6[6], R Q[3][3]) {
    R h[3][3], T[3][3], g[3][3];
    matmul3(dw, M, h);
    const R e[6] = {h[0][0], h[1][1], h[2][2], h[1][2] + h[2][1], h[0][2] + h[2][0], h[0][1] + h[1][0]};
    R s[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        R acc = 0;
#pragma unroll
        for (int c = 0; c < 6; ++c)
            acc = fmar(D21[r <= c ? voigt_packed(r, c) : voigt_packed(c, r)], e[c], acc);
        s[r] = acc;
    }
    tau_full(tau6, T);
    matmul3(h, T, g);
    g[0][0] += s[0];
    g[1][1] += s[1];
    g[2][2] += s[2];
    g[1][2] += s[3];
    g[2][1] += s[3];
    g[0][2] += s[4];
    g[2][0] += s[4];
    g[0][1] += s[5];
    g[1][0] += s[5];
    matmul3_bt(g, M, Q);
}

// Voigt matrix of J c * s for the neo-Hookean law of eq. hypref.
MFE_HD void spatial_tangent_voigt(const Kin& k, double mu, double lam, double s, double D21[21]) {
#pragma unroll
    for (int i = 0; i < 21; ++i) D21[i] = 0.0;
    const double g = (mu - 2.0 * lam * k.lJ) * s;
    const double l2 = 2.0 * lam * s;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = r; c < 3; ++c) D21[voigt_packed(r, c)] = l2 + (r == c ? 2.0 * g : 0.0);
    D21[voigt_packed(3, 3)] = g;
    D21[voigt_packed(4, 4)] = g;
    D21[voigt_packed(5, 5)] = g;
}

}  // namespace mfe
