// Host-side reference element of the periodic piezoelectric cell problem.
//
// Trilinear hexahedron of side h, local node l = a + 2b + 4c at (a, b, c) h,
// element dof 4l + f with f = (u_x, u_y, u_z, phi).  With the generalised
// strain g = (eps_xx, eps_yy, eps_zz, gamma_yz, gamma_xz, gamma_xy, E_x, E_y,
// E_z), E = -grad phi (Sec. 2.2 constitutive laws), and the symmetric
// generalised material matrix M = [[C, -e^T], [-e, -kappa]], the element
// matrices of the weak form are
//     K0 = sum_q w_q Bq^T M Bq   (32 x 32),   F0 = sum_q w_q Bq^T M   (32 x 9)
// over the exact 2x2x2 Gauss rule.  An ersatz element with scale s has
// matrices s K0 and s F0.  Block split (Sec. 2.5):  A0 = K0[u,u] (24 x 24),
// B0 = K0[phi,u] (8 x 24), -C0 = K0[phi,phi]; the element Schur block of
// Sec. 2.5.3 is S0 = C0 + B0 (A0 + delta I)^-1 B0^T with delta = 1e-10.
#pragma once
#include <array>
#include <cmath>
#include <vector>

#include "piezohom.h"

namespace phz {

// Units: stress scale 1e9 Pa, charge scale 1 C/m^2, permittivity 1e-9 F/m.
constexpr double kStress = 1.0e9;
constexpr double kCharge = 1.0;
constexpr double kPerm = kCharge * kCharge / kStress;

struct RefElement {
  double h = 1.0;
  double M[81];          // non-dimensional generalised material matrix
  double K0[32 * 32];    // dof 4l+f ordering
  double F0[32 * 9];
  double A0[24 * 24];    // (3l+f, 3l'+f')
  double B0[8 * 24];     // (l, 3l'+f')
  double S0[8 * 8];      // (l, l')
  double C0[8 * 8];      // (l, l'): the dielectric block; the operator's (phi, phi) block is -C0
  double Kfull[32 * 32]; // same as K0 (4l+f, 4l'+f'), kept for clarity
  // the quadrature terms of K0 and F0 per Gauss point q = i + 2j + 4k (points
  // (g_i, g_j, g_k)): an element whose material is s_q M at point q has
  // matrices sum_q s_q K0q[q] and sum_q s_q F0q[q]
  double K0q[8][32 * 32];
  double F0q[8][32 * 9];
};

inline void build_material_matrix(const phz_material& m, double* M) {
  for (int i = 0; i < 81; ++i) M[i] = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) M[i * 9 + j] = m.C[i * 6 + j] / kStress;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 6; ++j) {
      double v = -m.e[i * 6 + j] / kCharge;
      M[(6 + i) * 9 + j] = v;      // -e
      M[j * 9 + 6 + i] = v;        // -e^T
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[(6 + i) * 9 + 6 + j] = -m.kappa[i * 3 + j] / kPerm;
}

// 9 x 32 strain-displacement matrix at reference point xi in [0,1]^3.
inline void bmat_at(const double xi[3], double h, double* B) {
  for (int i = 0; i < 9 * 32; ++i) B[i] = 0.0;
  for (int l = 0; l < 8; ++l) {
    int a = l & 1, b = (l >> 1) & 1, c = (l >> 2) & 1;
    double fx = a ? xi[0] : 1.0 - xi[0], dfx = a ? 1.0 : -1.0;
    double fy = b ? xi[1] : 1.0 - xi[1], dfy = b ? 1.0 : -1.0;
    double fz = c ? xi[2] : 1.0 - xi[2], dfz = c ? 1.0 : -1.0;
    double gx = dfx * fy * fz / h, gy = fx * dfy * fz / h, gz = fx * fy * dfz / h;
    int col = 4 * l;
    B[0 * 32 + col + 0] = gx;
    B[1 * 32 + col + 1] = gy;
    B[2 * 32 + col + 2] = gz;
    B[3 * 32 + col + 1] = gz;  B[3 * 32 + col + 2] = gy;   // gamma_yz
    B[4 * 32 + col + 0] = gz;  B[4 * 32 + col + 2] = gx;   // gamma_xz
    B[5 * 32 + col + 0] = gy;  B[5 * 32 + col + 1] = gx;   // gamma_xy
    B[6 * 32 + col + 3] = -gx;                             // E = -grad phi
    B[7 * 32 + col + 3] = -gy;
    B[8 * 32 + col + 3] = -gz;
  }
}

// Solve (A + delta I) Z = R for SPD-plus-shift A (n x n) in long double.
inline void shifted_cholesky_solve(int n, const double* A, double delta, int nrhs,
                                   const double* R, double* Z) {
  std::vector<long double> L(n * n, 0.0L);
  for (int j = 0; j < n; ++j) {
    long double d = (long double)A[j * n + j] + delta;
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    d = sqrtl(d);
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      long double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / d;
    }
  }
  std::vector<long double> y(n);
  for (int r = 0; r < nrhs; ++r) {
    for (int i = 0; i < n; ++i) {
      long double v = R[i * nrhs + r];
      for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
      y[i] = v / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      long double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * y[k];
      y[i] = v / L[i * n + i];
    }
    for (int i = 0; i < n; ++i) Z[i * nrhs + r] = (double)y[i];
  }
}

inline RefElement build_ref_element(const phz_material& mat, double h, double delta = 1e-10) {
  RefElement R;
  R.h = h;
  build_material_matrix(mat, R.M);
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const double w = h * h * h / 8.0;
  for (int i = 0; i < 32 * 32; ++i) R.K0[i] = 0.0;
  for (int i = 0; i < 32 * 9; ++i) R.F0[i] = 0.0;
  for (int q = 0; q < 8; ++q) {
    for (int i = 0; i < 32 * 32; ++i) R.K0q[q][i] = 0.0;
    for (int i = 0; i < 32 * 9; ++i) R.F0q[q][i] = 0.0;
  }
  double B[9 * 32], MB[9 * 32];
  for (int q = 0; q < 8; ++q) {
    double xi[3] = {gp[q & 1], gp[(q >> 1) & 1], gp[(q >> 2) & 1]};
    bmat_at(xi, h, B);
    for (int a = 0; a < 9; ++a)
      for (int j = 0; j < 32; ++j) {
        double v = 0.0;
        for (int b = 0; b < 9; ++b) v += R.M[a * 9 + b] * B[b * 32 + j];
        MB[a * 32 + j] = v;
      }
    for (int i = 0; i < 32; ++i) {
      for (int j = 0; j < 32; ++j) {
        double v = 0.0;
        for (int a = 0; a < 9; ++a) v += B[a * 32 + i] * MB[a * 32 + j];
        R.K0[i * 32 + j] += w * v;
        R.K0q[q][i * 32 + j] = w * v;
      }
      for (int L = 0; L < 9; ++L) {
        double v = 0.0;
        for (int a = 0; a < 9; ++a) v += B[a * 32 + i] * R.M[a * 9 + L];
        R.F0[i * 9 + L] += w * v;
        R.F0q[q][i * 9 + L] = w * v;
      }
    }
  }
  // exact symmetry (the quadrature sum is symmetric up to rounding)
  for (int i = 0; i < 32; ++i)
    for (int j = i + 1; j < 32; ++j) {
      double v = 0.5 * (R.K0[i * 32 + j] + R.K0[j * 32 + i]);
      R.K0[i * 32 + j] = R.K0[j * 32 + i] = v;
      for (int q = 0; q < 8; ++q) {
        double vq = 0.5 * (R.K0q[q][i * 32 + j] + R.K0q[q][j * 32 + i]);
        R.K0q[q][i * 32 + j] = R.K0q[q][j * 32 + i] = vq;
      }
    }
  for (int i = 0; i < 32 * 32; ++i) R.Kfull[i] = R.K0[i];
  for (int l = 0; l < 8; ++l)
    for (int f = 0; f < 3; ++f)
      for (int lp = 0; lp < 8; ++lp)
        for (int fp = 0; fp < 3; ++fp)
          R.A0[(3 * l + f) * 24 + 3 * lp + fp] = R.K0[(4 * l + f) * 32 + 4 * lp + fp];
  for (int l = 0; l < 8; ++l)
    for (int lp = 0; lp < 8; ++lp)
      for (int fp = 0; fp < 3; ++fp)
        R.B0[l * 24 + 3 * lp + fp] = R.K0[(4 * l + 3) * 32 + 4 * lp + fp];
  for (int l = 0; l < 8; ++l)
    for (int lp = 0; lp < 8; ++lp) R.C0[l * 8 + lp] = -R.K0[(4 * l + 3) * 32 + 4 * lp + 3];
  // S0 = C0 + B0 (A0 + delta I)^-1 B0^T
  double Bt[24 * 8], Z[24 * 8];
  for (int i = 0; i < 24; ++i)
    for (int l = 0; l < 8; ++l) Bt[i * 8 + l] = R.B0[l * 24 + i];
  shifted_cholesky_solve(24, R.A0, delta, 8, Bt, Z);
  for (int l = 0; l < 8; ++l)
    for (int lp = 0; lp < 8; ++lp) {
      double v = -R.K0[(4 * l + 3) * 32 + 4 * lp + 3];
      for (int i = 0; i < 24; ++i) v += R.B0[l * 24 + i] * Z[i * 8 + lp];
      R.S0[l * 8 + lp] = v;
    }
  for (int l = 0; l < 8; ++l)
    for (int lp = l + 1; lp < 8; ++lp) {
      double v = 0.5 * (R.S0[l * 8 + lp] + R.S0[lp * 8 + l]);
      R.S0[l * 8 + lp] = R.S0[lp * 8 + l] = v;
    }
  return R;
}

// Dense symmetric positive definite inverse (Cholesky, in place), n x n.
// Returns false if a pivot is not positive.
inline bool spd_inverse(int n, std::vector<double>& A) {
  std::vector<long double> L(size_t(n) * n, 0.0L);
  for (int j = 0; j < n; ++j) {
    long double d = A[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) d -= L[size_t(j) * n + k] * L[size_t(j) * n + k];
    if (!(d > 0)) return false;
    d = sqrtl(d);
    L[size_t(j) * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      long double v = A[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) v -= L[size_t(i) * n + k] * L[size_t(j) * n + k];
      L[size_t(i) * n + j] = v / d;
    }
  }
  // inverse of L (lower), then A^-1 = L^-T L^-1
  std::vector<long double> Li(size_t(n) * n, 0.0L);
  for (int j = 0; j < n; ++j) {
    Li[size_t(j) * n + j] = 1.0L / L[size_t(j) * n + j];
    for (int i = j + 1; i < n; ++i) {
      long double v = 0.0L;
      for (int k = j; k < i; ++k) v -= L[size_t(i) * n + k] * Li[size_t(k) * n + j];
      Li[size_t(i) * n + j] = v / L[size_t(i) * n + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      long double v = 0.0L;
      for (int k = i; k < n; ++k) v += Li[size_t(k) * n + i] * Li[size_t(k) * n + j];
      A[size_t(i) * n + j] = A[size_t(j) * n + i] = (double)v;
    }
  return true;
}

}  // namespace phz
