// Compile-time constants of the reconstruction, per order.
//
// The target cell is mapped onto the reference triangle (0,0),(1,0),(0,1)
// (Sec. 2.2 eq. 02), so the smoothness form and the face-point basis values
// are the same for every cell of a given order; only the least-squares
// operators differ per cell.  Both tables are exact rational expressions
// evaluated here at compile time.
#pragma once

#include "internal.h"

namespace teno {

constexpr double cx_fact(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

// a! / (a-k)!
constexpr double cx_falling(int a, int k) {
  double f = 1.0;
  for (int t = 0; t < k; ++t) f *= (a - t);
  return f;
}

constexpr double cx_sqrt(double x) {
  double y = x > 1.0 ? x : 1.0;
  for (int it = 0; it < 100; ++it) y = 0.5 * (y + x / y);
  return y;
}

// Monomials xi^a eta^b with 1 <= a+b <= r in graded order
// (xi, eta, xi^2, xi eta, eta^2, xi^3, ...).
struct Exps {
  int a[20] = {};
  int b[20] = {};
  int n = 0;
};

constexpr Exps cx_exps(int r) {
  Exps e{};
  for (int d = 1; d <= r; ++d)
    for (int a = d; a >= 0; --a) {
      e.a[e.n] = a;
      e.b[e.n] = d - a;
      e.n++;
    }
  return e;
}

// int over the reference triangle of xi^a eta^b = a! b! / (a+b+2)!
constexpr double cx_moment(int a, int b) { return cx_fact(a) * cx_fact(b) / cx_fact(a + b + 2); }

template <int R>
struct SmoothForm {
  static constexpr int N = (R + 1) * (R + 2) / 2 - 1;
  struct Mat {
    double v[N][N] = {};
  };
  // B_lm = sum over multi-indices 1 <= |alpha| <= R (each once) of
  //        int_{T_ref} D^alpha phi_l D^alpha phi_m   (Sec. 2.3)
  static constexpr Mat make() {
    Mat M{};
    const Exps e = cx_exps(R);
    for (int l = 0; l < N; ++l)
      for (int m = 0; m < N; ++m) {
        double s = 0.0;
        for (int d = 1; d <= R; ++d)
          for (int ax = d; ax >= 0; --ax) {
            const int ay = d - ax;
            if (e.a[l] < ax || e.b[l] < ay || e.a[m] < ax || e.b[m] < ay) continue;
            const double cl = cx_falling(e.a[l], ax) * cx_falling(e.b[l], ay);
            const double cm = cx_falling(e.a[m], ax) * cx_falling(e.b[m], ay);
            s += cl * cm * cx_moment(e.a[l] + e.a[m] - 2 * ax, e.b[l] + e.b[m] - 2 * ay);
          }
        M.v[l][m] = s;
      }
    return M;
  }
  static constexpr Mat B = make();
  // upper triangle of B with the off-diagonal entries doubled:
  // a^T B a = sum_l a_l (U_ll a_l + sum_{m>l} U_lm a_m)
  static constexpr Mat upper() {
    Mat M{};
    for (int l = 0; l < N; ++l)
      for (int m = l; m < N; ++m) M.v[l][m] = (m == l ? 1.0 : 2.0) * B.v[l][m];
    return M;
  }
  static constexpr Mat U = upper();
  // B = L D L^T with L unit lower triangular (B is positive definite: the
  // derivatives up to order R vanish together only for a constant, and the
  // basis has zero mean).  Row l of Lt holds column l of L (Lt[l][m] = L_ml,
  // m >= l) and d holds D, so that a^T B a = sum_l d_l (sum_{m>=l} Lt_lm a_m)^2.
  struct Ldl {
    double Lt[N][N] = {};
    double d[N] = {};
  };
  static constexpr Ldl factor() {
    Ldl f{};
    for (int j = 0; j < N; ++j) {
      double dj = B.v[j][j];
      for (int k = 0; k < j; ++k) dj -= f.Lt[k][j] * f.Lt[k][j] * f.d[k];
      f.d[j] = dj;
      f.Lt[j][j] = 1.0;
      for (int i = j + 1; i < N; ++i) {
        double s = B.v[i][j];
        for (int k = 0; k < j; ++k) s -= f.Lt[k][i] * f.Lt[k][j] * f.d[k];
        f.Lt[j][i] = s / dj;
      }
    }
    return f;
  }
  static constexpr Ldl LDL = factor();
};

// Gauss-Legendre points on [0,1] (t) and weights summing to one (w).
template <int NQ>
struct FaceRule;

template <>
struct FaceRule<2> {
  static constexpr double t[2] = {0.5 - 0.5 / cx_sqrt(3.0), 0.5 + 0.5 / cx_sqrt(3.0)};
  static constexpr double w[2] = {0.5, 0.5};
};

template <>
struct FaceRule<3> {
  static constexpr double t[3] = {0.5 - 0.5 * cx_sqrt(0.6), 0.5, 0.5 + 0.5 * cx_sqrt(0.6)};
  static constexpr double w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
};

// psi_l at the face points: q = e*NQ + kappa, local edge e from vertex e to
// vertex e+1: e0 -> (t, 0), e1 -> (1-t, t), e2 -> (0, 1-t).
template <int R, int NQ>
struct FaceBasis {
  static constexpr int N = (R + 1) * (R + 2) / 2 - 1;
  struct Tab {
    double v[3 * NQ][N] = {};
  };
  static constexpr Tab make() {
    Tab T{};
    const Exps e = cx_exps(R);
    for (int ed = 0; ed < 3; ++ed)
      for (int k = 0; k < NQ; ++k) {
        const double t = FaceRule<NQ>::t[k];
        const double xi = ed == 0 ? t : (ed == 1 ? 1.0 - t : 0.0);
        const double eta = ed == 0 ? 0.0 : (ed == 1 ? t : 1.0 - t);
        for (int l = 0; l < N; ++l) {
          double p = 1.0;
          for (int i = 0; i < e.a[l]; ++i) p *= xi;
          for (int i = 0; i < e.b[l]; ++i) p *= eta;
          T.v[ed * NQ + k][l] = p - 2.0 * cx_moment(e.a[l], e.b[l]);
        }
      }
    return T;
  }
  static constexpr Tab P = make();
};

// Per-order sizes (match Dims in internal.h).
template <int P>
struct OrderT {
  static constexpr int R = P - 1;
  static constexpr int NU = (R + 1) * (R + 2) / 2 - 1;
  static constexpr int NL = (R + 1) * (R + 2) - 1;
  static constexpr int NQ = (P + 1) / 2;
  static constexpr int ROWS = 33 + NL;
  static constexpr int ROWS4 = (ROWS + 3) / 4;
  static constexpr int J = 165 + NU * NL;         // operator entries
  // stored entries per cell of a dense mesh (D) or of one on entry pairs
  template <bool D>
  static constexpr int JPD = 3 * small_block(D) + large_block(NL, NU, D);
};

}  // namespace teno
