// TEST INFRASTRUCTURE ONLY.  Plain FP64 CPU oracle of the unstructured-mesh
// finite-volume TENO residual on TETRAHEDRA: the three-dimensional form of
// the method (Ji, Liang & Fu, "A class of new high-order finite-volume TENO
// schemes for hyperbolic conservation laws with unstructured meshes"; Sec.
// 2-4 are written in (xi, eta, zeta), Sec. 5.9 runs the scheme on a
// tetrahedral mesh).  Only the tests and the smoke check load this library.
// It shares no code with the HIP path.
//
// User cell order, host pointers.  U[cell][5] = (rho, rho u, rho v, rho w, E).
//
// Steps, each following the passage cited beside it:
//   geometry and faces ................. Sec. 2.1, semi-discrete equation
//   stencils (central + 4 directional) . Sec. 3.1 (rules are a reading, below)
//   reference map, zero-mean basis,
//   constrained least squares, QR ...... Sec. 2.2, reconstruction eqs. 02-10
//                                        (N_k of eq. 03 with n_d = 3)
//   smoothness indicators .............. Sec. 2.3, WENO smoothness equation
//   scale separation, cutoff, selection  Sec. 3.2-3.3 (K = 4 small stencils)
//   face quadrature points ............. Sec. 2.1
//   rotation + HLL + Einfeldt speeds ... Sec. 4.1-4.2 (3D rotation frame)
//   residual, SSP-RK3 .................. Sec. 2.1, time-discretisation equation
//
// Readings where the paper is silent (the 2D readings carried to 3D):
//   * vertices v0..v3 positively oriented (v2, v3 swapped otherwise); local
//     face e is the face opposite vertex e, with vertices
//     (1,2,3), (0,3,2), (0,1,3), (0,2,1) so that its normal points out.
//   * reference map x = v0 + xi (v1-v0) + eta (v2-v0) + zeta (v3-v0).
//   * stencils: central = I0 + nearest 2 N_k - 1 cells by periodic
//     min-image centroid distance; directional e = I0 + nearest 19 cells
//     whose centroid lies in the closed cone from the target centroid
//     through the three vertices of local face e; ties by lower user id; a
//     cone left short by a wall is completed with the nearest cells outside.
//   * N_k counts the constant; N_s = 2 N_k cells including I0.
//   * beta sums every derivative multi-index once, in reference coordinates.
//   * face rule: symmetric triangle rules, 6 points of degree 4 (orders 3-4)
//     or Radon's 7 points of degree 5 (orders 5-6), in the barycentric
//     coordinates of the face's vertices in the cell's local order; the
//     neighbour evaluates the same physical points in its own order.
//   * HLL: Sec. 4 in the frame (n, t1, t2), t1 from n and the coordinate
//     axis least aligned with it; Roe sound speed from all three Roe
//     velocity components.
//   * dt = CFL * min_i |V_i| / sum_f |A_if| (|u_i . n_if| + c_i).
//   * flag bits (uint32): 5v+4 = large stencil kept (step i); 5v+k = small
//     stencil k kept in step ii.
//   * boundary faces (open axes): transmissive (the inner state) or
//     reflective (normal momentum reversed).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {
typedef struct oracle3_params {
  int32_t order;    // 3..6
  int32_t variant;  // 0 = TENO, 1 = LINEAR (large stencil everywhere)
  int32_t power;    // scale-separation exponent (paper: 6)
  int32_t fallback; // 1: a cell with a non-physical face point uses its average
  double ct;        // cutoff C_T (paper: 1e-6)
  double eps;       // epsilon in gamma_k (paper: 1e-12)
  double gamma;     // ratio of specific heats
  double tie_rel;   // near-tie band |chi/C_T - 1| <= tie_rel
} oracle3_params;

typedef struct oracle3_diag {
  int64_t nonphysical;
  int64_t first_bad_cell;
  int64_t near_ties;
  int64_t large_kept;
  int64_t fallbacks;
} oracle3_diag;
}

namespace {

thread_local std::string g_err;
int fail(const std::string& msg) {
  g_err = msg;
  return -1;
}

constexpr int NV = 5;  // conservative variables
constexpr int KS = 4;  // small directional stencils (one per face)
// local face e: vertices in the order that makes (b-a) x (c-a) point out
const int FV[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

double ipow(double x, int k) {
  double v = 1.0;
  for (int i = 0; i < k; ++i) v *= x;
  return v;
}

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [0, 1] (Newton iteration on P_n)
// ---------------------------------------------------------------------------
void gauss01(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double p0 = 1.0, p1 = x, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      p0 = 1.0;
      p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) <= 1e-15) break;
    }
    p0 = 1.0;
    p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    t[i] = 0.5 * (1.0 - x);
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
}

// Collapsed (Duffy) product rule on the reference tetrahedron
// {xi, eta, zeta >= 0, xi + eta + zeta <= 1}: xi = u (1-v)(1-w),
// eta = v (1-w), zeta = w, dV = (1-v)(1-w)^2 du dv dw; weights sum to 1/6.
struct TetRule {
  std::vector<double> xi, eta, zeta, w;
};

TetRule tet_rule(int n) {
  std::vector<double> t, wt;
  gauss01(n, t, wt);
  TetRule r;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c) {
        double u = t[a], v = t[b], w = t[c];
        r.xi.push_back(u * (1.0 - v) * (1.0 - w));
        r.eta.push_back(v * (1.0 - w));
        r.zeta.push_back(w);
        r.w.push_back(wt[a] * wt[b] * wt[c] * (1.0 - v) * (1.0 - w) * (1.0 - w));
      }
  return r;
}

// ---------------------------------------------------------------------------
// Basis (Sec. 2.2 eqs. 04-06): graded monomials xi^a eta^b zeta^c,
// 1 <= a+b+c <= r, each minus its mean over the reference tetrahedron.
// ---------------------------------------------------------------------------
struct Basis {
  int r = 0;
  std::vector<int> ea, eb, ec;
  std::vector<double> mean;
  int n() const { return (int)ea.size(); }
};

Basis make_basis(int r) {
  Basis b;
  b.r = r;
  for (int d = 1; d <= r; ++d)
    for (int a = d; a >= 0; --a)
      for (int bb = d - a; bb >= 0; --bb) {
        b.ea.push_back(a);
        b.eb.push_back(bb);
        b.ec.push_back(d - a - bb);
      }
  TetRule q = tet_rule(r / 2 + 3);
  for (int l = 0; l < b.n(); ++l) {
    double acc = 0.0;
    for (size_t k = 0; k < q.w.size(); ++k)
      acc += q.w[k] * ipow(q.xi[k], b.ea[l]) * ipow(q.eta[k], b.eb[l]) * ipow(q.zeta[k], b.ec[l]);
    b.mean.push_back(acc * 6.0);  // the reference tetrahedron has volume 1/6
  }
  return b;
}

double psi(const Basis& b, int l, double xi, double eta, double zeta) {
  return ipow(xi, b.ea[l]) * ipow(eta, b.eb[l]) * ipow(zeta, b.ec[l]) - b.mean[l];
}

// ---------------------------------------------------------------------------
// Householder QR (column-major m x n, m >= n), Sec. 2.2 eq. 10
// ---------------------------------------------------------------------------
struct QR {
  int m = 0, n = 0;
  std::vector<double> a, beta;
  double rmax = 0.0, rmin = 0.0;
};

bool qr_factor(QR& q) {
  const int m = q.m, n = q.n;
  q.beta.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double* col = &q.a[(size_t)j * m];
    double sigma = 0.0;
    for (int i = j + 1; i < m; ++i) sigma += col[i] * col[i];
    double x0 = col[j];
    double mu = std::sqrt(x0 * x0 + sigma);
    if (mu == 0.0) return false;
    double alpha = (x0 >= 0.0) ? -mu : mu;
    double v0 = x0 - alpha;
    for (int i = j + 1; i < m; ++i) col[i] /= v0;
    double vtv = 1.0;
    for (int i = j + 1; i < m; ++i) vtv += col[i] * col[i];
    double bta = 2.0 / vtv;
    q.beta[j] = bta;
    col[j] = alpha;
    for (int c = j + 1; c < n; ++c) {
      double* cc = &q.a[(size_t)c * m];
      double s = cc[j];
      for (int i = j + 1; i < m; ++i) s += col[i] * cc[i];
      s *= bta;
      cc[j] -= s;
      for (int i = j + 1; i < m; ++i) cc[i] -= s * col[i];
    }
  }
  q.rmax = 0.0;
  q.rmin = INFINITY;
  for (int j = 0; j < n; ++j) {
    double d = std::fabs(q.a[(size_t)j * m + j]);
    q.rmax = std::max(q.rmax, d);
    q.rmin = std::min(q.rmin, d);
  }
  return q.rmin > 1e-13 * q.rmax;
}

// least-squares solution of A x = b from the factors
void qr_solve(const QR& q, const double* b, double* x) {
  const int m = q.m, n = q.n;
  std::vector<double> y(b, b + m);
  for (int j = 0; j < n; ++j) {
    const double* col = &q.a[(size_t)j * m];
    double s = y[j];
    for (int i = j + 1; i < m; ++i) s += col[i] * y[i];
    s *= q.beta[j];
    y[j] -= s;
    for (int i = j + 1; i < m; ++i) y[i] -= s * col[i];
  }
  for (int j = n - 1; j >= 0; --j) {
    double s = y[j];
    for (int c = j + 1; c < n; ++c) s -= q.a[(size_t)c * m + j] * x[c];
    x[j] = s / q.a[(size_t)j * m + j];
  }
}

// ---------------------------------------------------------------------------
// Symmetric triangle rules for the face quadrature (reading above), in
// barycentric coordinates; weights sum to 1.
// ---------------------------------------------------------------------------
struct FaceRule {
  std::vector<double> l0, l1, l2, w;
};

FaceRule face_rule(int order) {
  FaceRule r;
  auto orbit3 = [&](double a, double w) {  // (1-2a, a, a) and its rotations
    double b = 1.0 - 2.0 * a;
    double p[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
    for (int k = 0; k < 3; ++k) {
      r.l0.push_back(p[k][0]);
      r.l1.push_back(p[k][1]);
      r.l2.push_back(p[k][2]);
      r.w.push_back(w);
    }
  };
  if (order <= 4) {
    // degree 4, six points (Dunavant, 1985)
    orbit3(0.445948490915965, 0.223381589678011);
    orbit3(0.091576213509771, 0.109951743655322);
  } else {
    // degree 5, seven points (Radon, 1948)
    const double s = std::sqrt(15.0);
    r.l0.push_back(1.0 / 3.0);
    r.l1.push_back(1.0 / 3.0);
    r.l2.push_back(1.0 / 3.0);
    r.w.push_back(9.0 / 40.0);
    orbit3((6.0 - s) / 21.0, (155.0 - s) / 1200.0);
    orbit3((6.0 + s) / 21.0, (155.0 + s) / 1200.0);
  }
  return r;
}

// reference coordinates of barycentric point (l0, l1, l2) on local face e
void face_ref_point(int e, double l0, double l1, double l2, double ref[3]) {
  static const double V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const double l[3] = {l0, l1, l2};
  for (int d = 0; d < 3; ++d) {
    ref[d] = 0.0;
    for (int j = 0; j < 3; ++j) ref[d] += l[j] * V[FV[e][j]][d];
  }
}

// ---------------------------------------------------------------------------
// Mesh
// ---------------------------------------------------------------------------
struct Stencil {
  std::vector<int> cells;
  std::vector<double> vol;  // |V'_s| in the target's reference space
  QR qr;
};

struct CellData {
  bool built = false;
  Stencil st[KS + 1];  // 0..3 directional (local faces), 4 = central (large)
};

struct Mesh {
  int nv = 0, nc = 0, nf = 0;
  bool periodic = false;  // all three axes periodic
  double P[3] = {0, 0, 0};
  std::vector<double> xyz;
  std::vector<int> tet;              // [nc][4] positively oriented
  std::vector<double> X;             // [nc][4][3] unwrapped about v0
  std::vector<double> vol, cen;      // cen [nc][3]
  std::vector<int> fL, fR, fLe, fRe; // face -> cells and local faces
  std::vector<double> fn, farea;     // unit normal out of L [nf][3], area
  std::vector<int> cf;               // [nc][4] face of each local face
  std::vector<int> pair;             // [nf][npt]: R's point of L's point k
  std::vector<int> bface, bidx, bkind;
  bool have_params = false;
  oracle3_params prm{};
  Basis big, small;
  FaceRule rule;
  std::vector<CellData> cd;
  int nb = 0;
  double bw[3] = {0, 0, 0};
  std::vector<int> bin_start, bin_cells;
};

void min_image(const Mesh& m, double d[3], double* shift = nullptr) {
  for (int a = 0; a < 3; ++a) {
    double k = 0.0;
    if (m.P[a] > 0.0) {
      k = std::nearbyint(d[a] / m.P[a]);
      d[a] -= m.P[a] * k;
    }
    if (shift) shift[a] = -m.P[a] * k;
  }
}

double det3(const double a[3], const double b[3], const double c[3]) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------------------
// Stencils (Sec. 3.1; rule in the header)
// ---------------------------------------------------------------------------
struct Cand {
  double d2;
  int id;
  bool operator<(const Cand& o) const { return d2 < o.d2 || (d2 == o.d2 && id < o.id); }
};

// Is displacement d (from the target centroid) in the closed cone through
// the vertices of local face k?  (k = KS: the central stencil, no cone.)
bool in_cone(const Mesh& m, int i, int k, const double d[3]) {
  if (k == KS) return true;
  const double* X = &m.X[(size_t)i * 12];
  const double* c = &m.cen[3 * (size_t)i];
  double A[3], B[3], C[3];
  for (int a = 0; a < 3; ++a) {
    A[a] = X[3 * FV[k][0] + a] - c[a];
    B[a] = X[3 * FV[k][1] + a] - c[a];
    C[a] = X[3 * FV[k][2] + a] - c[a];
  }
  // d = alpha A + beta B + gamma C (Cramer's rule); all three >= 0
  const double D = det3(A, B, C);
  const double al = det3(d, B, C), be = det3(A, d, C), ga = det3(A, B, d);
  return al * D >= 0.0 && be * D >= 0.0 && ga * D >= 0.0;
}

int stencil_rows(int degree) {
  int nk = (degree + 1) * (degree + 2) * (degree + 3) / 6;
  return 2 * nk - 1;
}

void disp(const Mesh& m, int i, int j, double d[3], double* shift = nullptr) {
  for (int a = 0; a < 3; ++a) d[a] = m.cen[3 * (size_t)j + a] - m.cen[3 * (size_t)i + a];
  min_image(m, d, shift);
}

bool stencil_brute(const Mesh& m, int i, int k, int want, std::vector<int>& out) {
  std::vector<Cand> c, rest;
  for (int j = 0; j < m.nc; ++j) {
    if (j == i) continue;
    double d[3];
    disp(m, i, j, d);
    double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (in_cone(m, i, k, d))
      c.push_back({d2, j});
    else
      rest.push_back({d2, j});
  }
  std::sort(c.begin(), c.end());
  out.clear();
  for (int s = 0; s < want && s < (int)c.size(); ++s) out.push_back(c[s].id);
  if ((int)out.size() < want && !m.periodic) {
    std::sort(rest.begin(), rest.end());
    for (size_t s = 0; s < rest.size() && (int)out.size() < want; ++s) out.push_back(rest[s].id);
  }
  return (int)out.size() == want;
}

void build_bins(Mesh& m) {
  if (!m.periodic) return;
  int nb = std::max(1, (int)std::cbrt((double)m.nc / 6.0));
  m.nb = nb;
  for (int a = 0; a < 3; ++a) m.bw[a] = m.P[a] / nb;
  std::vector<int> cnt(nb * nb * nb + 1, 0), bid(m.nc);
  for (int i = 0; i < m.nc; ++i) {
    int b[3];
    for (int a = 0; a < 3; ++a) {
      double x = m.cen[3 * (size_t)i + a];
      x -= m.P[a] * std::floor(x / m.P[a]);
      b[a] = std::min(nb - 1, std::max(0, (int)(x / m.bw[a])));
    }
    bid[i] = (b[2] * nb + b[1]) * nb + b[0];
    cnt[bid[i] + 1]++;
  }
  for (int b = 0; b < nb * nb * nb; ++b) cnt[b + 1] += cnt[b];
  m.bin_start = cnt;
  m.bin_cells.assign(m.nc, 0);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < m.nc; ++i) m.bin_cells[fill[bid[i]]++] = i;
}

// Shell search over the bin grid (periodic meshes); brute force otherwise.
bool stencil_search(const Mesh& m, int i, int k, int want, std::vector<int>& out) {
  if (!m.periodic || m.nb < 7) return stencil_brute(m, i, k, want, out);
  const int nb = m.nb;
  int b0[3];
  for (int a = 0; a < 3; ++a) {
    double x = m.cen[3 * (size_t)i + a];
    x -= m.P[a] * std::floor(x / m.P[a]);
    b0[a] = std::min(nb - 1, std::max(0, (int)(x / m.bw[a])));
  }
  const double bw = std::min(m.bw[0], std::min(m.bw[1], m.bw[2]));
  std::vector<Cand> c;
  for (int r = 0;; ++r) {
    if (2 * r + 1 > nb) return stencil_brute(m, i, k, want, out);
    for (int dz = -r; dz <= r; ++dz)
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) != r) continue;
          int bx = ((b0[0] + dx) % nb + nb) % nb, by = ((b0[1] + dy) % nb + nb) % nb;
          int bz = ((b0[2] + dz) % nb + nb) % nb;
          int b = (bz * nb + by) * nb + bx;
          for (int t = m.bin_start[b]; t < m.bin_start[b + 1]; ++t) {
            int j = m.bin_cells[t];
            if (j == i) continue;
            double d[3];
            disp(m, i, j, d);
            if (!in_cone(m, i, k, d)) continue;
            c.push_back({d[0] * d[0] + d[1] * d[1] + d[2] * d[2], j});
          }
        }
    if ((int)c.size() >= want) {
      std::nth_element(c.begin(), c.begin() + (want - 1), c.end());
      double kth = c[want - 1].d2;
      double bound = (r - 0.01) * bw;
      if (bound > 0.0 && kth < bound * bound) break;
    }
  }
  std::sort(c.begin(), c.end());
  out.clear();
  for (int s = 0; s < want; ++s) out.push_back(c[s].id);
  return true;
}

// ---------------------------------------------------------------------------
// Reconstruction set-up of one cell: stencils, A matrices, QR (Sec. 2.2)
// ---------------------------------------------------------------------------
bool build_cell(Mesh& m, int i, std::string& err) {
  CellData& cd = m.cd[i];
  if (cd.built) return true;
  const double* X0 = &m.X[(size_t)i * 12];
  // reference map: x - v0 = J (xi, eta, zeta), J's columns v1-v0, v2-v0, v3-v0
  double J[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) J[a][c] = X0[3 * (c + 1) + a] - X0[a];
  double col0[3] = {J[0][0], J[1][0], J[2][0]}, col1[3] = {J[0][1], J[1][1], J[2][1]},
         col2[3] = {J[0][2], J[1][2], J[2][2]};
  const double det = det3(col0, col1, col2);
  // rows of J^-1: cross products of columns over det
  double Ji[3][3];
  {
    double r0[3], r1[3], r2[3];
    cross(col1, col2, r0);
    cross(col2, col0, r1);
    cross(col0, col1, r2);
    for (int c = 0; c < 3; ++c) {
      Ji[0][c] = r0[c] / det;
      Ji[1][c] = r1[c] / det;
      Ji[2][c] = r2[c] / det;
    }
  }
  for (int k = 0; k <= KS; ++k) {
    const Basis& B = (k == KS) ? m.big : m.small;
    const int want = stencil_rows(B.r);
    Stencil& S = cd.st[k];
    if (!stencil_search(m, i, k, want, S.cells)) {
      err = "too few stencil candidates for cell " + std::to_string(i);
      return false;
    }
    const int n = B.n();
    TetRule rule = tet_rule(B.r / 2 + 3);
    S.qr.m = want;
    S.qr.n = n;
    S.qr.a.assign((size_t)want * n, 0.0);
    S.vol.assign(want, 0.0);
    for (int s = 0; s < want; ++s) {
      const int j = S.cells[s];
      double d[3], sh[3];
      disp(m, i, j, d, sh);
      for (int a = 0; a < 3; ++a)
        if (m.P[a] > 0.0 && std::fabs(d[a]) > 0.4 * m.P[a]) {
          err = "mesh too small for the stencil (member beyond 0.4 period) at cell " +
                std::to_string(i);
          return false;
        }
      const double* Xj = &m.X[(size_t)j * 12];
      double q[4][3];
      for (int v = 0; v < 4; ++v) {
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = Xj[3 * v + a] + sh[a] - X0[a];
        for (int r = 0; r < 3; ++r) q[v][r] = Ji[r][0] * p[0] + Ji[r][1] * p[1] + Ji[r][2] * p[2];
      }
      double e1[3], e2[3], e3[3];
      for (int a = 0; a < 3; ++a) {
        e1[a] = q[1][a] - q[0][a];
        e2[a] = q[2][a] - q[0][a];
        e3[a] = q[3][a] - q[0][a];
      }
      const double jac = std::fabs(det3(e1, e2, e3));  // 6 |V'_s|
      S.vol[s] = jac / 6.0;
      for (int l = 0; l < n; ++l) {
        double acc = 0.0;
        for (size_t t = 0; t < rule.w.size(); ++t) {
          double x[3];
          for (int a = 0; a < 3; ++a)
            x[a] = q[0][a] + rule.xi[t] * e1[a] + rule.eta[t] * e2[a] + rule.zeta[t] * e3[a];
          acc += rule.w[t] * ipow(x[0], B.ea[l]) * ipow(x[1], B.eb[l]) * ipow(x[2], B.ec[l]);
        }
        // int_{V'_s} psi_l = int phi_l - |V'_s| mean_{V'_0}(phi_l)
        S.qr.a[(size_t)l * want + s] = acc * jac - S.vol[s] * B.mean[l];
      }
    }
    if (!qr_factor(S.qr)) {
      err = "rank-deficient least-squares matrix at cell " + std::to_string(i);
      return false;
    }
  }
  cd.built = true;
  return true;
}

// ---------------------------------------------------------------------------
// Smoothness indicator (Sec. 2.3): sum over multi-indices 1 <= |alpha| <= r
// of int_{T_ref} (D^alpha P)^2, each alpha once.
// ---------------------------------------------------------------------------
double falling(int a, int k) {
  double v = 1.0;
  for (int t = 0; t < k; ++t) v *= (a - t);
  return v;
}

double smoothness(const Basis& B, const double* a) {
  TetRule q = tet_rule(B.r + 2);
  double beta = 0.0;
  for (int d = 1; d <= B.r; ++d)
    for (int ax = d; ax >= 0; --ax)
      for (int ay = d - ax; ay >= 0; --ay) {
        const int az = d - ax - ay;
        double acc = 0.0;
        for (size_t t = 0; t < q.w.size(); ++t) {
          double v = 0.0;
          for (int l = 0; l < B.n(); ++l) {
            if (B.ea[l] < ax || B.eb[l] < ay || B.ec[l] < az) continue;
            v += a[l] * falling(B.ea[l], ax) * falling(B.eb[l], ay) * falling(B.ec[l], az) *
                 ipow(q.xi[t], B.ea[l] - ax) * ipow(q.eta[t], B.eb[l] - ay) *
                 ipow(q.zeta[t], B.ec[l] - az);
          }
          acc += q.w[t] * v * v;
        }
        beta += acc;
      }
  return beta;
}

// ---------------------------------------------------------------------------
// Selection (Sec. 3.2-3.3) with K = 4 small stencils
// ---------------------------------------------------------------------------
struct Sel {
  unsigned flags = 0;  // bit 4 = large kept; bit k = small stencil k kept
  int ties = 0;
  double chiK = 0.0, chi_small[KS] = {0, 0, 0, 0};
};

double gamma_of(double beta, const oracle3_params& p) { return 1.0 / ipow(beta + p.eps, p.power); }

bool near_tie(double chi, const oracle3_params& p) {
  if (!(p.ct > 0.0)) return false;
  return std::fabs(chi / p.ct - 1.0) <= p.tie_rel;
}

Sel select(const double beta[KS + 1], const oracle3_params& p) {
  Sel s;
  if (p.variant == 1) {
    s.flags = 1u << KS;
    return s;
  }
  double g[KS + 1], sum_all = 0.0;
  for (int k = 0; k <= KS; ++k) {
    g[k] = gamma_of(beta[k], p);
    sum_all += g[k];
  }
  s.chiK = g[KS] / sum_all;
  if (near_tie(s.chiK, p)) s.ties++;
  if (s.chiK >= p.ct) {
    s.flags = 1u << KS;
    return s;
  }
  double sum_small = 0.0;
  for (int k = 0; k < KS; ++k) sum_small += g[k];
  for (int k = 0; k < KS; ++k) {
    s.chi_small[k] = g[k] / sum_small;
    if (near_tie(s.chi_small[k], p)) s.ties++;
    if (s.chi_small[k] >= p.ct) s.flags |= (1u << k);
  }
  return s;
}

bool physical(const double* u, double g) {
  for (int c = 0; c < NV; ++c)
    if (std::isnan(u[c])) return false;
  if (!(u[0] > 0.0)) return false;
  double p = (g - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
  return p > 0.0;
}

void note_bad(oracle3_diag* dg, int cell) {
  if (!dg) return;
  dg->nonphysical++;
  if (dg->first_bad_cell < 0 || cell < dg->first_bad_cell) dg->first_bad_cell = cell;
}

// ---------------------------------------------------------------------------
// Reconstruction of one cell: fp [4 faces][npt][5], flags (5 bits per
// variable), ties (0x1F per variable with a near tie)
// ---------------------------------------------------------------------------
void reconstruct_cell(const Mesh& m, int i, const double* U, bool frozen, uint32_t& flags,
                      double* fp, double* beta_out, oracle3_diag* dg, uint32_t* ties_out) {
  const CellData& cd = m.cd[i];
  const int nb = m.big.n(), ns = m.small.n(), npt = (int)m.rule.w.size();
  uint32_t out_flags = 0, tie = 0;
  for (int v = 0; v < NV; ++v) {
    const double u0 = U[NV * (size_t)i + v];
    std::vector<double> coef[KS + 1];
    for (int k = 0; k <= KS; ++k) {
      const Stencil& S = cd.st[k];
      std::vector<double> b(S.qr.m);
      for (int s = 0; s < S.qr.m; ++s) b[s] = S.vol[s] * (U[NV * (size_t)S.cells[s] + v] - u0);
      coef[k].assign(S.qr.n, 0.0);
      qr_solve(S.qr, b.data(), coef[k].data());
    }
    unsigned f5;
    if (frozen) {
      f5 = (flags >> (5 * v)) & 0x1Fu;
    } else {
      double beta[KS + 1];
      for (int k = 0; k <= KS; ++k) beta[k] = smoothness(k == KS ? m.big : m.small, coef[k].data());
      if (beta_out)
        for (int k = 0; k <= KS; ++k) beta_out[(KS + 1) * v + k] = beta[k];
      Sel s = select(beta, m.prm);
      f5 = s.flags;
      if (s.ties) tie |= 0x1Fu << (5 * v);
      if (dg) {
        dg->near_ties += s.ties;
        if (f5 & (1u << KS)) dg->large_kept++;
      }
    }
    out_flags |= f5 << (5 * v);
    // combined coefficients: the large stencil's, else the mean of the kept
    // small stencils' (Sec. 3.3 eq. TENO_weight)
    std::vector<double> abar(nb, 0.0);
    if (f5 & (1u << KS)) {
      abar = coef[KS];
    } else {
      int cnt = 0;
      for (int k = 0; k < KS; ++k) cnt += (f5 >> k) & 1u;
      for (int l = 0; l < ns && cnt > 0; ++l) {
        double acc = 0.0;
        for (int k = 0; k < KS; ++k)
          if (f5 & (1u << k)) acc += coef[k][l];
        abar[l] = acc / (double)cnt;
      }
    }
    for (int e = 0; e < 4; ++e)
      for (int q = 0; q < npt; ++q) {
        double ref[3];
        face_ref_point(e, m.rule.l0[q], m.rule.l1[q], m.rule.l2[q], ref);
        double val = u0;
        for (int l = 0; l < nb; ++l) val += abar[l] * psi(m.big, l, ref[0], ref[1], ref[2]);
        fp[(e * npt + q) * NV + v] = val;
      }
  }
  if (!frozen) {
    double u[NV];
    for (int c = 0; c < NV; ++c) u[c] = U[NV * (size_t)i + c];
    bool avg_ok = physical(u, m.prm.gamma), fp_ok = true;
    for (int q = 0; q < 4 * npt && fp_ok; ++q) fp_ok = physical(&fp[q * NV], m.prm.gamma);
    if (!(avg_ok && fp_ok)) note_bad(dg, i);
    if (!fp_ok && avg_ok && m.prm.fallback) {
      for (int q = 0; q < 4 * npt; ++q)
        for (int c = 0; c < NV; ++c) fp[q * NV + c] = u[c];
      out_flags = 0;
      if (dg) dg->fallbacks++;
    }
  }
  flags = out_flags;
  if (ties_out) *ties_out = tie;
}

// ---------------------------------------------------------------------------
// Rotated HLL flux with Einfeldt/Roe speeds (Sec. 4), 3D frame
// ---------------------------------------------------------------------------
void frame(const double n[3], double t1[3], double t2[3]) {
  // t1 = n x e_a / |n x e_a| with e_a the axis least aligned with n
  int a = 0;
  if (std::fabs(n[1]) < std::fabs(n[a])) a = 1;
  if (std::fabs(n[2]) < std::fabs(n[a])) a = 2;
  double e[3] = {0, 0, 0};
  e[a] = 1.0;
  cross(n, e, t1);
  double l = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
  for (int c = 0; c < 3; ++c) t1[c] /= l;
  cross(n, t1, t2);
}

void hll_flux(const double* uL, const double* uR, const double n[3], double g, double* out) {
  double t1[3], t2[3];
  frame(n, t1, t2);
  auto rot = [&](const double* u, double* w) {  // T U
    w[0] = u[0];
    w[1] = u[1] * n[0] + u[2] * n[1] + u[3] * n[2];
    w[2] = u[1] * t1[0] + u[2] * t1[1] + u[3] * t1[2];
    w[3] = u[1] * t2[0] + u[2] * t2[1] + u[3] * t2[2];
    w[4] = u[4];
  };
  double L[NV], R[NV];
  rot(uL, L);
  rot(uR, R);
  auto flux = [&](const double* w, double* F, double& un, double& c, double& H) {
    double rho = w[0], u = w[1] / rho, v = w[2] / rho, ww = w[3] / rho;
    double p = (g - 1.0) * (w[4] - 0.5 * rho * (u * u + v * v + ww * ww));
    F[0] = rho * u;
    F[1] = rho * u * u + p;
    F[2] = rho * u * v;
    F[3] = rho * u * ww;
    F[4] = u * (w[4] + p);
    un = u;
    c = std::sqrt(g * p / rho);
    H = (w[4] + p) / rho;
  };
  double FL[NV], FR[NV], unL, cL, HL, unR, cR, HR;
  flux(L, FL, unL, cL, HL);
  flux(R, FR, unR, cR, HR);
  // Roe averages
  const double D = std::sqrt(R[0] / L[0]);
  auto roe = [&](double xl, double xr) { return (xl + D * xr) / (1.0 + D); };
  const double ut = roe(L[1] / L[0], R[1] / R[0]);
  const double vt = roe(L[2] / L[0], R[2] / R[0]);
  const double wt = roe(L[3] / L[0], R[3] / R[0]);
  const double Ht = roe(HL, HR);
  const double ct = std::sqrt((g - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt + wt * wt)));
  const double SL = std::min(unL - cL, ut - ct);
  const double SR = std::max(unR + cR, ut + ct);
  double F[NV];
  if (SL >= 0.0) {
    for (int c = 0; c < NV; ++c) F[c] = FL[c];
  } else if (SR <= 0.0) {
    for (int c = 0; c < NV; ++c) F[c] = FR[c];
  } else {
    for (int c = 0; c < NV; ++c) F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (R[c] - L[c])) / (SR - SL);
  }
  // back to the Cartesian frame: T^-1
  out[0] = F[0];
  for (int a = 0; a < 3; ++a) out[1 + a] = F[1] * n[a] + F[2] * t1[a] + F[3] * t2[a];
  out[4] = F[4];
}

// outer state of boundary face b: transmissive copies the inner state,
// reflective reverses the normal momentum
void boundary_state(const Mesh& m, int b, const double* uL, const double n[3], double* uR) {
  for (int c = 0; c < NV; ++c) uR[c] = uL[c];
  if (m.bkind[b] == 2) {
    const double mn = uL[1] * n[0] + uL[2] * n[1] + uL[3] * n[2];
    for (int a = 0; a < 3; ++a) uR[1 + a] = uL[1 + a] - 2.0 * mn * n[a];
  }
}

void face_flux(const Mesh& m, int f, const double* fp, double* phi) {
  const int npt = (int)m.rule.w.size();
  const int L = m.fL[f], R = m.fR[f], eL = m.fLe[f], eR = m.fRe[f];
  const double* n = &m.fn[3 * (size_t)f];
  for (int c = 0; c < NV; ++c) phi[c] = 0.0;
  for (int k = 0; k < npt; ++k) {
    const double* uL = &fp[(((size_t)L * 4 + eL) * npt + k) * NV];
    double ub[NV];
    const double* uR = ub;
    if (R >= 0)
      uR = &fp[(((size_t)R * 4 + eR) * npt + m.pair[(size_t)f * npt + k]) * NV];
    else
      boundary_state(m, m.bidx[f], uL, n, ub);
    double F[NV];
    hll_flux(uL, uR, n, m.prm.gamma, F);
    for (int c = 0; c < NV; ++c) phi[c] += m.rule.w[k] * F[c];
  }
  for (int c = 0; c < NV; ++c) phi[c] *= m.farea[f];
}

void assemble(const Mesh& m, const std::vector<double>& phi, int i, double* Ri) {
  double acc[NV] = {0, 0, 0, 0, 0};
  for (int e = 0; e < 4; ++e) {
    const int f = m.cf[4 * (size_t)i + e];
    const double s = (m.fL[f] == i && m.fLe[f] == e) ? 1.0 : -1.0;
    for (int c = 0; c < NV; ++c) acc[c] += s * phi[NV * (size_t)f + c];
  }
  for (int c = 0; c < NV; ++c) Ri[c] = -acc[c] / m.vol[i];
}

void residual_full(const Mesh& m, const double* U, double* R, uint32_t* flags, bool frozen,
                   double* fp_out, oracle3_diag* dg, uint32_t* ties) {
  const int npt = (int)m.rule.w.size();
  std::vector<double> fp((size_t)m.nc * 4 * npt * NV);
  std::vector<uint32_t> fl(m.nc, 0), tl(m.nc, 0);
  if (frozen)
    for (int i = 0; i < m.nc; ++i) fl[i] = flags[i];
  int64_t nt = 0, lk = 0, fb = 0, nbad = 0, first = m.nc;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nt, lk, fb, nbad) reduction(min : first)
  for (int i = 0; i < m.nc; ++i) {
    oracle3_diag local{0, -1, 0, 0, 0};
    reconstruct_cell(m, i, U, frozen, fl[i], &fp[(size_t)i * 4 * npt * NV], nullptr, &local, &tl[i]);
    nt += local.near_ties;
    lk += local.large_kept;
    fb += local.fallbacks;
    nbad += local.nonphysical;
    if (local.nonphysical && i < first) first = i;
  }
  if (dg) {
    dg->near_ties += nt;
    dg->large_kept += lk;
    dg->fallbacks += fb;
    dg->nonphysical += nbad;
    if (nbad > 0 && (dg->first_bad_cell < 0 || first < dg->first_bad_cell)) dg->first_bad_cell = first;
  }
  if (fp_out) std::copy(fp.begin(), fp.end(), fp_out);
  std::vector<double> phi((size_t)m.nf * NV);
#pragma omp parallel for schedule(static)
  for (int f = 0; f < m.nf; ++f) face_flux(m, f, fp.data(), &phi[NV * (size_t)f]);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < m.nc; ++i) assemble(m, phi, i, &R[NV * (size_t)i]);
  if (flags && !frozen)
    for (int i = 0; i < m.nc; ++i) flags[i] = fl[i];
  if (ties)
    for (int i = 0; i < m.nc; ++i) ties[i] = frozen ? 0u : tl[i];
}

bool ready(const Mesh& m) {
  if (!m.have_params) {
    g_err = "oracle3_setup not called";
    return false;
  }
  return true;
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

const char* oracle3_last_error(void) { return g_err.c_str(); }

void oracle3_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}

// Mesh of tetrahedra: xyz [nv][3], tet [nc][4] (either orientation),
// period [3] (0 = open axis) or NULL (all open).
void* oracle3_mesh_create(int nv, const double* xyz, int nc, const int* tet, const double* period) {
  if (nv <= 0 || nc <= 0 || !xyz || !tet) {
    fail("empty mesh");
    return nullptr;
  }
  Mesh* m = new Mesh();
  m->nv = nv;
  m->nc = nc;
  m->xyz.assign(xyz, xyz + 3 * (size_t)nv);
  m->tet.assign(tet, tet + 4 * (size_t)nc);
  if (period)
    for (int a = 0; a < 3; ++a) m->P[a] = period[a] > 0.0 ? period[a] : 0.0;
  m->periodic = m->P[0] > 0.0 && m->P[1] > 0.0 && m->P[2] > 0.0;
  m->X.assign((size_t)nc * 12, 0.0);
  m->vol.assign(nc, 0.0);
  m->cen.assign(3 * (size_t)nc, 0.0);
  for (int i = 0; i < nc; ++i) {
    int* t = &m->tet[4 * (size_t)i];
    for (int v = 0; v < 4; ++v)
      if (t[v] < 0 || t[v] >= nv) {
        fail("vertex index out of range");
        delete m;
        return nullptr;
      }
    double p[4][3];
    for (int v = 0; v < 4; ++v)
      for (int a = 0; a < 3; ++a) p[v][a] = xyz[3 * (size_t)t[v] + a];
    for (int v = 1; v < 4; ++v) {
      double d[3] = {p[v][0] - p[0][0], p[v][1] - p[0][1], p[v][2] - p[0][2]};
      min_image(*m, d);
      for (int a = 0; a < 3; ++a) p[v][a] = p[0][a] + d[a];
    }
    double e1[3], e2[3], e3[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = p[1][a] - p[0][a];
      e2[a] = p[2][a] - p[0][a];
      e3[a] = p[3][a] - p[0][a];
    }
    double d6 = det3(e1, e2, e3);
    if (d6 < 0.0) {
      std::swap(t[2], t[3]);
      for (int a = 0; a < 3; ++a) std::swap(p[2][a], p[3][a]);
      d6 = -d6;
    }
    if (!(d6 > 0.0)) {
      fail("degenerate tetrahedron " + std::to_string(i));
      delete m;
      return nullptr;
    }
    m->vol[i] = d6 / 6.0;
    for (int v = 0; v < 4; ++v)
      for (int a = 0; a < 3; ++a) m->X[(size_t)i * 12 + 3 * v + a] = p[v][a];
    for (int a = 0; a < 3; ++a) m->cen[3 * (size_t)i + a] = 0.25 * (p[0][a] + p[1][a] + p[2][a] + p[3][a]);
  }
  // faces: key = sorted global vertex ids; L = lower (cell, local face)
  struct HF {
    int a, b, c, id;  // sorted vertex ids, 4 * cell + local face
    bool operator<(const HF& o) const {
      if (a != o.a) return a < o.a;
      if (b != o.b) return b < o.b;
      if (c != o.c) return c < o.c;
      return id < o.id;
    }
  };
  std::vector<HF> hf;
  hf.reserve(4 * (size_t)nc);
  for (int i = 0; i < nc; ++i)
    for (int e = 0; e < 4; ++e) {
      int v[3] = {m->tet[4 * (size_t)i + FV[e][0]], m->tet[4 * (size_t)i + FV[e][1]],
                  m->tet[4 * (size_t)i + FV[e][2]]};
      std::sort(v, v + 3);
      hf.push_back({v[0], v[1], v[2], 4 * i + e});
    }
  std::sort(hf.begin(), hf.end());
  m->cf.assign(4 * (size_t)nc, -1);
  auto face_geom = [&](int ci, int ce) {
    const double* X = &m->X[(size_t)ci * 12];
    double ab[3], ac[3], nn[3];
    for (int a = 0; a < 3; ++a) {
      ab[a] = X[3 * FV[ce][1] + a] - X[3 * FV[ce][0] + a];
      ac[a] = X[3 * FV[ce][2] + a] - X[3 * FV[ce][0] + a];
    }
    cross(ab, ac, nn);
    double l = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    for (int a = 0; a < 3; ++a) m->fn.push_back(nn[a] / l);
    m->farea.push_back(0.5 * l);
  };
  for (size_t t = 0; t < hf.size();) {
    size_t u = t + 1;
    while (u < hf.size() && hf[u].a == hf[t].a && hf[u].b == hf[t].b && hf[u].c == hf[t].c) ++u;
    if (u - t > 2) {
      fail("non-manifold face");
      delete m;
      return nullptr;
    }
    const int ci = hf[t].id / 4, ce = hf[t].id % 4;
    const int f = m->nf++;
    m->fL.push_back(ci);
    m->fLe.push_back(ce);
    face_geom(ci, ce);
    m->cf[4 * (size_t)ci + ce] = f;
    if (u - t == 2) {
      const int cj = hf[t + 1].id / 4, cje = hf[t + 1].id % 4;
      m->fR.push_back(cj);
      m->fRe.push_back(cje);
      m->cf[4 * (size_t)cj + cje] = f;
    } else {
      if (m->periodic) {
        fail("open face on a mesh periodic in all axes");
        delete m;
        return nullptr;
      }
      m->fR.push_back(-1);
      m->fRe.push_back(-1);
      m->bface.push_back(f);
    }
    t = u;
  }
  m->bidx.assign(m->nf, -1);
  for (size_t b = 0; b < m->bface.size(); ++b) m->bidx[m->bface[b]] = (int)b;
  m->bkind.assign(m->bface.size(), 1);
  return m;
}

void oracle3_mesh_destroy(void* h) { delete (Mesh*)h; }

int oracle3_mesh_counts(void* h, int* nc, int* nf, int* nb) {
  Mesh* m = (Mesh*)h;
  if (nc) *nc = m->nc;
  if (nf) *nf = m->nf;
  if (nb) *nb = (int)m->bface.size();
  return 0;
}

// vol [nc], cen [nc][3], tet [nc][4] as oriented
int oracle3_mesh_geometry(void* h, double* vol, double* cen, int* tet) {
  Mesh* m = (Mesh*)h;
  if (vol) std::copy(m->vol.begin(), m->vol.end(), vol);
  if (cen) std::copy(m->cen.begin(), m->cen.end(), cen);
  if (tet) std::copy(m->tet.begin(), m->tet.end(), tet);
  return 0;
}

// fL, fR, fLe, fRe [nf], normal [nf][3] (out of L), area [nf], cf [nc][4]
int oracle3_mesh_faces(void* h, int* fL, int* fR, int* fLe, int* fRe, double* n, double* area,
                       int* cf) {
  Mesh* m = (Mesh*)h;
  std::copy(m->fL.begin(), m->fL.end(), fL);
  std::copy(m->fR.begin(), m->fR.end(), fR);
  std::copy(m->fLe.begin(), m->fLe.end(), fLe);
  std::copy(m->fRe.begin(), m->fRe.end(), fRe);
  std::copy(m->fn.begin(), m->fn.end(), n);
  std::copy(m->farea.begin(), m->farea.end(), area);
  std::copy(m->cf.begin(), m->cf.end(), cf);
  return 0;
}

// boundary faces: verts [nb][3] (user vertex ids in the cell's local face
// order), cell [nb]
int oracle3_boundary_faces(void* h, int* verts, int* cell) {
  Mesh* m = (Mesh*)h;
  for (size_t b = 0; b < m->bface.size(); ++b) {
    const int f = m->bface[b], i = m->fL[f], e = m->fLe[f];
    for (int j = 0; j < 3; ++j) verts[3 * b + j] = m->tet[4 * (size_t)i + FV[e][j]];
    if (cell) cell[b] = i;
  }
  return 0;
}

// kind [nb]: 1 transmissive, 2 reflective
int oracle3_set_boundary(void* h, const int* kind) {
  Mesh* m = (Mesh*)h;
  for (size_t b = 0; b < m->bface.size(); ++b) {
    if (kind[b] != 1 && kind[b] != 2) return fail("boundary kind must be 1 or 2");
    m->bkind[b] = kind[b];
  }
  return 0;
}

int oracle3_setup(void* h, const oracle3_params* p, int all) {
  Mesh* m = (Mesh*)h;
  if (p->order < 3 || p->order > 6) return fail("order must be 3..6");
  if (p->variant != 0 && p->variant != 1) return fail("variant must be 0 (TENO) or 1 (LINEAR)");
  if (p->ct < 0.0 || p->ct > 1.0 / KS) return fail("C_T must lie in [0, 1/K]");
  m->prm = *p;
  m->big = make_basis(p->order - 1);
  m->small = make_basis(2);
  m->rule = face_rule(p->order);
  // pairing of the face points: L's point k is the neighbour's point whose
  // barycentric coordinates, in the neighbour's vertex order, name the same
  // physical point
  const int npt = (int)m->rule.w.size();
  m->pair.assign((size_t)m->nf * npt, -1);
  for (int f = 0; f < m->nf; ++f) {
    if (m->fR[f] < 0) continue;
    const int* tl = &m->tet[4 * (size_t)m->fL[f]];
    const int* tr = &m->tet[4 * (size_t)m->fR[f]];
    int vl[3], vr[3];
    for (int j = 0; j < 3; ++j) {
      vl[j] = tl[FV[m->fLe[f]][j]];
      vr[j] = tr[FV[m->fRe[f]][j]];
    }
    for (int k = 0; k < npt; ++k) {
      const double lk[3] = {m->rule.l0[k], m->rule.l1[k], m->rule.l2[k]};
      for (int q = 0; q < npt; ++q) {
        const double lq[3] = {m->rule.l0[q], m->rule.l1[q], m->rule.l2[q]};
        bool same = true;
        for (int j = 0; j < 3 && same; ++j) {
          int jl = -1;
          for (int t = 0; t < 3; ++t)
            if (vl[t] == vr[j]) jl = t;
          same = jl >= 0 && std::fabs(lq[j] - lk[jl]) <= 1e-12;
        }
        if (same) {
          m->pair[(size_t)f * npt + k] = q;
          break;
        }
      }
      if (m->pair[(size_t)f * npt + k] < 0) return fail("face points do not pair up");
    }
  }
  m->cd.assign(m->nc, CellData());
  build_bins(*m);
  m->have_params = true;
  if (all) {
    int bad = -1;
    std::string err;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < m->nc; ++i) {
      std::string e;
      if (!build_cell(*m, i, e)) {
#pragma omp critical
        {
          if (bad < 0 || i < bad) {
            bad = i;
            err = e;
          }
        }
      }
    }
    if (bad >= 0) return fail(err);
  }
  return 0;
}

// face-point pairing [nf][npt] (-1 on boundary faces); returns npt
int oracle3_face_pairing(void* h, int* pair) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  std::copy(m->pair.begin(), m->pair.end(), pair);
  return (int)m->rule.w.size();
}

int oracle3_prepare_cells(void* h, int n, const int* cells) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  std::vector<int> list(cells, cells + n);
  for (int c : list)
    if (c < 0 || c >= m->nc) return fail("cell index out of range");
  std::sort(list.begin(), list.end());
  list.erase(std::unique(list.begin(), list.end()), list.end());
  int bad = -1;
  std::string err;
#pragma omp parallel for schedule(dynamic, 16)
  for (int t = 0; t < (int)list.size(); ++t) {
    std::string e;
    if (!build_cell(*m, list[t], e)) {
#pragma omp critical
      {
        if (bad < 0) {
          bad = list[t];
          err = e;
        }
      }
    }
  }
  if (bad >= 0) return fail(err);
  return 0;
}

// Members of stencil k (0..3 directional through local face k, 4 central)
// of cell i, nearest first, target excluded; returns the row count.
int oracle3_stencil(void* h, int i, int k, int* out, int brute) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (i < 0 || i >= m->nc || k < 0 || k > KS) return fail("cell or stencil out of range");
  std::vector<int> s;
  const int want = stencil_rows(k == KS ? m->big.r : m->small.r);
  bool ok = brute ? stencil_brute(*m, i, k, want, s) : stencil_search(*m, i, k, want, s);
  if (!ok) return fail("too few candidates");
  std::copy(s.begin(), s.end(), out);
  return want;
}

// M = pinv(A) diag(|V'_s|) of stencil k of cell i: [n_coef][rows] row-major
int oracle3_lsq_operator(void* h, int i, int k, double* M, double* rcond) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (oracle3_prepare_cells(h, 1, &i)) return -1;
  const Stencil& S = m->cd[i].st[k];
  std::vector<double> e(S.qr.m, 0.0), x(S.qr.n);
  for (int s = 0; s < S.qr.m; ++s) {
    e[s] = S.vol[s];
    qr_solve(S.qr, e.data(), x.data());
    e[s] = 0.0;
    for (int l = 0; l < S.qr.n; ++l) M[(size_t)l * S.qr.m + s] = x[l];
  }
  if (rcond) *rcond = S.qr.rmin / S.qr.rmax;
  return S.qr.m;
}

// fp [n][4][npt][5], flags [n], beta [n][5 vars][5 stencils] (nullable), ties [n]
int oracle3_reconstruct_cells(void* h, const double* U, int n, const int* cells, double* fp,
                              uint32_t* flags, double* beta, oracle3_diag* dg, uint32_t* ties) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (oracle3_prepare_cells(h, n, cells)) return -1;
  const int npt = (int)m->rule.w.size();
  int64_t nt = 0, lk = 0, fb = 0, nbad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nt, lk, fb, nbad)
  for (int t = 0; t < n; ++t) {
    oracle3_diag local{0, -1, 0, 0, 0};
    uint32_t fl = 0, tl = 0;
    reconstruct_cell(*m, cells[t], U, false, fl, &fp[(size_t)t * 4 * npt * NV],
                     beta ? &beta[(size_t)t * NV * (KS + 1)] : nullptr, &local, &tl);
    if (flags) flags[t] = fl;
    if (ties) ties[t] = tl;
    nt += local.near_ties;
    lk += local.large_kept;
    fb += local.fallbacks;
    nbad += local.nonphysical;
  }
  if (dg) {
    dg->near_ties += nt;
    dg->large_kept += lk;
    dg->fallbacks += fb;
    dg->nonphysical += nbad;
  }
  return 0;
}

// Full residual R [nc][5]; flags [nc] out (in when frozen); fp_out
// [nc][4][npt][5] nullable; ties [nc] nullable
int oracle3_residual(void* h, const double* U, double* R, uint32_t* flags, int frozen,
                     double* fp_out, oracle3_diag* dg, uint32_t* ties) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (frozen && !flags) return fail("frozen selection needs flags");
  for (int i = 0; i < m->nc; ++i)
    if (!m->cd[i].built) return fail("oracle3_setup(all=1) required for the full residual");
  residual_full(*m, U, R, flags, frozen != 0, fp_out, dg, ties);
  return 0;
}

// Residual of the listed cells only (builds what it needs): R_out [n][5]
int oracle3_residual_cells(void* h, const double* U, int n, const int* cells, double* R_out,
                           uint32_t* flags_out) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  const int npt = (int)m->rule.w.size();
  std::vector<int> need;
  for (int t = 0; t < n; ++t) {
    const int i = cells[t];
    need.push_back(i);
    for (int e = 0; e < 4; ++e) {
      const int f = m->cf[4 * (size_t)i + e];
      const int other = (m->fL[f] == i && m->fLe[f] == e) ? m->fR[f] : m->fL[f];
      if (other >= 0) need.push_back(other);
    }
  }
  std::sort(need.begin(), need.end());
  need.erase(std::unique(need.begin(), need.end()), need.end());
  if (oracle3_prepare_cells(h, (int)need.size(), need.data())) return -1;
  std::vector<double> fpn(need.size() * 4 * npt * NV);
  std::vector<uint32_t> fln(need.size(), 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (size_t t = 0; t < need.size(); ++t)
    reconstruct_cell(*m, need[t], U, false, fln[t], &fpn[t * 4 * npt * NV], nullptr, nullptr, nullptr);
  auto slot = [&](int c) {
    return (size_t)(std::lower_bound(need.begin(), need.end(), c) - need.begin());
  };
  for (int t = 0; t < n; ++t) {
    const int i = cells[t];
    double acc[NV] = {0, 0, 0, 0, 0};
    for (int e = 0; e < 4; ++e) {
      const int f = m->cf[4 * (size_t)i + e];
      const int L = m->fL[f], R = m->fR[f], eL = m->fLe[f], eR = m->fRe[f];
      const double* nn = &m->fn[3 * (size_t)f];
      double phi[NV] = {0, 0, 0, 0, 0};
      for (int k = 0; k < npt; ++k) {
        const double* uL = &fpn[((slot(L) * 4 + eL) * npt + k) * NV];
        double ub[NV];
        const double* uR = ub;
        if (R >= 0)
          uR = &fpn[((slot(R) * 4 + eR) * npt + m->pair[(size_t)f * npt + k]) * NV];
        else
          boundary_state(*m, m->bidx[f], uL, nn, ub);
        double F[NV];
        hll_flux(uL, uR, nn, m->prm.gamma, F);
        for (int c = 0; c < NV; ++c) phi[c] += m->rule.w[k] * F[c];
      }
      const double s = (L == i && eL == e) ? 1.0 : -1.0;
      for (int c = 0; c < NV; ++c) acc[c] += s * (phi[c] * m->farea[f]);
    }
    for (int c = 0; c < NV; ++c) R_out[NV * (size_t)t + c] = -acc[c] / m->vol[i];
    if (flags_out) flags_out[t] = fln[slot(i)];
  }
  return 0;
}

// dt = cfl * min_i |V_i| / sum_f |A_if| (|u_i . n_if| + c_i)
double oracle3_dt(void* h, const double* U, double cfl) {
  Mesh* m = (Mesh*)h;
  const double g = m->have_params ? m->prm.gamma : 1.4;
  double best = INFINITY;
  for (int i = 0; i < m->nc; ++i) {
    const double* u = &U[NV * (size_t)i];
    const double vx = u[1] / u[0], vy = u[2] / u[0], vz = u[3] / u[0];
    const double p = (g - 1.0) * (u[4] - 0.5 * u[0] * (vx * vx + vy * vy + vz * vz));
    const double c = std::sqrt(g * p / u[0]);
    double den = 0.0;
    for (int e = 0; e < 4; ++e) {
      const int f = m->cf[4 * (size_t)i + e];
      const double* nn = &m->fn[3 * (size_t)f];
      den += m->farea[f] * (std::fabs(vx * nn[0] + vy * nn[1] + vz * nn[2]) + c);
    }
    best = std::min(best, m->vol[i] / den);
  }
  return cfl * best;
}

// One SSP-RK3 step; flags3 [3][nc] (out, or in when frozen); stages
// [3][nc][5] nullable (stage inputs); ties3 [3][nc] nullable
int oracle3_rk_step(void* h, const double* U, double* Uout, double dt, uint32_t* flags3,
                    int frozen, double* stages, oracle3_diag* dg, uint32_t* ties3) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  const size_t n5 = NV * (size_t)m->nc;
  std::vector<double> R(n5), U1(n5), U2(n5);
  std::vector<uint32_t> fl(m->nc);
  auto fls = [&](int s) -> uint32_t* {
    if (frozen) std::copy(flags3 + (size_t)s * m->nc, flags3 + (size_t)(s + 1) * m->nc, fl.begin());
    return fl.data();
  };
  auto keep = [&](int s) {
    if (flags3 && !frozen) std::copy(fl.begin(), fl.end(), flags3 + (size_t)s * m->nc);
  };
  auto tie = [&](int s) -> uint32_t* { return ties3 ? ties3 + (size_t)s * m->nc : nullptr; };
  if (stages) std::copy(U, U + n5, stages);
  if (oracle3_residual(h, U, R.data(), fls(0), frozen, nullptr, dg, tie(0))) return -1;
  keep(0);
  for (size_t t = 0; t < n5; ++t) U1[t] = U[t] + dt * R[t];
  if (stages) std::copy(U1.begin(), U1.end(), stages + n5);
  if (oracle3_residual(h, U1.data(), R.data(), fls(1), frozen, nullptr, dg, tie(1))) return -1;
  keep(1);
  for (size_t t = 0; t < n5; ++t) U2[t] = 0.75 * U[t] + 0.25 * U1[t] + 0.25 * (dt * R[t]);
  if (stages) std::copy(U2.begin(), U2.end(), stages + 2 * n5);
  if (oracle3_residual(h, U2.data(), R.data(), fls(2), frozen, nullptr, dg, tie(2))) return -1;
  keep(2);
  const double a = 1.0 / 3.0, b = 2.0 / 3.0;
  for (size_t t = 0; t < n5; ++t) Uout[t] = a * U[t] + b * U2[t] + b * (dt * R[t]);
  return 0;
}

// ---- stand-alone pieces for the pins ----------------------------------------
// face rule of an order: bary [npt][3], w [npt]; returns npt
int oracle3_face_rule(int order, double* bary, double* w) {
  FaceRule r = face_rule(order);
  for (size_t k = 0; k < r.w.size(); ++k) {
    bary[3 * k] = r.l0[k];
    bary[3 * k + 1] = r.l1[k];
    bary[3 * k + 2] = r.l2[k];
    w[k] = r.w[k];
  }
  return (int)r.w.size();
}

// integral of xi^a eta^b zeta^c over the reference tetrahedron (n-point rule)
double oracle3_tet_moment(int a, int b, int c, int n) {
  TetRule q = tet_rule(n);
  double acc = 0.0;
  for (size_t k = 0; k < q.w.size(); ++k)
    acc += q.w[k] * ipow(q.xi[k], a) * ipow(q.eta[k], b) * ipow(q.zeta[k], c);
  return acc;
}

int oracle3_basis(int r, int* ea, int* eb, int* ec, double* mean) {
  Basis b = make_basis(r);
  for (int l = 0; l < b.n(); ++l) {
    ea[l] = b.ea[l];
    eb[l] = b.eb[l];
    ec[l] = b.ec[l];
    mean[l] = b.mean[l];
  }
  return b.n();
}

double oracle3_smoothness(int r, const double* coef) { return smoothness(make_basis(r), coef); }

unsigned oracle3_select(const oracle3_params* p, const double* beta, double* chi, int* ties) {
  Sel s = select(beta, *p);
  if (chi) {
    for (int k = 0; k < KS; ++k) chi[k] = s.chi_small[k];
    chi[KS] = s.chiK;
  }
  if (ties) *ties = s.ties;
  return s.flags;
}

void oracle3_hll(const double* uL, const double* uR, const double* n, double g, double* out) {
  hll_flux(uL, uR, n, g, out);
}

}  // extern "C"
