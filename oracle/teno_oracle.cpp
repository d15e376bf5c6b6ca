// TEST INFRASTRUCTURE ONLY.  Plain FP64 CPU oracle of the unstructured-mesh
// finite-volume TENO residual (Ji, Liang & Fu, "A class of new high-order
// finite-volume TENO schemes for hyperbolic conservation laws with unstructured
// meshes").  Only the tests, the smoke check and the benchmark's CPU-baseline
// leg may load this library.  It shares no code with the HIP path.
//
// Everything runs in the caller's (user) cell order with host pointers.
// Conservative state layout: U[cell][4] = (rho, rho*u, rho*v, E).
//
// Steps, each following the passage cited beside it:
//   geometry and faces ................. Sec. 2.1, semi-discrete equation
//   stencils (central + directional) ... Sec. 3.1 (rules are a reading, below)
//   reference map, zero-mean basis,
//   constrained least squares, QR ...... Sec. 2.2, reconstruction eqs. 02-10
//   smoothness indicators .............. Sec. 2.3, WENO smoothness equation
//   scale separation, cutoff, selection  Sec. 3.2-3.3
//   face Gauss points .................. Sec. 2.1
//   rotation + HLL + Einfeldt speeds ... Sec. 4.1-4.2
//   residual, SSP-RK3 .................. Sec. 2.1, time-discretisation equation
//
// Readings where the paper is silent (each a parameter or documented choice):
//   * stencil rule: central = I0 + nearest 2N_k-1 cells by periodic min-image
//     centroid distance; directional j = I0 + nearest 11 cells whose centroid
//     lies in the closed cone from the target centroid through the endpoints
//     of local edge j; ties by lower user id.
//   * N_k counts the constant; N_s = 2 N_k cells including I0 (2N_k-1 rows).
//   * beta sums every derivative multi-index once, in reference coordinates.
//   * N_q = ceil(p/2) Gauss-Legendre points per face.
//   * Roe sound speed uses both Roe velocity components.
//   * dt = CFL * min_i |V_i| / sum_j |A_ij| (|u_i . n_ij| + c_i).
//   * flag bits: 4v+3 = large stencil kept (step i); 4v+k = small stencil k
//     kept in step ii.
//
// Derivatives: the residual is templated on the scalar so that a complex-step
// Jacobian-vector product is exact to round-off with the selection frozen.
// The vector-Jacobian product is the hand-transposed chain (gather, flux,
// reconstruction) with the flux Jacobian taken by complex step.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cplx;

extern "C" {
typedef struct oracle_params {
  int32_t order;    // 3..6
  int32_t nq;       // face Gauss points, 0 = ceil(order/2)
  int32_t variant;  // 0 = TENO, 1 = LINEAR (large stencil everywhere), 2 = CWENO
  int32_t power;    // scale-separation exponent (paper: 6)
  double ct;        // cutoff C_T (paper: 1e-6)
  double eps;       // epsilon in gamma_k (paper: 1e-12)
  double gamma;     // ratio of specific heats
  double tie_rel;   // near-tie band |chi/C_T - 1| <= tie_rel
  int32_t fallback; // 1: a cell with a non-physical face point uses its cell
                    // average on every face (flags 0); 0: paper as stated
  int32_t characteristic;  // 1: select in characteristic variables, per face
  double dk_prime;  // CWENO: d_K = 1 - 1/dk_prime (paper: 1e4)
} oracle_params;

typedef struct oracle_diag {
  int64_t nonphysical;    // face points / cell averages with rho<=0, p<=0 or NaN
  int64_t first_bad_cell; // lowest offending cell id, -1 if none
  int64_t near_ties;      // chi values within tie_rel of C_T
  int64_t large_kept;     // (cell, variable) pairs that kept the large stencil
  int64_t fallbacks;      // cells reconstructed at first order (fallback on)
} oracle_diag;
}

namespace {

thread_local std::string g_err;

int fail(const std::string& msg) {
  g_err = msg;
  return -1;
}

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [0, 1] by Newton iteration on P_n.
// ---------------------------------------------------------------------------
void legendre(int n, double x, double& pn, double& pm) {
  // P_n(x) and P_{n-1}(x) by the three-term recurrence (n >= 1)
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pm = p0;
}

void gauss01(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pn, pm, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, x, pn, pm);
      dp = n * (x * pn - pm) / (x * x - 1.0);
      double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) <= 1e-15) break;
    }
    legendre(n, x, pn, pm);
    dp = n * (x * pn - pm) / (x * x - 1.0);
    // x_i decreases with i, so t = (1 - x)/2 increases.
    t[i] = 0.5 * (1.0 - x);
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);  // (2/((1-x^2)P'^2)) / 2
  }
}

// Collapsed (Duffy) product rule on the triangle (q0, q1, q2):
//   x(u, s) = q0 + u (q1 - q0) + u s (q2 - q1),  dA = u |2 area| du ds.
struct TriRule {
  std::vector<double> u, s, w;  // unit-square nodes, weights include u
};

TriRule tri_rule(int n) {
  std::vector<double> t, wt;
  gauss01(n, t, wt);
  TriRule r;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      r.u.push_back(t[i]);
      r.s.push_back(t[j]);
      r.w.push_back(wt[i] * wt[j] * t[i]);
    }
  return r;
}

// ---------------------------------------------------------------------------
// Monomial basis phi = xi^a eta^b, 1 <= a+b <= r, graded order
// (xi, eta, xi^2, xi eta, eta^2, ...).  Sec. 2.2, basis definition.
// ---------------------------------------------------------------------------
struct Basis {
  int r = 0;
  std::vector<int> ea, eb;
  std::vector<double> mean;  // (1/|T_ref|) int_{T_ref} phi_l, by quadrature
  int n() const { return (int)ea.size(); }
};

double ipow(double x, int k) {
  double v = 1.0;
  for (int i = 0; i < k; ++i) v *= x;
  return v;
}

Basis make_basis(int r) {
  Basis b;
  b.r = r;
  for (int d = 1; d <= r; ++d)
    for (int a = d; a >= 0; --a) {
      b.ea.push_back(a);
      b.eb.push_back(d - a);
    }
  TriRule q = tri_rule(r + 2);
  // T_ref = (0,0), (1,0), (0,1): area 1/2; the rule's |2 area| factor is 1.
  for (int l = 0; l < b.n(); ++l) {
    double acc = 0.0;
    for (size_t k = 0; k < q.w.size(); ++k) {
      double xi = q.u[k] - q.u[k] * q.s[k];
      double eta = q.u[k] * q.s[k];
      acc += q.w[k] * ipow(xi, b.ea[l]) * ipow(eta, b.eb[l]);
    }
    b.mean.push_back(acc / 0.5);
  }
  return b;
}

double psi(const Basis& b, int l, double xi, double eta) {
  return ipow(xi, b.ea[l]) * ipow(eta, b.eb[l]) - b.mean[l];
}

// ---------------------------------------------------------------------------
// Householder QR of a column-major m x n matrix (m >= n), Sec. 2.2 eq. 10.
// ---------------------------------------------------------------------------
struct QR {
  int m = 0, n = 0;
  std::vector<double> a;     // column-major: R in the upper triangle,
                             // Householder vectors below (v_0 = 1 implicit)
  std::vector<double> beta;  // reflector scale
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
    // v = x - alpha e1 with alpha = -sign(x0) mu (no cancellation)
    double alpha = (x0 >= 0.0) ? -mu : mu;
    double v0 = x0 - alpha;
    // normalise v so that v_0 = 1
    for (int i = j + 1; i < m; ++i) col[i] /= v0;
    double vtv = 1.0;
    for (int i = j + 1; i < m; ++i) vtv += col[i] * col[i];
    double bta = 2.0 / vtv;
    q.beta[j] = bta;
    col[j] = alpha;
    // apply (I - beta v v^T) to the remaining columns
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

// Least-squares solution x = argmin |A x - b|; b has m entries, x gets n.
template <class T>
void qr_solve(const QR& q, const T* b, T* x) {
  const int m = q.m, n = q.n;
  std::vector<T> y(b, b + m);
  for (int j = 0; j < n; ++j) {
    const double* col = &q.a[(size_t)j * m];
    T s = y[j];
    for (int i = j + 1; i < m; ++i) s += col[i] * y[i];
    s *= q.beta[j];
    y[j] -= s;
    for (int i = j + 1; i < m; ++i) y[i] -= s * col[i];
  }
  for (int j = n - 1; j >= 0; --j) {
    T s = y[j];
    for (int c = j + 1; c < n; ++c) s -= q.a[(size_t)c * m + j] * x[c];
    x[j] = s / q.a[(size_t)j * m + j];
  }
}

// Transpose of the map b -> x above: given xbar (n), return bbar (m).
void qr_solve_transpose(const QR& q, const double* xbar, double* bbar) {
  const int m = q.m, n = q.n;
  std::vector<double> y(m, 0.0);
  // back substitution transposed: x = R^{-1} y[0:n]  =>  ybar = R^{-T} xbar
  for (int j = 0; j < n; ++j) {
    double s = xbar[j];
    for (int c = 0; c < j; ++c) s -= q.a[(size_t)j * m + c] * y[c];
    y[j] = s / q.a[(size_t)j * m + j];
  }
  // reflections transposed, in reverse order (each is symmetric)
  for (int j = n - 1; j >= 0; --j) {
    const double* col = &q.a[(size_t)j * m];
    double s = y[j];
    for (int i = j + 1; i < m; ++i) s += col[i] * y[i];
    s *= q.beta[j];
    y[j] -= s;
    for (int i = j + 1; i < m; ++i) y[i] -= s * col[i];
  }
  for (int i = 0; i < m; ++i) bbar[i] = y[i];
}

// ---------------------------------------------------------------------------
// Mesh
// ---------------------------------------------------------------------------
struct Stencil {
  std::vector<int> cells;      // members other than the target, nearest first
  std::vector<double> vol;     // |V'_s| of each member in reference space
  QR qr;
};

struct CellData {
  bool built = false;
  Stencil st[4];  // 0..2 directional (local edges), 3 = central (large)
};

struct Mesh {
  int nv = 0, nc = 0, nf = 0;
  bool periodic = false;              // both axes periodic
  double P[2] = {0.0, 0.0};           // period per axis; 0: open axis
  std::vector<double> xy;
  std::vector<int> tri;
  std::vector<double> X;              // [nc][3][2] unwrapped about v0
  std::vector<double> area, cen;      // cen [nc][2]
  std::vector<int> fL, fR, fLe, fRe;  // face -> cells, local edges
  std::vector<double> fn, flen;       // face unit normal (out of L), length
  std::vector<int> cf;                // [nc][3] face of each local edge
  // boundary faces (open axes): fR = fRe = -1; numbered by the (first,
  // second) vertex of the face in its cell's counter-clockwise order
  std::vector<int> bface, bidx;       // [nb] face; [nf] index or -1
  std::vector<int> bkind;             // [nb] 1 transmissive, 2 reflective, 3 prescribed
  std::vector<double> bstate;         // [nb][4]
  // reconstruction setup
  bool have_params = false;
  oracle_params prm{};
  int nq = 0;
  Basis big, small;
  std::vector<double> gq_t, gq_w;     // face rule on [0,1]
  std::vector<CellData> cd;
  // spatial bins for neighbour search
  int nbx = 0, nby = 0;
  double bwx = 0.0, bwy = 0.0;
  std::vector<int> bin_start, bin_cells;
};

void min_image(const Mesh& m, double& dx, double& dy) {
  if (m.P[0] > 0.0) dx -= m.P[0] * std::nearbyint(dx / m.P[0]);
  if (m.P[1] > 0.0) dy -= m.P[1] * std::nearbyint(dy / m.P[1]);
}

// ---------------------------------------------------------------------------
// Stencils (Sec. 3.1; rule as stated in the header)
// ---------------------------------------------------------------------------
struct Cand {
  double d2;
  int id;
  bool operator<(const Cand& o) const { return d2 < o.d2 || (d2 == o.d2 && id < o.id); }
};

// Does cell j belong to stencil kind k of cell i (geometric filter only)?
bool in_cone(const Mesh& m, int i, int k, double dx, double dy) {
  if (k == 3) return true;
  const double* X = &m.X[(size_t)i * 6];
  double cx = m.cen[2 * i], cy = m.cen[2 * i + 1];
  int a = k, b = (k + 1) % 3;
  double ax = X[2 * a] - cx, ay = X[2 * a + 1] - cy;
  double bx = X[2 * b] - cx, by = X[2 * b + 1] - cy;
  // d = alpha A + beta B with alpha, beta >= 0
  double alpha_num = dx * by - dy * bx;
  double beta_num = ax * dy - ay * dx;
  return alpha_num >= 0.0 && beta_num >= 0.0;
}

int stencil_rows(int degree) { return (degree + 1) * (degree + 2) - 1; }

// Min-image displacement of centroid j from centroid i; (sx, sy) is the
// period shift that moves cell j's coordinates to that image.
void disp(const Mesh& m, int i, int j, double& dx, double& dy, double* sx = nullptr,
          double* sy = nullptr) {
  dx = m.cen[2 * j] - m.cen[2 * i];
  dy = m.cen[2 * j + 1] - m.cen[2 * i + 1];
  double kx = 0.0, ky = 0.0;
  if (m.P[0] > 0.0) {
    kx = std::nearbyint(dx / m.P[0]);
    dx -= m.P[0] * kx;
  }
  if (m.P[1] > 0.0) {
    ky = std::nearbyint(dy / m.P[1]);
    dy -= m.P[1] * ky;
  }
  if (sx) *sx = -m.P[0] * kx;
  if (sy) *sy = -m.P[1] * ky;
}

// Reading for meshes with boundaries: a directional stencil whose cone holds
// fewer than `want` cells is completed with the nearest cells outside it.
bool stencil_brute(const Mesh& m, int i, int k, int want, std::vector<int>& out) {
  std::vector<Cand> c, rest;
  for (int j = 0; j < m.nc; ++j) {
    if (j == i) continue;
    double dx, dy;
    disp(m, i, j, dx, dy);
    if (in_cone(m, i, k, dx, dy))
      c.push_back({dx * dx + dy * dy, j});
    else
      rest.push_back({dx * dx + dy * dy, j});
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
  double lx = m.periodic ? m.P[0] : 1.0, ly = m.periodic ? m.P[1] : 1.0;
  int nb = std::max(1, (int)std::sqrt((double)m.nc / 2.0));
  m.nbx = m.nby = nb;
  m.bwx = lx / nb;
  m.bwy = ly / nb;
  std::vector<int> cnt(nb * nb + 1, 0), bid(m.nc);
  for (int i = 0; i < m.nc; ++i) {
    double x = m.cen[2 * i], y = m.cen[2 * i + 1];
    x -= lx * std::floor(x / lx);
    y -= ly * std::floor(y / ly);
    int bx = std::min(nb - 1, std::max(0, (int)(x / m.bwx)));
    int by = std::min(nb - 1, std::max(0, (int)(y / m.bwy)));
    bid[i] = by * nb + bx;
    cnt[bid[i] + 1]++;
  }
  for (int b = 0; b < nb * nb; ++b) cnt[b + 1] += cnt[b];
  m.bin_start = cnt;
  m.bin_cells.assign(m.nc, 0);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < m.nc; ++i) m.bin_cells[fill[bid[i]]++] = i;
}

// Ring search over the bin grid; falls back to brute force on small meshes.
bool stencil_search(const Mesh& m, int i, int k, int want, std::vector<int>& out) {
  if (!m.periodic || m.nbx < 7) return stencil_brute(m, i, k, want, out);
  double lx = m.P[0], ly = m.P[1];
  double x = m.cen[2 * i], y = m.cen[2 * i + 1];
  x -= lx * std::floor(x / lx);
  y -= ly * std::floor(y / ly);
  int bx0 = std::min(m.nbx - 1, std::max(0, (int)(x / m.bwx)));
  int by0 = std::min(m.nby - 1, std::max(0, (int)(y / m.bwy)));
  double bw = std::min(m.bwx, m.bwy);
  std::vector<Cand> c;
  for (int r = 0;; ++r) {
    if (2 * r + 1 > m.nbx || 2 * r + 1 > m.nby) return stencil_brute(m, i, k, want, out);
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        if (std::max(std::abs(dx), std::abs(dy)) != r) continue;
        int bx = ((bx0 + dx) % m.nbx + m.nbx) % m.nbx;
        int by = ((by0 + dy) % m.nby + m.nby) % m.nby;
        int b = by * m.nbx + bx;
        for (int t = m.bin_start[b]; t < m.bin_start[b + 1]; ++t) {
          int j = m.bin_cells[t];
          if (j == i) continue;
          double ddx, ddy;
          disp(m, i, j, ddx, ddy);
          if (!in_cone(m, i, k, ddx, ddy)) continue;
          c.push_back({ddx * ddx + ddy * ddy, j});
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
// Reconstruction set-up for one cell: stencils, A matrices, QR (Sec. 2.2)
// ---------------------------------------------------------------------------
bool build_cell(Mesh& m, int i, std::string& err) {
  CellData& cd = m.cd[i];
  if (cd.built) return true;
  const double* X0 = &m.X[(size_t)i * 6];
  double j00 = X0[2] - X0[0], j01 = X0[4] - X0[0];
  double j10 = X0[3] - X0[1], j11 = X0[5] - X0[1];
  double det = j00 * j11 - j01 * j10;
  for (int k = 0; k < 4; ++k) {
    const Basis& B = (k == 3) ? m.big : m.small;
    int want = stencil_rows(B.r);
    Stencil& S = cd.st[k];
    if (!stencil_search(m, i, k, want, S.cells)) {
      err = "too few stencil candidates for cell " + std::to_string(i);
      return false;
    }
    const int n = B.n();
    TriRule rule = tri_rule((B.r + 3) / 2 + 1);
    S.qr.m = want;
    S.qr.n = n;
    S.qr.a.assign((size_t)want * n, 0.0);
    S.vol.assign(want, 0.0);
    for (int s = 0; s < want; ++s) {
      int j = S.cells[s];
      double dx, dy, ox, oy;
      disp(m, i, j, dx, dy, &ox, &oy);
      // members must stay within 0.4 period of the target along each periodic axis
      if ((m.P[0] > 0.0 && std::fabs(dx) > 0.4 * m.P[0]) ||
          (m.P[1] > 0.0 && std::fabs(dy) > 0.4 * m.P[1])) {
        err = "mesh too small for the stencil (member beyond 0.4 period) at cell " +
              std::to_string(i);
        return false;
      }
      const double* Xj = &m.X[(size_t)j * 6];
      double q[3][2];
      for (int v = 0; v < 3; ++v) {
        double px = Xj[2 * v] + ox - X0[0], py = Xj[2 * v + 1] + oy - X0[1];
        q[v][0] = (j11 * px - j01 * py) / det;
        q[v][1] = (-j10 * px + j00 * py) / det;
      }
      double a2 = std::fabs((q[1][0] - q[0][0]) * (q[2][1] - q[1][1]) -
                            (q[1][1] - q[0][1]) * (q[2][0] - q[1][0]));
      S.vol[s] = 0.5 * a2;
      for (int l = 0; l < n; ++l) {
        double acc = 0.0;
        for (size_t t = 0; t < rule.w.size(); ++t) {
          double u = rule.u[t], w = rule.s[t];
          double xi = q[0][0] + u * (q[1][0] - q[0][0]) + u * w * (q[2][0] - q[1][0]);
          double eta = q[0][1] + u * (q[1][1] - q[0][1]) + u * w * (q[2][1] - q[1][1]);
          acc += rule.w[t] * ipow(xi, B.ea[l]) * ipow(eta, B.eb[l]);
        }
        // int_{V'_s} psi_l = int phi_l - |V'_s| * mean_{V'_0}(phi_l)
        S.qr.a[(size_t)l * want + s] = acc * a2 - S.vol[s] * B.mean[l];
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
// Smoothness indicator (Sec. 2.3): sum over derivative multi-indices
// 1 <= |alpha| <= r of int_{T_ref} (D^alpha P)^2, each alpha counted once.
// ---------------------------------------------------------------------------
double falling(int a, int k) {
  double v = 1.0;
  for (int t = 0; t < k; ++t) v *= (a - t);
  return v;
}

double smoothness(const Basis& B, const double* a) {
  TriRule q = tri_rule(B.r + 1);
  double beta = 0.0;
  for (int d = 1; d <= B.r; ++d)
    for (int ax = d; ax >= 0; --ax) {
      int ay = d - ax;
      double acc = 0.0;
      for (size_t t = 0; t < q.w.size(); ++t) {
        double xi = q.u[t] - q.u[t] * q.s[t];
        double eta = q.u[t] * q.s[t];
        double v = 0.0;
        for (int l = 0; l < B.n(); ++l) {
          if (B.ea[l] < ax || B.eb[l] < ay) continue;
          v += a[l] * falling(B.ea[l], ax) * falling(B.eb[l], ay) *
               ipow(xi, B.ea[l] - ax) * ipow(eta, B.eb[l] - ay);
        }
        acc += q.w[t] * v * v;
      }
      beta += acc;
    }
  return beta;
}

// ---------------------------------------------------------------------------
// Face points (Sec. 2.1) in reference coordinates of local edge e.
// ---------------------------------------------------------------------------
void face_point(int e, double t, double& xi, double& eta) {
  if (e == 0) { xi = t; eta = 0.0; }
  else if (e == 1) { xi = 1.0 - t; eta = t; }
  else { xi = 0.0; eta = 1.0 - t; }
}

// ---------------------------------------------------------------------------
// Selection (Sec. 3.2-3.3).  Returns the 4-bit flag of one variable and the
// combined coefficients abar (length of the large basis).
// ---------------------------------------------------------------------------
struct Sel {
  unsigned flags = 0;
  int ties = 0;
  double chiK = 0.0, chi_small[3] = {0, 0, 0};
};

double gamma_of(double beta, const oracle_params& p) {
  double x = beta + p.eps;
  return 1.0 / ipow(x, p.power);
}

bool near_tie(double chi, const oracle_params& p) {
  if (!(p.ct > 0.0)) return false;
  return std::fabs(chi / p.ct - 1.0) <= p.tie_rel;
}

Sel select(const double beta[4], const oracle_params& p) {
  Sel s;
  if (p.variant == 1) {
    s.flags = 8u;
    return s;
  }
  double g[4];
  for (int k = 0; k < 4; ++k) g[k] = gamma_of(beta[k], p);
  double sum_all = g[0] + g[1] + g[2] + g[3];
  s.chiK = g[3] / sum_all;
  if (near_tie(s.chiK, p)) s.ties++;
  if (s.chiK >= p.ct) {
    s.flags = 8u;
    return s;
  }
  double sum_small = g[0] + g[1] + g[2];
  for (int k = 0; k < 3; ++k) {
    s.chi_small[k] = g[k] / sum_small;
    if (near_tie(s.chi_small[k], p)) s.ties++;
    if (s.chi_small[k] >= p.ct) s.flags |= (1u << k);
  }
  return s;
}

// CWENO weights (Sec. 2.4): linear weights d_K = 1 - 1/d'_K for the large
// stencil and d_k = (1 - d_K)/K for the K = 3 small ones; alpha_k =
// d_k / (beta_k + eps)^power, omega_k = alpha_k / sum alpha.  d gets the
// linear weights.
void cweno_weights(const double beta[4], const oracle_params& p, double omega[4], double d[4]) {
  d[3] = 1.0 - 1.0 / p.dk_prime;
  for (int k = 0; k < 3; ++k) d[k] = (1.0 - d[3]) / 3.0;
  double alpha[4], sum = 0.0;
  for (int k = 0; k < 4; ++k) {
    alpha[k] = d[k] / ipow(beta[k] + p.eps, p.power);
    sum += alpha[k];
  }
  for (int k = 0; k < 4; ++k) omega[k] = alpha[k] / sum;
}

inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }

bool physical(const double* u, double g) {
  for (int c = 0; c < 4; ++c)
    if (std::isnan(u[c])) return false;
  if (!(u[0] > 0.0)) return false;
  double p = (g - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
  return p > 0.0;
}

void note_bad(oracle_diag* dg, int cell) {
  if (!dg) return;
  dg->nonphysical++;
  if (dg->first_bad_cell < 0 || cell < dg->first_bad_cell) dg->first_bad_cell = cell;
}

// ---------------------------------------------------------------------------
// Least-squares coefficients of variable v of cell i on its four stencils
// (Sec. 2.2 eqs. 08-10): right-hand side |V'_s| (U_s - U_0), QR solve.
// ---------------------------------------------------------------------------
template <class T>
void lsq_coefficients(const CellData& cd, const T* U, int i, int v, std::vector<T> coef[4]) {
  const T u0 = U[4 * i + v];
  for (int k = 0; k < 4; ++k) {
    const Stencil& S = cd.st[k];
    std::vector<T> b(S.qr.m);
    for (int s = 0; s < S.qr.m; ++s) b[s] = S.vol[s] * (U[4 * S.cells[s] + v] - u0);
    coef[k].assign(S.qr.n, T(0.0));
    qr_solve(S.qr, b.data(), coef[k].data());
  }
}

// Combined coefficients of the TENO selection with flags f4 (Sec. 3.3): the
// large stencil's, else the mean of the kept small stencils' (zero when none
// is kept, which only the first-order fallback produces).
template <class T>
void teno_combine(unsigned f4, const std::vector<T> coef[4], int nb, int ns, std::vector<T>& abar) {
  abar.assign(nb, T(0.0));
  if (f4 & 8u) {
    for (int l = 0; l < nb; ++l) abar[l] = coef[3][l];
    return;
  }
  int cnt = (int)((f4 & 1u) + ((f4 >> 1) & 1u) + ((f4 >> 2) & 1u));
  for (int l = 0; l < ns && cnt > 0; ++l) {
    T acc = T(0.0);
    for (int k = 0; k < 3; ++k)
      if (f4 & (1u << k)) acc += coef[k][l];
    abar[l] = acc / (double)cnt;
  }
}

// Combined coefficients of CWENO (Sec. 2.4):
// P = (w_K/d_K)(P_K - sum_k d_k P_k) + sum_k w_k P_k.
template <class T>
void cweno_combine(const double w[4], const double d[4], const std::vector<T> coef[4], int nb, int ns,
                   std::vector<T>& abar) {
  abar.assign(nb, T(0.0));
  for (int l = 0; l < nb; ++l) {
    T opt = coef[3][l];
    if (l < ns)
      for (int k = 0; k < 3; ++k) opt -= d[k] * coef[k][l];
    abar[l] = (w[3] / d[3]) * opt;
    if (l < ns)
      for (int k = 0; k < 3; ++k) abar[l] += w[k] * coef[k][l];
  }
}

// ---------------------------------------------------------------------------
// Reconstruction of one cell (all four variables); templated for complex step.
// fp gets [3][nq][4]; flags in/out (frozen when `frozen` is true).
// ---------------------------------------------------------------------------
template <class T>
void reconstruct_cell(const Mesh& m, int i, const T* U, bool frozen, uint16_t& flags,
                      T* fp, double* beta_out, oracle_diag* dg, uint16_t* ties_out = nullptr) {
  const CellData& cd = m.cd[i];
  const int nb = m.big.n(), ns = m.small.n();
  uint16_t out_flags = 0, tie_nib = 0;
  for (int v = 0; v < 4; ++v) {
    T u0 = U[4 * i + v];
    std::vector<T> coef[4];
    lsq_coefficients(cd, U, i, v, coef);
    if (m.prm.variant == 2) {
      // CWENO (Sec. 2.4): P = (w_K/d_K)(P_K - sum_k d_k P_k) + sum_k w_k P_k
      double beta[4], w[4], d[4];
      for (int k = 0; k < 4; ++k) {
        std::vector<double> rc(coef[k].size());
        for (size_t l = 0; l < rc.size(); ++l) rc[l] = std::real(coef[k][l]);
        beta[k] = smoothness(k == 3 ? m.big : m.small, rc.data());
      }
      if (beta_out) for (int k = 0; k < 4; ++k) beta_out[4 * v + k] = beta[k];
      cweno_weights(beta, m.prm, w, d);
      std::vector<T> abar;
      cweno_combine(w, d, coef, nb, ns, abar);
      for (int e = 0; e < 3; ++e)
        for (int kq = 0; kq < m.nq; ++kq) {
          double xi, eta;
          face_point(e, m.gq_t[kq], xi, eta);
          T val = u0;
          for (int l = 0; l < nb; ++l) val += abar[l] * psi(m.big, l, xi, eta);
          fp[(e * m.nq + kq) * 4 + v] = val;
        }
      continue;  // no selection: flags stay 0
    }
    unsigned f4;
    if (frozen) {
      f4 = (flags >> (4 * v)) & 0xFu;
    } else {
      double beta[4];
      for (int k = 0; k < 4; ++k) {
        std::vector<double> re(coef[k].size());
        for (size_t l = 0; l < re.size(); ++l) re[l] = std::real(coef[k][l]);
        beta[k] = smoothness(k == 3 ? m.big : m.small, re.data());
      }
      if (beta_out) for (int k = 0; k < 4; ++k) beta_out[4 * v + k] = beta[k];
      Sel s = select(beta, m.prm);
      f4 = s.flags;
      if (s.ties) tie_nib |= (uint16_t)(0xFu << (4 * v));
      if (dg) {
        dg->near_ties += s.ties;
        if (f4 & 8u) dg->large_kept++;
      }
    }
    out_flags |= (uint16_t)(f4 << (4 * v));
    std::vector<T> abar;
    teno_combine(f4, coef, nb, ns, abar);
    for (int e = 0; e < 3; ++e)
      for (int kq = 0; kq < m.nq; ++kq) {
        double xi, eta;
        face_point(e, m.gq_t[kq], xi, eta);
        T val = u0;
        for (int l = 0; l < nb; ++l) val += abar[l] * psi(m.big, l, xi, eta);
        fp[(e * m.nq + kq) * 4 + v] = val;
      }
  }
  if (!frozen) {
    // non-physical states: cell average or any face point with rho <= 0,
    // p <= 0 or NaN (counted once per cell)
    double u[4];
    for (int c = 0; c < 4; ++c) u[c] = re(U[4 * i + c]);
    bool avg_ok = physical(u, m.prm.gamma);
    bool fp_ok = true;
    for (int q = 0; q < 3 * m.nq && fp_ok; ++q) {
      for (int c = 0; c < 4; ++c) u[c] = re(fp[q * 4 + c]);
      fp_ok = physical(u, m.prm.gamma);
    }
    if (!(avg_ok && fp_ok)) note_bad(dg, i);
    if (!fp_ok && avg_ok && m.prm.fallback) {
      for (int q = 0; q < 3 * m.nq; ++q)
        for (int c = 0; c < 4; ++c) fp[q * 4 + c] = U[4 * i + c];
      out_flags = 0;
      if (dg) dg->fallbacks++;
    }
  }
  flags = out_flags;
  if (ties_out) *ties_out = tie_nib;
}

// +1 when cell i is the L side of the face on its local edge e (the face
// normal points out of i), else -1.
double side_sign(const Mesh& m, int i, int e) {
  const int f = m.cf[3 * i + e];
  double s = (m.fL[f] == i && m.fLe[f] == e) ? 1.0 : -1.0;
  return s;
}

// ---------------------------------------------------------------------------
// Characteristic variables (Sec. 2.3, remark on which variables the
// nonlinear reconstruction acts on).  Reading: on local edge e of cell i the
// variables are w = L U with R = L^-1 the right eigenvectors of the Euler
// flux Jacobian in the direction of the edge's outward unit normal n,
// evaluated at the cell's mean state; a non-physical mean (no real sound
// speed) keeps the conservative variables (L = R = I).  Every face of the
// cell has its own projection, selection and flags.
// ---------------------------------------------------------------------------

// R (row-major, R[4*row + col]); column k is the right eigenvector of speed
// u.n - c, u.n (entropy), u.n (shear), u.n + c.
void char_right(const double* u, double nx, double ny, double g, double* R) {
  const double rho = u[0], vx = u[1] / rho, vy = u[2] / rho;
  const double q2 = vx * vx + vy * vy;
  const double p = (g - 1.0) * (u[3] - 0.5 * rho * q2);
  const double c = std::sqrt(g * p / rho);
  const double H = (u[3] + p) / rho;
  const double un = vx * nx + vy * ny, ut = -vx * ny + vy * nx;
  const double cols[4][4] = {{1.0, vx - c * nx, vy - c * ny, H - c * un},
                             {1.0, vx, vy, 0.5 * q2},
                             {0.0, -ny, nx, ut},
                             {1.0, vx + c * nx, vy + c * ny, H + c * un}};
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 4; ++k) R[4 * r + k] = cols[k][r];
}

// Inverse of a 4x4 matrix by Gauss-Jordan elimination with partial pivoting.
bool invert4(const double* A, double* Ainv) {
  double a[4][8];
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 8; ++k) a[r][k] = k < 4 ? A[4 * r + k] : (k - 4 == r ? 1.0 : 0.0);
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
    if (!(std::fabs(a[piv][col]) > 0.0)) return false;
    if (piv != col)
      for (int k = 0; k < 8; ++k) std::swap(a[piv][k], a[col][k]);
    const double d = a[col][col];
    for (int k = 0; k < 8; ++k) a[col][k] /= d;
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      const double f = a[r][col];
      for (int k = 0; k < 8; ++k) a[r][k] -= f * a[col][k];
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 4; ++k) Ainv[4 * r + k] = a[r][k + 4];
  return true;
}

// L and R of cell state u for direction n; identity when u is not physical.
void char_basis(const double* u, double nx, double ny, double g, double* R, double* L) {
  bool ok = physical(u, g);
  if (ok) {
    char_right(u, nx, ny, g, R);
    ok = invert4(R, L);
  }
  if (!ok)
    for (int t = 0; t < 16; ++t) R[t] = L[t] = (t % 5 == 0) ? 1.0 : 0.0;
}

// Outward unit normal of local edge e of cell i.
void edge_normal(const Mesh& m, int i, int e, double& nx, double& ny) {
  const int f = m.cf[3 * i + e];
  const double s = side_sign(m, i, e);
  nx = s * m.fn[2 * f];
  ny = s * m.fn[2 * f + 1];
}

// Characteristic reconstruction of one cell: fp [3][nq][4], flags3[e] = the
// flags of local edge e (bit 4v+3: large stencil kept for characteristic
// variable v, bits 4v..4v+2: small stencils kept).
void reconstruct_cell_char(const Mesh& m, int i, const double* U, uint16_t* flags3, double* fp,
                           oracle_diag* dg, uint16_t* ties3 = nullptr) {
  const CellData& cd = m.cd[i];
  const int nb = m.big.n(), ns = m.small.n();
  // least-squares coefficients of the conservative variables (linear in
  // the data, so those of w = L U are L times these)
  std::vector<double> coef[4][4];  // [variable][stencil]
  for (int v = 0; v < 4; ++v) lsq_coefficients(cd, U, i, v, coef[v]);
  const double* u0 = &U[4 * i];
  for (int e = 0; e < 3; ++e) {
    double nx, ny, R[16], L[16];
    edge_normal(m, i, e, nx, ny);
    char_basis(u0, nx, ny, m.prm.gamma, R, L);
    uint16_t fe = 0, te = 0;
    std::vector<double> dw[4];  // per characteristic variable: value minus mean at the points
    for (int v = 0; v < 4; ++v) {
      std::vector<double> wc[4];
      double beta[4];
      for (int k = 0; k < 4; ++k) {
        wc[k].assign(coef[0][k].size(), 0.0);
        for (size_t l = 0; l < wc[k].size(); ++l)
          for (int j = 0; j < 4; ++j) wc[k][l] += L[4 * v + j] * coef[j][k][l];
        beta[k] = smoothness(k == 3 ? m.big : m.small, wc[k].data());
      }
      std::vector<double> abar;
      if (m.prm.variant == 2) {
        double w[4], d[4];
        cweno_weights(beta, m.prm, w, d);
        cweno_combine(w, d, wc, nb, ns, abar);
      } else {
        Sel s = select(beta, m.prm);
        if (dg) {
          dg->near_ties += s.ties;
          if (s.flags & 8u) dg->large_kept++;
        }
        if (s.ties) te |= (uint16_t)(0xFu << (4 * v));
        fe |= (uint16_t)(s.flags << (4 * v));
        teno_combine(s.flags, wc, nb, ns, abar);
      }
      dw[v].assign(m.nq, 0.0);
      for (int kq = 0; kq < m.nq; ++kq) {
        double xi, eta;
        face_point(e, m.gq_t[kq], xi, eta);
        for (int l = 0; l < nb; ++l) dw[v][kq] += abar[l] * psi(m.big, l, xi, eta);
      }
    }
    flags3[e] = fe;
    if (ties3) ties3[e] = te;
    // back to conservative variables: U = U_0 + R dw
    for (int kq = 0; kq < m.nq; ++kq)
      for (int c = 0; c < 4; ++c) {
        double val = u0[c];
        for (int v = 0; v < 4; ++v) val += R[4 * c + v] * dw[v][kq];
        fp[(e * m.nq + kq) * 4 + c] = val;
      }
  }
  // non-physical states, as in the conservative reconstruction
  double u[4];
  for (int c = 0; c < 4; ++c) u[c] = u0[c];
  bool avg_ok = physical(u, m.prm.gamma);
  bool fp_ok = true;
  for (int q = 0; q < 3 * m.nq && fp_ok; ++q) {
    for (int c = 0; c < 4; ++c) u[c] = fp[q * 4 + c];
    fp_ok = physical(u, m.prm.gamma);
  }
  if (!(avg_ok && fp_ok)) note_bad(dg, i);
  if (!fp_ok && avg_ok && m.prm.fallback) {
    for (int q = 0; q < 3 * m.nq; ++q)
      for (int c = 0; c < 4; ++c) fp[q * 4 + c] = u0[c];
    flags3[0] = flags3[1] = flags3[2] = 0;
    if (dg) dg->fallbacks++;
  }
}

// ---------------------------------------------------------------------------
// Rotated HLL flux with Einfeldt/Roe wave speeds (Sec. 4).
// ---------------------------------------------------------------------------

template <class T>
T min_re(const T& a, const T& b) { return re(b) < re(a) ? b : a; }
template <class T>
T max_re(const T& a, const T& b) { return re(b) > re(a) ? b : a; }

template <class T>
void hll_flux(const T* uL, const T* uR, double nx, double ny, double g, T* out) {
  // T U: momentum into (normal, tangential) components
  T L[4] = {uL[0], uL[1] * nx + uL[2] * ny, -uL[1] * ny + uL[2] * nx, uL[3]};
  T R[4] = {uR[0], uR[1] * nx + uR[2] * ny, -uR[1] * ny + uR[2] * nx, uR[3]};
  T unL = L[1] / L[0], utL = L[2] / L[0];
  T unR = R[1] / R[0], utR = R[2] / R[0];
  T pL = (g - 1.0) * (L[3] - 0.5 * L[0] * (unL * unL + utL * utL));
  T pR = (g - 1.0) * (R[3] - 0.5 * R[0] * (unR * unR + utR * utR));
  T cL = std::sqrt(g * pL / L[0]);
  T cR = std::sqrt(g * pR / R[0]);
  T HL = (L[3] + pL) / L[0];
  T HR = (R[3] + pR) / R[0];
  T D = std::sqrt(R[0] / L[0]);
  T ut = (unL + D * unR) / (1.0 + D);
  T vt = (utL + D * utR) / (1.0 + D);
  T Ht = (HL + D * HR) / (1.0 + D);
  T ct = std::sqrt((g - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt)));
  T SL = min_re(unL - cL, ut - ct);
  T SR = max_re(unR + cR, ut + ct);
  T FL[4] = {L[1], L[1] * unL + pL, L[1] * utL, unL * (L[3] + pL)};
  T FR[4] = {R[1], R[1] * unR + pR, R[1] * utR, unR * (R[3] + pR)};
  T F[4];
  if (re(SL) >= 0.0) {
    for (int c = 0; c < 4; ++c) F[c] = FL[c];
  } else if (re(SR) <= 0.0) {
    for (int c = 0; c < 4; ++c) F[c] = FR[c];
  } else {
    for (int c = 0; c < 4; ++c)
      F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (R[c] - L[c])) / (SR - SL);
  }
  // T^{-1}
  out[0] = F[0];
  out[1] = F[1] * nx - F[2] * ny;
  out[2] = F[1] * ny + F[2] * nx;
  out[3] = F[3];
}


// ---------------------------------------------------------------------------
// Full residual (Sec. 2.1): R_i = -(1/|V_i|) sum_faces s_if Phi_f
// ---------------------------------------------------------------------------
// Outer state of boundary face b (normal n out of the domain) for the
// Riemann problem at a Gauss point: transmissive copies the inner state,
// reflective mirrors its velocity in the face, prescribed takes the given
// state.
template <class T>
void boundary_state(const Mesh& m, int b, const T* uL, double nx, double ny, T* uR) {
  if (m.bkind[b] == 3) {
    for (int c = 0; c < 4; ++c) uR[c] = T(m.bstate[4 * (size_t)b + c]);
  } else if (m.bkind[b] == 2) {
    // momentum (mn, mt) in the face frame -> (-mn, mt)
    T mn = uL[1] * nx + uL[2] * ny, mt = -uL[1] * ny + uL[2] * nx;
    uR[0] = uL[0];
    uR[1] = -mn * nx - mt * ny;
    uR[2] = -mn * ny + mt * nx;
    uR[3] = uL[3];
  } else {
    for (int c = 0; c < 4; ++c) uR[c] = uL[c];
  }
}

template <class T>
void face_flux(const Mesh& m, int f, const T* fp, T* phi) {
  const int nq = m.nq;
  int L = m.fL[f], R = m.fR[f], eL = m.fLe[f], eR = m.fRe[f];
  for (int c = 0; c < 4; ++c) phi[c] = T(0.0);
  for (int k = 0; k < nq; ++k) {
    const T* uL = &fp[((size_t)L * 3 * nq + eL * nq + k) * 4];
    T ub[4];
    const T* uR = ub;
    if (R >= 0)
      uR = &fp[((size_t)R * 3 * nq + eR * nq + (nq - 1 - k)) * 4];
    else
      boundary_state(m, m.bidx[f], uL, m.fn[2 * f], m.fn[2 * f + 1], ub);
    T F[4];
    hll_flux(uL, uR, m.fn[2 * f], m.fn[2 * f + 1], m.prm.gamma, F);
    for (int c = 0; c < 4; ++c) phi[c] += m.gq_w[k] * F[c];
  }
  for (int c = 0; c < 4; ++c) phi[c] *= m.flen[f];
}

template <class T>
void assemble(const Mesh& m, const std::vector<T>& phi, int i, T* Ri) {
  T acc[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int e = 0; e < 3; ++e) {
    int f = m.cf[3 * i + e];
    double s = side_sign(m, i, e);
    for (int c = 0; c < 4; ++c) acc[c] += s * phi[4 * (size_t)f + c];
  }
  for (int c = 0; c < 4; ++c) Ri[c] = -acc[c] / m.area[i];
}

template <class T>
void residual_full(const Mesh& m, const T* U, T* R, uint16_t* flags, bool frozen,
                   double* fp_out, oracle_diag* dg, uint16_t* ties = nullptr) {
  const int nq = m.nq;
  const bool chr = m.prm.characteristic != 0;  // flags per local edge, never frozen
  std::vector<T> fp((size_t)m.nc * 3 * nq * 4);
  std::vector<uint16_t> fl((size_t)m.nc * (chr ? 3 : 1), 0);
  std::vector<uint16_t> tl(fl.size(), 0);
  if (frozen) for (int i = 0; i < m.nc; ++i) fl[i] = flags[i];
  int64_t nt = 0, lk = 0, fb = 0, nbad = 0, first = m.nc;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nt, lk, fb, nbad) reduction(min : first)
  for (int i = 0; i < m.nc; ++i) {
    oracle_diag local{0, -1, 0, 0, 0};
    if constexpr (std::is_same<T, double>::value) {
      if (chr)
        reconstruct_cell_char(m, i, U, &fl[3 * (size_t)i], &fp[(size_t)i * 3 * nq * 4], &local,
                              &tl[3 * (size_t)i]);
      else
        reconstruct_cell(m, i, U, frozen, fl[i], &fp[(size_t)i * 3 * nq * 4], nullptr, &local,
                         &tl[i]);
    } else {
      reconstruct_cell(m, i, U, frozen, fl[i], &fp[(size_t)i * 3 * nq * 4], nullptr, &local);
    }
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
  if (fp_out)
    for (size_t t = 0; t < fp.size(); ++t) fp_out[t] = re(fp[t]);
  std::vector<T> phi((size_t)m.nf * 4);
#pragma omp parallel for schedule(static)
  for (int f = 0; f < m.nf; ++f) face_flux(m, f, fp.data(), &phi[4 * (size_t)f]);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < m.nc; ++i) assemble(m, phi, i, &R[4 * (size_t)i]);
  if (flags && !frozen) {
    if (chr) {
      for (int e = 0; e < 3; ++e)
        for (int i = 0; i < m.nc; ++i) flags[(size_t)e * m.nc + i] = fl[3 * (size_t)i + e];
    } else {
      for (int i = 0; i < m.nc; ++i) flags[i] = fl[i];
    }
  }
  if (ties) {
    if (chr) {
      for (int e = 0; e < 3; ++e)
        for (int i = 0; i < m.nc; ++i) ties[(size_t)e * m.nc + i] = tl[3 * (size_t)i + e];
    } else {
      for (int i = 0; i < m.nc; ++i) ties[i] = tl[i];
    }
  }
}

bool ready(const Mesh& m) {
  if (!m.have_params) { g_err = "oracle_setup not called"; return false; }
  return true;
}

}  // namespace

// ===========================================================================
// C interface (host pointers, user cell order)
// ===========================================================================
extern "C" {

const char* oracle_last_error(void) { return g_err.c_str(); }

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_default_params(oracle_params* p) {
  p->order = 5;
  p->nq = 0;
  p->variant = 0;
  p->power = 6;
  p->ct = 1e-6;
  p->eps = 1e-12;
  p->gamma = 1.4;
  p->tie_rel = 1e-10;
  p->fallback = 0;
  p->characteristic = 0;
  p->dk_prime = 1e4;
}

// Geometry and faces (Sec. 2.1).  period: per axis, 0 = open axis; NULL =
// both open.  Edges with one cell are boundary faces, allowed when an axis
// is open.
void* oracle_mesh_create(int nv, const double* xy, int nc, const int* tri, const double* period) {
  if (nv <= 0 || nc <= 0 || !xy || !tri) { fail("empty mesh"); return nullptr; }
  Mesh* m = new Mesh();
  m->nv = nv;
  m->nc = nc;
  m->xy.assign(xy, xy + 2 * (size_t)nv);
  m->tri.assign(tri, tri + 3 * (size_t)nc);
  if (period) {
    m->P[0] = period[0] > 0.0 ? period[0] : 0.0;
    m->P[1] = period[1] > 0.0 ? period[1] : 0.0;
  }
  m->periodic = m->P[0] > 0.0 && m->P[1] > 0.0;
  m->X.assign((size_t)nc * 6, 0.0);
  m->area.assign(nc, 0.0);
  m->cen.assign(2 * (size_t)nc, 0.0);
  for (int i = 0; i < nc; ++i) {
    int* t = &m->tri[3 * (size_t)i];
    for (int v = 0; v < 3; ++v)
      if (t[v] < 0 || t[v] >= nv) { fail("vertex index out of range"); delete m; return nullptr; }
    double p[3][2];
    for (int v = 0; v < 3; ++v) {
      p[v][0] = xy[2 * t[v]];
      p[v][1] = xy[2 * t[v] + 1];
    }
    for (int v = 1; v < 3; ++v) {
      double dx = p[v][0] - p[0][0], dy = p[v][1] - p[0][1];
      double ddx = dx, ddy = dy;
      min_image(*m, ddx, ddy);
      p[v][0] = p[0][0] + ddx;
      p[v][1] = p[0][1] + ddy;
    }
    double a2 = (p[1][0] - p[0][0]) * (p[2][1] - p[0][1]) - (p[2][0] - p[0][0]) * (p[1][1] - p[0][1]);
    if (a2 < 0.0) {
      std::swap(t[1], t[2]);
      std::swap(p[1][0], p[2][0]);
      std::swap(p[1][1], p[2][1]);
      a2 = -a2;
    }
    if (!(a2 > 0.0)) { fail("degenerate triangle " + std::to_string(i)); delete m; return nullptr; }
    m->area[i] = 0.5 * a2;
    for (int v = 0; v < 3; ++v) {
      m->X[(size_t)i * 6 + 2 * v] = p[v][0];
      m->X[(size_t)i * 6 + 2 * v + 1] = p[v][1];
    }
    m->cen[2 * i] = (p[0][0] + p[1][0] + p[2][0]) / 3.0;
    m->cen[2 * i + 1] = (p[0][1] + p[1][1] + p[2][1]) / 3.0;
  }
  // faces: each undirected edge once; L = lower cell id of the two
  std::vector<std::pair<std::pair<int, int>, int>> he;  // ((a,b), 3*cell+e)
  he.reserve(3 * (size_t)nc);
  for (int i = 0; i < nc; ++i)
    for (int e = 0; e < 3; ++e) {
      int a = m->tri[3 * i + e], b = m->tri[3 * i + (e + 1) % 3];
      he.push_back({{a, b}, 3 * i + e});
    }
  std::sort(he.begin(), he.end());
  for (size_t t = 1; t < he.size(); ++t)
    if (he[t].first == he[t - 1].first) { fail("non-manifold edge"); delete m; return nullptr; }
  m->cf.assign(3 * (size_t)nc, -1);
  for (size_t t = 0; t < he.size(); ++t) {
    int a = he[t].first.first, b = he[t].first.second;
    int ci = he[t].second / 3, ce = he[t].second % 3;
    auto it = std::lower_bound(he.begin(), he.end(), std::make_pair(std::make_pair(b, a), -1));
    if (it == he.end() || it->first != std::make_pair(b, a)) {
      if (m->periodic) {
        fail("open edge on a mesh periodic in both axes");
        delete m;
        return nullptr;
      }
      // boundary face: the cell's edge, normal pointing out of the domain
      int f = m->nf++;
      m->fL.push_back(ci);
      m->fLe.push_back(ce);
      m->fR.push_back(-1);
      m->fRe.push_back(-1);
      const double* X = &m->X[(size_t)ci * 6];
      double ex = X[2 * ((ce + 1) % 3)] - X[2 * ce];
      double ey = X[2 * ((ce + 1) % 3) + 1] - X[2 * ce + 1];
      double len = std::sqrt(ex * ex + ey * ey);
      m->flen.push_back(len);
      m->fn.push_back(ey / len);
      m->fn.push_back(-ex / len);
      m->cf[3 * ci + ce] = f;
      m->bface.push_back(f);
      continue;
    }
    int cj = it->second / 3, cje = it->second % 3;
    if (ci > cj || (ci == cj && ce > cje)) continue;  // the other half creates it
    int f = m->nf++;
    m->fL.push_back(ci);
    m->fLe.push_back(ce);
    m->fR.push_back(cj);
    m->fRe.push_back(cje);
    const double* X = &m->X[(size_t)ci * 6];
    double ex = X[2 * ((ce + 1) % 3)] - X[2 * ce];
    double ey = X[2 * ((ce + 1) % 3) + 1] - X[2 * ce + 1];
    double len = std::sqrt(ex * ex + ey * ey);
    m->flen.push_back(len);
    m->fn.push_back(ey / len);
    m->fn.push_back(-ex / len);
    m->cf[3 * ci + ce] = f;
    m->cf[3 * cj + cje] = f;
  }
  m->bidx.assign(m->nf, -1);
  for (size_t b = 0; b < m->bface.size(); ++b) m->bidx[m->bface[b]] = (int)b;
  m->bkind.assign(m->bface.size(), 1);
  m->bstate.assign(4 * m->bface.size(), 0.0);
  return m;
}

int oracle_boundary_count(void* h) { return (int)((Mesh*)h)->bface.size(); }

// verts [nb][2] (user vertex ids, counter-clockwise in the cell), cell [nb]
int oracle_boundary_faces(void* h, int* verts, int* cell) {
  Mesh* m = (Mesh*)h;
  for (size_t b = 0; b < m->bface.size(); ++b) {
    int f = m->bface[b], i = m->fL[f], e = m->fLe[f];
    verts[2 * b] = m->tri[3 * i + e];
    verts[2 * b + 1] = m->tri[3 * i + (e + 1) % 3];
    if (cell) cell[b] = i;
  }
  return 0;
}

// kind [nb] (1 transmissive, 2 reflective, 3 prescribed), state [nb][4]
int oracle_set_boundary(void* h, const int* kind, const double* state) {
  Mesh* m = (Mesh*)h;
  for (size_t b = 0; b < m->bface.size(); ++b) {
    if (kind[b] < 1 || kind[b] > 3) return fail("boundary kind must be 1, 2 or 3");
    m->bkind[b] = kind[b];
    for (int c = 0; c < 4; ++c) m->bstate[4 * b + c] = state ? state[4 * b + c] : 0.0;
  }
  return 0;
}

void oracle_mesh_destroy(void* h) { delete (Mesh*)h; }

int oracle_mesh_counts(void* h, int* nc, int* nf) {
  Mesh* m = (Mesh*)h;
  *nc = m->nc;
  *nf = m->nf;
  return 0;
}

// area[nc], centroid[nc][2], tri_ccw[nc][3]
int oracle_mesh_geometry(void* h, double* area, double* cen, int* tri_ccw) {
  Mesh* m = (Mesh*)h;
  if (area) std::memcpy(area, m->area.data(), sizeof(double) * m->nc);
  if (cen) std::memcpy(cen, m->cen.data(), sizeof(double) * 2 * m->nc);
  if (tri_ccw) std::memcpy(tri_ccw, m->tri.data(), sizeof(int) * 3 * m->nc);
  return 0;
}

// fL, fR, fLe, fRe [nf]; normal [nf][2]; length [nf]; cell_face [nc][3]
int oracle_mesh_faces(void* h, int* fL, int* fR, int* fLe, int* fRe, double* n, double* len, int* cf) {
  Mesh* m = (Mesh*)h;
  size_t nf = m->nf;
  if (fL) std::memcpy(fL, m->fL.data(), sizeof(int) * nf);
  if (fR) std::memcpy(fR, m->fR.data(), sizeof(int) * nf);
  if (fLe) std::memcpy(fLe, m->fLe.data(), sizeof(int) * nf);
  if (fRe) std::memcpy(fRe, m->fRe.data(), sizeof(int) * nf);
  if (n) std::memcpy(n, m->fn.data(), sizeof(double) * 2 * nf);
  if (len) std::memcpy(len, m->flen.data(), sizeof(double) * nf);
  if (cf) std::memcpy(cf, m->cf.data(), sizeof(int) * 3 * m->nc);
  return 0;
}

// Parameters; optionally builds reconstruction data for every cell (all=1).
int oracle_setup(void* h, const oracle_params* p, int all) {
  Mesh* m = (Mesh*)h;
  if (p->order < 3 || p->order > 6) return fail("order must be 3..6");
  if (p->variant < 0 || p->variant > 2) return fail("variant must be 0, 1 or 2");
  if (p->variant == 2 && !(p->dk_prime > 1.0)) return fail("CWENO needs dk_prime > 1");
  if (p->characteristic != 0 && p->characteristic != 1) return fail("characteristic must be 0 or 1");
  if (p->ct < 0.0 || p->ct > 1.0 / 3.0) return fail("C_T must lie in [0, 1/K]");
  m->prm = *p;
  m->nq = p->nq > 0 ? p->nq : (p->order + 1) / 2;
  m->big = make_basis(p->order - 1);
  m->small = make_basis(2);
  gauss01(m->nq, m->gq_t, m->gq_w);
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
          if (bad < 0 || i < bad) { bad = i; err = e; }
        }
      }
    }
    if (bad >= 0) return fail(err);
  }
  return 0;
}

// Builds reconstruction data for the listed cells (and nothing else).
int oracle_prepare_cells(void* h, int n, const int* cells) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  std::vector<int> list;
  for (int t = 0; t < n; ++t) {
    if (cells[t] < 0 || cells[t] >= m->nc) return fail("cell index out of range");
    list.push_back(cells[t]);
  }
  std::sort(list.begin(), list.end());
  list.erase(std::unique(list.begin(), list.end()), list.end());
  int bad = -1;
  std::string err;
#pragma omp parallel for schedule(dynamic, 16)
  for (int t = 0; t < (int)list.size(); ++t) {
    std::string e;
    int i = list[t];
    if (!build_cell(*m, i, e)) {
#pragma omp critical
      { if (bad < 0) { bad = i; err = e; } }
    }
  }
  if (bad >= 0) return fail(err);
  return 0;
}

// Members of stencil k of cell i (nearest first, target excluded).
int oracle_stencil(void* h, int i, int k, int* out, int brute) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  int want = stencil_rows(k == 3 ? m->big.r : 2);
  std::vector<int> v;
  bool ok = brute ? stencil_brute(*m, i, k, want, v) : stencil_search(*m, i, k, want, v);
  if (!ok) return fail("too few stencil candidates");
  std::copy(v.begin(), v.end(), out);
  return want;
}

// Least-squares operator of stencil k of cell i as an explicit matrix:
// coef = Mop * (U_s - U_0), Mop [n_coef][rows] row-major.  Also cond estimate.
int oracle_lsq_operator(void* h, int i, int k, double* Mop, double* rcond) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  std::string err;
  if (!build_cell(*m, i, err)) return fail(err);
  const Stencil& S = m->cd[i].st[k];
  std::vector<double> b(S.qr.m), x(S.qr.n);
  for (int s = 0; s < S.qr.m; ++s) {
    std::fill(b.begin(), b.end(), 0.0);
    b[s] = S.vol[s];
    qr_solve(S.qr, b.data(), x.data());
    for (int l = 0; l < S.qr.n; ++l) Mop[(size_t)l * S.qr.m + s] = x[l];
  }
  if (rcond) *rcond = S.qr.rmin / S.qr.rmax;
  return S.qr.m;
}

// Raw least-squares helpers for pinning: solve min |A x - b| (A column-major).
int oracle_lsq_solve(int m_, int n_, const double* A, const double* b, double* x) {
  QR q;
  q.m = m_;
  q.n = n_;
  q.a.assign(A, A + (size_t)m_ * n_);
  if (!qr_factor(q)) return fail("rank deficient");
  qr_solve(q, b, x);
  return 0;
}

// Gauss-Legendre nodes/weights on [0,1].
int oracle_gauss01(int n, double* t, double* w) {
  std::vector<double> tt, ww;
  gauss01(n, tt, ww);
  std::copy(tt.begin(), tt.end(), t);
  std::copy(ww.begin(), ww.end(), w);
  return 0;
}

// int over T_ref of xi^a eta^b by the oracle's collapsed rule (n x n points).
double oracle_tref_moment(int a, int b, int n) {
  TriRule q = tri_rule(n);
  double acc = 0.0;
  for (size_t t = 0; t < q.w.size(); ++t) {
    double xi = q.u[t] - q.u[t] * q.s[t];
    double eta = q.u[t] * q.s[t];
    acc += q.w[t] * ipow(xi, a) * ipow(eta, b);
  }
  return acc;
}

// Integral of xi^a eta^b over an arbitrary triangle q[3][2] (collapsed rule).
double oracle_tri_moment(const double* q, int a, int b, int n) {
  TriRule r = tri_rule(n);
  double a2 = std::fabs((q[2] - q[0]) * (q[5] - q[3]) - (q[3] - q[1]) * (q[4] - q[2]));
  double acc = 0.0;
  for (size_t t = 0; t < r.w.size(); ++t) {
    double u = r.u[t], w = r.s[t];
    double xi = q[0] + u * (q[2] - q[0]) + u * w * (q[4] - q[2]);
    double eta = q[1] + u * (q[3] - q[1]) + u * w * (q[5] - q[3]);
    acc += r.w[t] * ipow(xi, a) * ipow(eta, b);
  }
  return acc * a2;
}

// Smoothness indicator of the polynomial sum_l a_l psi_l of degree r.
double oracle_smoothness(int r, const double* a) {
  Basis B = make_basis(r);
  return smoothness(B, a);
}

// Number of basis functions of degree r and their exponents.
int oracle_basis(int r, int* ea, int* eb, double* mean) {
  Basis B = make_basis(r);
  for (int l = 0; l < B.n(); ++l) {
    if (ea) ea[l] = B.ea[l];
    if (eb) eb[l] = B.eb[l];
    if (mean) mean[l] = B.mean[l];
  }
  return B.n();
}

// Selection of one variable from four smoothness indicators.
int oracle_select(const oracle_params* p, const double* beta, double* chi_out, int* ties) {
  Sel s = select(beta, *p);
  if (chi_out) {
    chi_out[0] = s.chi_small[0];
    chi_out[1] = s.chi_small[1];
    chi_out[2] = s.chi_small[2];
    chi_out[3] = s.chiK;
  }
  if (ties) *ties = s.ties;
  return (int)s.flags;
}

// CWENO weights of one (cell, variable) from its four smoothness indicators
// (Sec. 2.4); omega [4], d [4] (linear weights).
void oracle_cweno_weights(const oracle_params* p, const double* beta, double* omega, double* d) {
  cweno_weights(beta, *p, omega, d);
}

// HLL flux through unit normal n (Sec. 4).
// Right and left eigenvectors (row-major 4x4) of the flux Jacobian in the
// direction (nx, ny) at state u; identity for a non-physical state.
void oracle_char_basis(const double* u, double nx, double ny, double g, double* R, double* L) {
  char_basis(u, nx, ny, g, R, L);
}

void oracle_hll(const double* uL, const double* uR, double nx, double ny, double g, double* out) {
  hll_flux(uL, uR, nx, ny, g, out);
}

// Reconstructed face-point states of listed cells: fp [n][3][nq][4],
// flags [n] ([n][3], one per local edge, in characteristic variables), beta
// [n][4 vars][4 stencils] (nullable; conservative variables only).  ties
// (nullable, laid out like flags): nibble v is 0xF where the selection of
// variable v met a near tie (Sec. 3.3 cutoff; |chi/C_T - 1| <= tie_rel for
// one of its chi), else 0.
int oracle_reconstruct_cells(void* h, const double* U, int n, const int* cells, double* fp,
                             uint16_t* flags, double* beta, oracle_diag* dg, uint16_t* ties) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (oracle_prepare_cells(h, n, cells) != 0) return -1;
  const int nq = m->nq;
  int64_t nt = 0, lk = 0, fb = 0, nbad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nt, lk, fb, nbad)
  for (int t = 0; t < n; ++t) {
    oracle_diag local{0, -1, 0, 0, 0};
    if (m->prm.characteristic) {
      uint16_t fl3[3] = {0, 0, 0}, tl3[3] = {0, 0, 0};
      reconstruct_cell_char(*m, cells[t], U, fl3, &fp[(size_t)t * 3 * nq * 4], &local, tl3);
      for (int e = 0; e < 3; ++e) {
        if (flags) flags[3 * (size_t)t + e] = fl3[e];
        if (ties) ties[3 * (size_t)t + e] = tl3[e];
      }
    } else {
      uint16_t fl = 0, tl = 0;
      reconstruct_cell(*m, cells[t], U, false, fl, &fp[(size_t)t * 3 * nq * 4],
                       beta ? &beta[(size_t)t * 16] : nullptr, &local, &tl);
      if (flags) flags[t] = fl;
      if (ties) ties[t] = tl;
    }
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

// Full residual R[nc][4]; flags[nc] out (or in when frozen=1; in
// characteristic variables [3][nc], one per local edge, out only); fp_out
// [nc][3][nq][4] nullable; diag nullable; ties nullable, laid out like
// flags, the near-tie nibbles of each cell (all 0 when frozen).
int oracle_residual(void* h, const double* U, double* R, uint16_t* flags, int frozen,
                    double* fp_out, oracle_diag* dg, uint16_t* ties) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (frozen && !flags) return fail("frozen selection needs flags");
  if (frozen && m->prm.characteristic) return fail("no frozen selection in characteristic variables");
  for (int i = 0; i < m->nc; ++i)
    if (!m->cd[i].built) return fail("oracle_setup(all=1) required for the full residual");
  residual_full(*m, U, R, flags, frozen != 0, fp_out, dg, frozen ? nullptr : ties);
  if (frozen && ties) std::fill(ties, ties + m->nc, (uint16_t)0);
  return 0;
}

// Residual of the listed cells only: R_out [n][4]; builds what it needs.
int oracle_residual_cells(void* h, const double* U, int n, const int* cells, double* R_out,
                          uint16_t* flags_out) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  const int nq = m->nq;
  // cells whose reconstruction is needed: the listed ones and their neighbours
  std::vector<int> need;
  for (int t = 0; t < n; ++t) {
    int i = cells[t];
    need.push_back(i);
    for (int e = 0; e < 3; ++e) {
      int f = m->cf[3 * i + e];
      int other = m->fL[f] == i && m->fLe[f] == e ? m->fR[f] : m->fL[f];
      if (other >= 0) need.push_back(other);
    }
  }
  std::sort(need.begin(), need.end());
  need.erase(std::unique(need.begin(), need.end()), need.end());
  if (oracle_prepare_cells(h, (int)need.size(), need.data()) != 0) return -1;
  const int fw = m->prm.characteristic ? 3 : 1;
  std::vector<double> fpn(need.size() * 3 * nq * 4);
  std::vector<uint16_t> fln(need.size() * fw, 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (size_t t = 0; t < need.size(); ++t) {
    if (fw == 3)
      reconstruct_cell_char(*m, need[t], U, &fln[3 * t], &fpn[t * 3 * nq * 4], nullptr);
    else
      reconstruct_cell(*m, need[t], U, false, fln[t], &fpn[t * 3 * nq * 4], nullptr, nullptr);
  }
  auto slot = [&](int c) {
    return (size_t)(std::lower_bound(need.begin(), need.end(), c) - need.begin());
  };
  for (int t = 0; t < n; ++t) {
    int i = cells[t];
    double acc[4] = {0, 0, 0, 0};
    for (int e = 0; e < 3; ++e) {
      int f = m->cf[3 * i + e];
      int L = m->fL[f], R = m->fR[f], eL = m->fLe[f], eR = m->fRe[f];
      size_t sL = slot(L), sR = R >= 0 ? slot(R) : 0;
      double phi[4] = {0, 0, 0, 0};
      for (int k = 0; k < nq; ++k) {
        const double* uL = &fpn[(sL * 3 * nq + eL * nq + k) * 4];
        double ub[4];
        const double* uR = ub;
        if (R >= 0)
          uR = &fpn[(sR * 3 * nq + eR * nq + (nq - 1 - k)) * 4];
        else
          boundary_state(*m, m->bidx[f], uL, m->fn[2 * f], m->fn[2 * f + 1], ub);
        double F[4];
        hll_flux(uL, uR, m->fn[2 * f], m->fn[2 * f + 1], m->prm.gamma, F);
        for (int c = 0; c < 4; ++c) phi[c] += m->gq_w[k] * F[c];
      }
      double s = (L == i && eL == e) ? 1.0 : -1.0;
      for (int c = 0; c < 4; ++c) acc[c] += s * (phi[c] * m->flen[f]);
    }
    for (int c = 0; c < 4; ++c) R_out[4 * (size_t)t + c] = -acc[c] / m->area[i];
    if (flags_out)
      for (int w = 0; w < fw; ++w) flags_out[(size_t)t * fw + w] = fln[slot(i) * fw + w];
  }
  return 0;
}

// Time step (reading): dt = cfl * min_i |V_i| / sum_j |A_ij| (|u.n| + c).
double oracle_dt(void* h, const double* U, double cfl) {
  Mesh* m = (Mesh*)h;
  double g = m->have_params ? m->prm.gamma : 1.4;
  double best = INFINITY;
  for (int i = 0; i < m->nc; ++i) {
    const double* u = &U[4 * (size_t)i];
    double vx = u[1] / u[0], vy = u[2] / u[0];
    double p = (g - 1.0) * (u[3] - 0.5 * u[0] * (vx * vx + vy * vy));
    double c = std::sqrt(g * p / u[0]);
    double den = 0.0;
    for (int e = 0; e < 3; ++e) {
      int f = m->cf[3 * i + e];
      double un = vx * m->fn[2 * f] + vy * m->fn[2 * f + 1];
      den += m->flen[f] * (std::fabs(un) + c);
    }
    double lim = m->area[i] / den;
    if (lim < best) best = lim;
  }
  return cfl * best;
}

// One SSP-RK3 step (Sec. 2.1, time discretisation); flags3 [3][nc] nullable
// (out, or in when frozen=1; [3][3][nc] out in characteristic variables);
// stages [3][nc][4] nullable (stage inputs); ties3 nullable, laid out like
// flags3, the near-tie nibbles of each stage.
int oracle_rk_step(void* h, const double* U, double* Uout, double dt, uint16_t* flags3,
                   int frozen, double* stages, oracle_diag* dg, uint16_t* ties3) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  const size_t n4 = 4 * (size_t)m->nc;
  std::vector<double> R(n4), U1(n4), U2(n4);
  const size_t nfl = (size_t)m->nc * (m->prm.characteristic ? 3 : 1);
  std::vector<uint16_t> fl(nfl);
  auto stage_flags = [&](int s) -> uint16_t* {
    if (frozen) {
      std::copy(flags3 + (size_t)s * nfl, flags3 + (size_t)(s + 1) * nfl, fl.begin());
    }
    return fl.data();
  };
  auto keep = [&](int s) {
    if (flags3 && !frozen) std::copy(fl.begin(), fl.end(), flags3 + (size_t)s * nfl);
  };
  auto tie = [&](int s) -> uint16_t* { return ties3 ? ties3 + (size_t)s * nfl : nullptr; };
  if (stages) std::copy(U, U + n4, stages);
  if (oracle_residual(h, U, R.data(), stage_flags(0), frozen, nullptr, dg, tie(0))) return -1;
  keep(0);
  for (size_t t = 0; t < n4; ++t) U1[t] = U[t] + dt * R[t];
  if (stages) std::copy(U1.begin(), U1.end(), stages + n4);
  if (oracle_residual(h, U1.data(), R.data(), stage_flags(1), frozen, nullptr, dg, tie(1))) return -1;
  keep(1);
  for (size_t t = 0; t < n4; ++t) U2[t] = 0.75 * U[t] + 0.25 * U1[t] + 0.25 * (dt * R[t]);
  if (stages) std::copy(U2.begin(), U2.end(), stages + 2 * n4);
  if (oracle_residual(h, U2.data(), R.data(), stage_flags(2), frozen, nullptr, dg, tie(2))) return -1;
  keep(2);
  const double a = 1.0 / 3.0, b = 2.0 / 3.0;
  for (size_t t = 0; t < n4; ++t) Uout[t] = a * U[t] + b * U2[t] + b * (dt * R[t]);
  return 0;
}

// Jacobian-vector product of the residual with the selection frozen, by
// complex step: Jv = Im R(U + i h v) / h.
int oracle_jvp(void* h, const double* U, const uint16_t* flags, const double* v, double* Jv) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (m->prm.variant == 2) return fail("CWENO has no frozen selection: no adjoint");
  if (m->prm.characteristic) return fail("no adjoint in characteristic variables");
  const size_t n4 = 4 * (size_t)m->nc;
  const double hh = 1e-30;
  std::vector<cplx> Uc(n4), Rc(n4);
  for (size_t t = 0; t < n4; ++t) Uc[t] = cplx(U[t], hh * v[t]);
  std::vector<uint16_t> fl(flags, flags + m->nc);
  residual_full(*m, Uc.data(), Rc.data(), fl.data(), true, nullptr, nullptr);
  for (size_t t = 0; t < n4; ++t) Jv[t] = Rc[t].imag() / hh;
  return 0;
}

// Vector-Jacobian product (J^T lam) of the residual with frozen selection.
int oracle_vjp(void* h, const double* U, const uint16_t* flags, const double* lam, double* Ubar) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (m->prm.variant == 2) return fail("CWENO has no frozen selection: no adjoint");
  if (m->prm.characteristic) return fail("no adjoint in characteristic variables");
  const int nq = m->nq, nc = m->nc;
  const size_t n4 = 4 * (size_t)nc;
  // forward face points with the frozen selection
  std::vector<double> fp((size_t)nc * 3 * nq * 4);
  std::vector<uint16_t> fl(flags, flags + nc);
  for (int i = 0; i < nc; ++i)
    reconstruct_cell(*m, i, U, true, fl[i], &fp[(size_t)i * 3 * nq * 4], nullptr, nullptr);
  // gather transposed: Phi_f gets lam_R/|V_R| - lam_L/|V_L| (only the inner
  // cell's term on a boundary face)
  std::vector<double> fpbar(fp.size(), 0.0);
  const double hh = 1e-30;
  for (int f = 0; f < m->nf; ++f) {
    int L = m->fL[f], R = m->fR[f], eL = m->fLe[f], eR = m->fRe[f];
    const bool bnd = R < 0;
    double pb[4];
    if (!bnd)
      for (int c = 0; c < 4; ++c) pb[c] = lam[4 * (size_t)R + c] / m->area[R] - lam[4 * (size_t)L + c] / m->area[L];
    else
      for (int c = 0; c < 4; ++c) pb[c] = -lam[4 * (size_t)L + c] / m->area[L];
    for (int k = 0; k < nq; ++k) {
      size_t oL = ((size_t)L * 3 * nq + eL * nq + k) * 4;
      size_t oR = bnd ? 0 : ((size_t)R * 3 * nq + eR * nq + (nq - 1 - k)) * 4;
      double sc = m->flen[f] * m->gq_w[k];
      for (int side = 0; side < (bnd ? 1 : 2); ++side)
        for (int c = 0; c < 4; ++c) {
          cplx a[4], b[4], F[4];
          for (int t = 0; t < 4; ++t) {
            a[t] = cplx(fp[oL + t], 0.0);
            b[t] = cplx(bnd ? 0.0 : fp[oR + t], 0.0);
          }
          if (side == 0) a[c] += cplx(0.0, hh);
          else b[c] += cplx(0.0, hh);
          // the outer state of a boundary face follows the (perturbed) inner one
          if (bnd) boundary_state(*m, m->bidx[f], a, m->fn[2 * f], m->fn[2 * f + 1], b);
          hll_flux(a, b, m->fn[2 * f], m->fn[2 * f + 1], m->prm.gamma, F);
          double acc = 0.0;
          for (int t = 0; t < 4; ++t) acc += pb[t] * (F[t].imag() / hh);
          fpbar[(side == 0 ? oL : oR) + c] += sc * acc;
        }
    }
  }
  // reconstruction transposed
  std::fill(Ubar, Ubar + n4, 0.0);
  const int nb = m->big.n(), ns = m->small.n();
  for (int i = 0; i < nc; ++i) {
    const CellData& cd = m->cd[i];
    for (int v = 0; v < 4; ++v) {
      unsigned f4 = (flags[i] >> (4 * v)) & 0xFu;
      std::vector<double> abar(nb, 0.0);
      double ub = 0.0;
      for (int e = 0; e < 3; ++e)
        for (int kq = 0; kq < nq; ++kq) {
          double g = fpbar[((size_t)i * 3 * nq + e * nq + kq) * 4 + v];
          double xi, eta;
          face_point(e, m->gq_t[kq], xi, eta);
          ub += g;
          for (int l = 0; l < nb; ++l) abar[l] += g * psi(m->big, l, xi, eta);
        }
      Ubar[4 * (size_t)i + v] += ub;
      for (int k = 0; k < 4; ++k) {
        std::vector<double> cb;
        if (k == 3) {
          if (!(f4 & 8u)) continue;
          cb = abar;
        } else {
          if ((f4 & 8u) || !(f4 & (1u << k))) continue;
          int cnt = (int)((f4 & 1u) + ((f4 >> 1) & 1u) + ((f4 >> 2) & 1u));
          cb.assign(ns, 0.0);
          for (int l = 0; l < ns; ++l) cb[l] = abar[l] / (double)cnt;
        }
        const Stencil& S = cd.st[k];
        std::vector<double> bb(S.qr.m);
        qr_solve_transpose(S.qr, cb.data(), bb.data());
        for (int s = 0; s < S.qr.m; ++s) {
          double d = S.vol[s] * bb[s];
          Ubar[4 * (size_t)S.cells[s] + v] += d;
          Ubar[4 * (size_t)i + v] -= d;
        }
      }
    }
  }
  return 0;
}

// Comparison scale of the residual's adjoint (test infrastructure: it sets
// the tolerance of parity tests, it is not part of the method).  S[i][v] is
// the sum of the magnitudes of every term the adjoint adds into U_bar[i][v],
// each term bounded through its own factors: at a face point,
// |A| w_k sum_t |Phi_bar_t| |dF_t/du_c| (the flux derivative by complex
// step, exact); for a stencil row s, |V'_s| sum_l |pinv(A)_ls| |abar_l|, with
// abar_l = sum over the face points of |psi_l| times the face-point term.  A
// sum of these terms formed in any order, from factors that carry a few
// rounding errors each, is exact to a small multiple of the unit roundoff
// times S, which is what the GPU adjoint is held to.
int oracle_vjp_scale(void* h, const double* U, const uint16_t* flags, const double* lam, double* S) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  if (m->prm.variant == 2) return fail("CWENO has no frozen selection: no adjoint");
  if (m->prm.characteristic) return fail("no adjoint in characteristic variables");
  const int nq = m->nq, nc = m->nc;
  std::vector<double> fp((size_t)nc * 3 * nq * 4);
  for (int i = 0; i < nc; ++i) {
    uint16_t fi = flags[i];
    reconstruct_cell(*m, i, U, true, fi, &fp[(size_t)i * 3 * nq * 4], nullptr, nullptr);
  }
  std::vector<double> gabs(fp.size(), 0.0);
  const double step = 1e-30;
  for (int f = 0; f < m->nf; ++f) {
    const int cl = m->fL[f], cr = m->fR[f];
    const bool open_face = cr < 0;
    double w[4];
    for (int c = 0; c < 4; ++c) {
      w[c] = std::fabs(lam[4 * (size_t)cl + c]) / m->area[cl];
      if (!open_face) w[c] += std::fabs(lam[4 * (size_t)cr + c]) / m->area[cr];
    }
    for (int k = 0; k < nq; ++k) {
      const size_t pl = ((size_t)cl * 3 * nq + m->fLe[f] * nq + k) * 4;
      const size_t pr = open_face ? 0 : ((size_t)cr * 3 * nq + m->fRe[f] * nq + (nq - 1 - k)) * 4;
      const double wk = m->flen[f] * m->gq_w[k];
      for (int side = 0; side < (open_face ? 1 : 2); ++side)
        for (int c = 0; c < 4; ++c) {
          cplx ul[4], ur[4], F[4];
          for (int t = 0; t < 4; ++t) {
            ul[t] = cplx(fp[pl + t], side == 0 && t == c ? step : 0.0);
            ur[t] = cplx(open_face ? 0.0 : fp[pr + t], side == 1 && t == c ? step : 0.0);
          }
          if (open_face) boundary_state(*m, m->bidx[f], ul, m->fn[2 * f], m->fn[2 * f + 1], ur);
          hll_flux(ul, ur, m->fn[2 * f], m->fn[2 * f + 1], m->prm.gamma, F);
          double sum = 0.0;
          for (int t = 0; t < 4; ++t) sum += w[t] * std::fabs(F[t].imag() / step);
          gabs[(side == 0 ? pl : pr) + c] += wk * sum;
        }
    }
  }
  std::fill(S, S + 4 * (size_t)nc, 0.0);
  const int nb = m->big.n(), ns = m->small.n();
  for (int i = 0; i < nc; ++i) {
    const CellData& cd = m->cd[i];
    // pinv(A) of each stencil, column s = the solve of unit vector e_s
    std::vector<double> pinv[4];
    for (int k = 0; k < 4; ++k) {
      const QR& q = cd.st[k].qr;
      pinv[k].assign((size_t)q.m * q.n, 0.0);
      std::vector<double> e(q.m, 0.0), x(q.n);
      for (int r = 0; r < q.m; ++r) {
        e[r] = 1.0;
        qr_solve(q, e.data(), x.data());
        e[r] = 0.0;
        for (int l = 0; l < q.n; ++l) pinv[k][(size_t)r * q.n + l] = x[l];
      }
    }
    for (int v = 0; v < 4; ++v) {
      const unsigned f4 = (flags[i] >> (4 * v)) & 0xFu;
      std::vector<double> aabs(nb, 0.0);
      for (int e = 0; e < 3; ++e)
        for (int kq = 0; kq < nq; ++kq) {
          const double g = gabs[((size_t)i * 3 * nq + e * nq + kq) * 4 + v];
          double xi, eta;
          face_point(e, m->gq_t[kq], xi, eta);
          S[4 * (size_t)i + v] += g;
          for (int l = 0; l < nb; ++l) aabs[l] += g * std::fabs(psi(m->big, l, xi, eta));
        }
      const int kept_small = (int)((f4 & 1u) + ((f4 >> 1) & 1u) + ((f4 >> 2) & 1u));
      for (int k = 0; k < 4; ++k) {
        double wgt;
        if (k == 3) {
          if (!(f4 & 8u)) continue;
          wgt = 1.0;
        } else {
          if ((f4 & 8u) || !(f4 & (1u << k))) continue;
          wgt = 1.0 / (double)kept_small;
        }
        const Stencil& St = cd.st[k];
        const int nco = k == 3 ? nb : ns;
        for (int r = 0; r < St.qr.m; ++r) {
          double t = 0.0;
          for (int l = 0; l < nco; ++l) t += std::fabs(pinv[k][(size_t)r * St.qr.n + l]) * aabs[l];
          t *= wgt * St.vol[r];
          S[4 * (size_t)St.cells[r] + v] += t;
          S[4 * (size_t)i + v] += t;
        }
      }
    }
  }
  return 0;
}

// The same comparison scale through one SSP-RK3 step: the step adjoint's
// stage chain with every coefficient and adjoint replaced by its magnitude.
int oracle_vjp_rk_step_scale(void* h, const double* stages, const uint16_t* flags3, double dt,
                             const double* lam_out, double* S_in) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  const size_t nc = m->nc, n4 = 4 * nc;
  std::vector<double> lo(n4), q(n4), s2(n4), s1(n4), s0(n4), tot(n4);
  for (size_t t = 0; t < n4; ++t) lo[t] = std::fabs(lam_out[t]);
  for (size_t t = 0; t < n4; ++t) q[t] = (2.0 / 3.0) * dt * lo[t];
  if (oracle_vjp_scale(h, stages + 2 * n4, flags3 + 2 * nc, q.data(), s2.data())) return -1;
  for (size_t t = 0; t < n4; ++t) s2[t] += (2.0 / 3.0) * lo[t];
  for (size_t t = 0; t < n4; ++t) q[t] = 0.25 * dt * s2[t];
  if (oracle_vjp_scale(h, stages + n4, flags3 + nc, q.data(), s1.data())) return -1;
  for (size_t t = 0; t < n4; ++t) s1[t] += 0.25 * s2[t];
  for (size_t t = 0; t < n4; ++t) q[t] = dt * s1[t];
  if (oracle_vjp_scale(h, stages, flags3, q.data(), s0.data())) return -1;
  for (size_t t = 0; t < n4; ++t) S_in[t] = lo[t] / 3.0 + 0.75 * s2[t] + s1[t] + s0[t];
  return 0;
}

// Adjoint of one SSP-RK3 step with frozen dt and selection.  stages [3][nc][4]
// are the stage inputs (U^n, U^(1), U^(2)) and flags3 [3][nc] their flags;
// lam_out is the adjoint of U^{n+1}; lam_in receives the adjoint of U^n.
int oracle_vjp_rk_step(void* h, const double* stages, const uint16_t* flags3, double dt,
                       const double* lam_out, double* lam_in) {
  Mesh* m = (Mesh*)h;
  if (!ready(*m)) return -1;
  const size_t nc = m->nc, n4 = 4 * nc;
  const double* U0 = stages;
  const double* U1 = stages + n4;
  const double* U2 = stages + 2 * n4;
  std::vector<double> g(n4), lam2(n4), lam1(n4), acc(n4);
  const double a = 1.0 / 3.0, b = 2.0 / 3.0;
  // U' = a U0 + b U2 + b dt R(U2)
  for (size_t t = 0; t < n4; ++t) acc[t] = a * lam_out[t];
  for (size_t t = 0; t < n4; ++t) g[t] = b * dt * lam_out[t];
  if (oracle_vjp(h, U2, flags3 + 2 * nc, g.data(), lam2.data())) return -1;
  for (size_t t = 0; t < n4; ++t) lam2[t] += b * lam_out[t];
  // U2 = 0.75 U0 + 0.25 U1 + 0.25 dt R(U1)
  for (size_t t = 0; t < n4; ++t) acc[t] += 0.75 * lam2[t];
  for (size_t t = 0; t < n4; ++t) g[t] = 0.25 * dt * lam2[t];
  if (oracle_vjp(h, U1, flags3 + nc, g.data(), lam1.data())) return -1;
  for (size_t t = 0; t < n4; ++t) lam1[t] += 0.25 * lam2[t];
  // U1 = U0 + dt R(U0)
  for (size_t t = 0; t < n4; ++t) acc[t] += lam1[t];
  for (size_t t = 0; t < n4; ++t) g[t] = dt * lam1[t];
  std::vector<double> l0(n4);
  if (oracle_vjp(h, U0, flags3, g.data(), l0.data())) return -1;
  for (size_t t = 0; t < n4; ++t) lam_in[t] = acc[t] + l0[t];
  return 0;
}

}  // extern "C"
