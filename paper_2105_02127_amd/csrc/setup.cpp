// Host set-up of libteno: geometry, faces, stencils, reference-space least
// squares and the device-ready packed layouts.  Runs once per mesh; the
// per-stage work happens in the HIP kernels.
//
//  * geometry and faces ............. Sec. 2.1 (semi-discrete form)
//  * stencils ........................ Sec. 3.1: central stencil of 2N_k cells
//    (the target and its 2N_k-1 nearest cells by periodic centroid distance)
//    and three third-order directional stencils (the target and the 11 nearest
//    cells whose centroid lies in the closed cone from the target centroid
//    through the two endpoints of one local edge); ties by lower user id.
//  * least squares ................... Sec. 2.2 eqs. 02-10: affine map of the
//    target onto the reference triangle, zero-mean monomial basis, rows
//    A_sl = int_{V'_s} psi_l, Householder QR, operator M = pinv(A) diag|V'_s|.
//    Monomial integrals use Radon's 7-point degree-5 rule (exact for every
//    basis function up to degree 5, i.e. order 6).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <mutex>

#include "internal.h"

namespace teno {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }
int fail(int code, const std::string& msg) {
  g_error = msg;
  return code;
}
const char* last_error() { return g_error.c_str(); }

Dims dims_for(int order, int nq_req, bool dense) {
  Dims d;
  d.order = order;
  d.r = order - 1;
  int nk = (d.r + 1) * (d.r + 2) / 2;
  d.nu = nk - 1;
  d.nl = 2 * nk - 1;
  d.nq = nq_req > 0 ? nq_req : (order + 1) / 2;
  d.rows = 3 * kSmallRows + d.nl;
  d.rows4 = (d.rows + 3) / 4;
  d.J = 3 * kSmallCoef * kSmallRows + d.nu * d.nl;
  d.dense = dense;
  d.lblk = large_block(d.nl, d.nu, dense);
  d.Jp = 3 * small_block(dense) + d.lblk;
  return d;
}

// ---------------------------------------------------------------------------
// simple parallel-for over [0, n) with std::thread
// ---------------------------------------------------------------------------
template <class F>
static void parallel_for(int n, int threads, F&& f) {
  if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
  threads = std::min(threads, std::max(1, n / 64));
  if (threads <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  const int chunk = 64;
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int b = next.fetch_add(chunk);
        if (b >= n) break;
        int e = std::min(n, b + chunk);
        for (int i = b; i < e; ++i) f(i);
      }
    });
  for (auto& th : pool) th.join();
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
// Minimum-image difference on the periodic axes (kx, ky: periods removed).
static inline void wrap_delta(const Mesh& m, double& dx, double& dy, double& kx, double& ky) {
  kx = ky = 0.0;
  if (m.P[0] > 0.0) {
    kx = std::nearbyint(dx / m.P[0]);
    dx -= m.P[0] * kx;
  }
  if (m.P[1] > 0.0) {
    ky = std::nearbyint(dy / m.P[1]);
    dy -= m.P[1] * ky;
  }
}

int mesh_create(int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri,
                const double* period, Mesh& m) {
  if (n_vert <= 0 || n_cell <= 0 || !xy || !tri) return fail(TENO_EARG, "empty mesh");
  m.nv = n_vert;
  m.nc = n_cell;
  if (period) {
    m.P[0] = period[0];
    m.P[1] = period[1];
    if (!(m.P[0] >= 0.0 && m.P[1] >= 0.0))
      return fail(TENO_EARG, "period must be positive, or 0 for an open axis");
  }
  m.tri.assign(tri, tri + 3 * (size_t)n_cell);
  m.X.resize(6 * (size_t)n_cell);
  m.area.resize(n_cell);
  m.cen.resize(2 * (size_t)n_cell);
  for (int i = 0; i < n_cell; ++i) {
    int32_t* t = &m.tri[3 * (size_t)i];
    double px[3], py[3];
    for (int v = 0; v < 3; ++v) {
      if (t[v] < 0 || t[v] >= n_vert) return fail(TENO_EMESH, "vertex id out of range");
      px[v] = xy[2 * (size_t)t[v]];
      py[v] = xy[2 * (size_t)t[v] + 1];
    }
    for (int v = 1; v < 3; ++v) {
      double dx = px[v] - px[0], dy = py[v] - py[0], kx, ky;
      wrap_delta(m, dx, dy, kx, ky);
      px[v] = px[0] + dx;
      py[v] = py[0] + dy;
    }
    double twice = (px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]);
    if (twice < 0.0) {
      std::swap(t[1], t[2]);
      std::swap(px[1], px[2]);
      std::swap(py[1], py[2]);
      twice = -twice;
    }
    if (!(twice > 0.0)) return fail(TENO_EMESH, "degenerate triangle " + std::to_string(i));
    m.area[i] = 0.5 * twice;
    for (int v = 0; v < 3; ++v) {
      m.X[6 * (size_t)i + 2 * v] = px[v];
      m.X[6 * (size_t)i + 2 * v + 1] = py[v];
    }
    m.cen[2 * (size_t)i] = (px[0] + px[1] + px[2]) / 3.0;
    m.cen[2 * (size_t)i + 1] = (py[0] + py[1] + py[2]) / 3.0;
  }
  for (int a = 0; a < 2; ++a) {
    if (m.P[a] > 0.0) {
      m.lo[a] = 0.0;
      m.hi[a] = m.P[a];
      continue;
    }
    m.lo[a] = m.hi[a] = m.cen[a];
    for (int i = 0; i < n_cell; ++i) {
      m.lo[a] = std::min(m.lo[a], m.cen[2 * (size_t)i + a]);
      m.hi[a] = std::max(m.hi[a], m.cen[2 * (size_t)i + a]);
    }
    if (!(m.hi[a] > m.lo[a])) m.hi[a] = m.lo[a] + 1.0;
  }
  // Faces from directed edges: key (a, b) -> half-edge 3*cell+e.  An
  // undirected edge is one face; L is the cell with the lower user id.
  const size_t nh = 3 * (size_t)n_cell;
  std::vector<uint64_t> key(nh);
  std::vector<int32_t> order(nh);
  for (int i = 0; i < n_cell; ++i)
    for (int e = 0; e < 3; ++e) {
      uint64_t a = (uint32_t)m.tri[3 * (size_t)i + e], b = (uint32_t)m.tri[3 * (size_t)i + (e + 1) % 3];
      key[3 * (size_t)i + e] = (a << 32) | b;
    }
  for (size_t h = 0; h < nh; ++h) order[h] = (int32_t)h;
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
  for (size_t h = 1; h < nh; ++h)
    if (key[order[h]] == key[order[h - 1]]) return fail(TENO_EMESH, "non-manifold edge");
  m.cface.assign(nh, -1);
  for (size_t h = 0; h < nh; ++h) {
    int32_t he = order[h];
    uint64_t k = key[he];
    uint64_t twin = (k << 32) | (k >> 32);
    auto it = std::lower_bound(order.begin(), order.end(), twin,
                               [&](int32_t x, uint64_t v) { return key[x] < v; });
    const int ci = he / 3, ce = he % 3;
    if (it == order.end() || key[*it] != twin) {
      // an edge with one cell: a boundary face, allowed on meshes with an open axis
      if (!m.open()) return fail(TENO_EMESH, "open edge on a mesh periodic in both axes");
      int f = m.nf++;
      m.fL.push_back(ci);
      m.fLe.push_back(ce);
      m.fR.push_back(-1);
      m.fRe.push_back(-1);
      const double* X = &m.X[6 * (size_t)ci];
      double ex = X[2 * ((ce + 1) % 3)] - X[2 * ce];
      double ey = X[2 * ((ce + 1) % 3) + 1] - X[2 * ce + 1];
      double len = std::sqrt(ex * ex + ey * ey);
      m.flen.push_back(len);
      m.fnx.push_back(ey / len);
      m.fny.push_back(-ex / len);
      m.cface[3 * (size_t)ci + ce] = f;
      m.bface.push_back(f);
      continue;
    }
    int32_t ho = *it;
    int co = ho / 3, coe = ho % 3;
    if (co < ci || (co == ci && coe < ce)) continue;  // created from the other side
    int f = m.nf++;
    m.fL.push_back(ci);
    m.fLe.push_back(ce);
    m.fR.push_back(co);
    m.fRe.push_back(coe);
    const double* X = &m.X[6 * (size_t)ci];
    double ex = X[2 * ((ce + 1) % 3)] - X[2 * ce];
    double ey = X[2 * ((ce + 1) % 3) + 1] - X[2 * ce + 1];
    double len = std::sqrt(ex * ex + ey * ey);
    m.flen.push_back(len);
    m.fnx.push_back(ey / len);
    m.fny.push_back(-ex / len);
    m.cface[3 * (size_t)ci + ce] = f;
    m.cface[3 * (size_t)co + coe] = f;
  }
  m.bkind.assign(m.bface.size(), TENO_BC_TRANSMISSIVE);
  m.bstate.assign(4 * m.bface.size(), 0.0);
  return TENO_OK;
}

// ---------------------------------------------------------------------------
// neighbour search: uniform bins over the box (periodic axes wrap), search
// radius grown until the wanted count is found strictly inside the covered
// disc or every bin is covered
// ---------------------------------------------------------------------------
struct Bins {
  int n = 1;
  double wx = 1.0, wy = 1.0;
  std::vector<int32_t> start, cells;
};

// Bin coordinate of a centroid along axis a (periodic axes wrap).
static inline double bin_coord(const Mesh& m, int a, double x) {
  if (m.P[a] > 0.0) return x - m.P[a] * std::floor(x / m.P[a]);
  return x - m.lo[a];
}

static void bins_build(const Mesh& m, Bins& b) {
  double lx = m.hi[0] - m.lo[0], ly = m.hi[1] - m.lo[1];
  b.n = std::max(1, (int)std::floor(std::sqrt(m.nc * 0.5)));
  b.wx = lx / b.n;
  b.wy = ly / b.n;
  std::vector<int32_t> id(m.nc);
  b.start.assign((size_t)b.n * b.n + 1, 0);
  for (int i = 0; i < m.nc; ++i) {
    double x = bin_coord(m, 0, m.cen[2 * (size_t)i]), y = bin_coord(m, 1, m.cen[2 * (size_t)i + 1]);
    int bx = std::min(b.n - 1, std::max(0, (int)(x / b.wx)));
    int by = std::min(b.n - 1, std::max(0, (int)(y / b.wy)));
    id[i] = by * b.n + bx;
    b.start[id[i] + 1]++;
  }
  for (int k = 0; k < b.n * b.n; ++k) b.start[k + 1] += b.start[k];
  b.cells.resize(m.nc);
  std::vector<int32_t> pos(b.start.begin(), b.start.end() - 1);
  for (int i = 0; i < m.nc; ++i) b.cells[pos[id[i]]++] = i;
}

struct Hit {
  double d2;
  int32_t id;
};

static inline bool hit_less(const Hit& a, const Hit& b) {
  return a.d2 < b.d2 || (a.d2 == b.d2 && a.id < b.id);
}

// Closed cone test for directional stencil k of cell i (k = 3: everything).
static inline bool cone_ok(const Mesh& m, int i, int k, double dx, double dy) {
  if (k == 3) return true;
  const double* X = &m.X[6 * (size_t)i];
  double cx = m.cen[2 * (size_t)i], cy = m.cen[2 * (size_t)i + 1];
  int a = k, b = (k + 1) % 3;
  double ax = X[2 * a] - cx, ay = X[2 * a + 1] - cy;
  double bx = X[2 * b] - cx, by = X[2 * b + 1] - cy;
  return (dx * by - dy * bx) >= 0.0 && (ax * dy - ay * dx) >= 0.0;
}

// Cells j != i passing the cone test of stencil k, by distance.
static void search(const Mesh& m, const Bins& b, int i, int k, int want, std::vector<Hit>& scratch) {
  double cx = m.cen[2 * (size_t)i], cy = m.cen[2 * (size_t)i + 1];
  auto consider = [&](int j) {
    if (j == i) return;
    double dx = m.cen[2 * (size_t)j] - cx, dy = m.cen[2 * (size_t)j + 1] - cy, kx, ky;
    wrap_delta(m, dx, dy, kx, ky);
    if (!cone_ok(m, i, k, dx, dy)) return;
    scratch.push_back({dx * dx + dy * dy, j});
  };
  scratch.clear();
  bool full = b.n < 7;
  if (!full) {
    const int bx0 = std::min(b.n - 1, std::max(0, (int)(bin_coord(m, 0, cx) / b.wx)));
    const int by0 = std::min(b.n - 1, std::max(0, (int)(bin_coord(m, 1, cy) / b.wy)));
    const double w = std::min(b.wx, b.wy);
    int rad = 1;
    for (;;) {
      // bin range per axis: a periodic axis wraps (whole axis once the block
      // would overlap itself), an open axis is clipped
      int lo[2], hi[2];
      bool whole[2];
      const int c0[2] = {bx0, by0};
      for (int a = 0; a < 2; ++a) {
        if (m.P[a] > 0.0) {
          whole[a] = 2 * rad + 1 > b.n;
          lo[a] = whole[a] ? 0 : c0[a] - rad;
          hi[a] = whole[a] ? b.n - 1 : c0[a] + rad;
        } else {
          lo[a] = std::max(0, c0[a] - rad);
          hi[a] = std::min(b.n - 1, c0[a] + rad);
          whole[a] = lo[a] == 0 && hi[a] == b.n - 1;
        }
      }
      if (whole[0] && whole[1]) {
        full = true;
        break;
      }
      scratch.clear();
      for (int oy = lo[1]; oy <= hi[1]; ++oy)
        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
          int bx = (ox + b.n) % b.n, by = (oy + b.n) % b.n;
          int bin = by * b.n + bx;
          for (int t = b.start[bin]; t < b.start[bin + 1]; ++t) consider(b.cells[t]);
        }
      // every cell outside the (2 rad + 1)^2 block is at least rad*w away
      double reach = (rad - 0.01) * w;
      if ((int)scratch.size() >= want) {
        std::nth_element(scratch.begin(), scratch.begin() + (want - 1), scratch.end(), hit_less);
        if (scratch[want - 1].d2 < reach * reach) break;
      }
      rad *= 2;
    }
  }
  if (full) {
    scratch.clear();
    for (int j = 0; j < m.nc; ++j) consider(j);
  }
}

// Stencil k of cell i: the `want` nearest cells in the closed cone (k < 3)
// or overall (k = 3).  Near a boundary a cone may hold fewer cells; the
// stencil is then completed with the nearest cells outside the cone.
static bool find_stencil(const Mesh& m, const Bins& b, int i, int k, int want,
                         std::vector<Hit>& scratch, int32_t* out) {
  search(m, b, i, k, want, scratch);
  int have = std::min<int>(want, (int)scratch.size());
  std::partial_sort(scratch.begin(), scratch.begin() + have, scratch.end(), hit_less);
  for (int s = 0; s < have; ++s) out[s] = scratch[s].id;
  if (have == want) return true;
  if (k == 3 || !m.open()) return false;
  search(m, b, i, 3, want + have, scratch);
  std::sort(scratch.begin(), scratch.end(), hit_less);
  for (const Hit& h : scratch) {
    if (have == want) break;
    if (std::find(out, out + have, h.id) == out + have) out[have++] = h.id;
  }
  return have == want;
}

// ---------------------------------------------------------------------------
// least squares (Sec. 2.2): basis, exact moments, Householder pseudo-inverse
// ---------------------------------------------------------------------------
static double fact(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

struct Basis {
  int n = 0;
  int ea[21], eb[21];
  double mean[21];  // average of xi^a eta^b over the reference triangle
};

static Basis basis_of(int r) {
  Basis B;
  for (int deg = 1; deg <= r; ++deg)
    for (int a = deg; a >= 0; --a) {
      B.ea[B.n] = a;
      B.eb[B.n] = deg - a;
      B.mean[B.n] = 2.0 * fact(a) * fact(deg - a) / fact(deg + 2);
      B.n++;
    }
  return B;
}

// Radon's seven-point rule (degree 5) on a triangle, barycentric form.
struct Radon {
  double l[7][3], w[7];
  Radon() {
    const double s15 = std::sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
    double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3},
                        {a1, a1, 1 - 2 * a1}, {a1, 1 - 2 * a1, a1}, {1 - 2 * a1, a1, a1},
                        {a2, a2, 1 - 2 * a2}, {a2, 1 - 2 * a2, a2}, {1 - 2 * a2, a2, a2}};
    double ww[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
    std::memcpy(l, pts, sizeof(l));
    std::memcpy(w, ww, sizeof(w));
  }
};

// Householder QR of the m x n row-major matrix A, then
//   Op[l][s] = (R^{-1} Q_1^T)[l][s] * scale[s].
// Returns min|R_jj|/max|R_jj| (0 on breakdown).
double pinv_scaled(int m, int n, std::vector<double>& A, const double* scale, double* Op) {
  // A row-major [m][n]; Householder vectors stored in place below the diagonal
  std::vector<double> vj(m), beta(n);
  for (int j = 0; j < n; ++j) {
    double nrm2 = 0.0;
    for (int i = j; i < m; ++i) nrm2 += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    double nrm = std::sqrt(nrm2);
    if (nrm == 0.0) return 0.0;
    double x0 = A[(size_t)j * n + j];
    double alpha = x0 > 0.0 ? -nrm : nrm;
    // v = x - alpha e_1, scaled to v_j = 1
    double v0 = x0 - alpha;
    for (int i = j + 1; i < m; ++i) A[(size_t)i * n + j] /= v0;
    double vv = 1.0;
    for (int i = j + 1; i < m; ++i) vv += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    beta[j] = 2.0 / vv;
    for (int c = j + 1; c < n; ++c) {
      double s = A[(size_t)j * n + c];
      for (int i = j + 1; i < m; ++i) s += A[(size_t)i * n + j] * A[(size_t)i * n + c];
      s *= beta[j];
      A[(size_t)j * n + c] -= s;
      for (int i = j + 1; i < m; ++i) A[(size_t)i * n + c] -= s * A[(size_t)i * n + j];
    }
    A[(size_t)j * n + j] = alpha;
  }
  double rmax = 0.0, rmin = INFINITY;
  for (int j = 0; j < n; ++j) {
    double d = std::fabs(A[(size_t)j * n + j]);
    rmax = std::max(rmax, d);
    rmin = std::min(rmin, d);
  }
  if (!(rmin > 1e-13 * rmax)) return 0.0;
  // Q_1 (m x n): apply H_{n-1} ... H_0 to the first n columns of I
  std::vector<double> Q((size_t)m * n, 0.0);
  for (int j = 0; j < n; ++j) Q[(size_t)j * n + j] = 1.0;
  for (int j = n - 1; j >= 0; --j)
    for (int c = 0; c < n; ++c) {
      double s = Q[(size_t)j * n + c];
      for (int i = j + 1; i < m; ++i) s += A[(size_t)i * n + j] * Q[(size_t)i * n + c];
      s *= beta[j];
      Q[(size_t)j * n + c] -= s;
      for (int i = j + 1; i < m; ++i) Q[(size_t)i * n + c] -= s * A[(size_t)i * n + j];
    }
  // Op[:, s] = R^{-1} Q_1[s, :]^T * scale[s]
  std::vector<double> x(n);
  for (int s = 0; s < m; ++s) {
    for (int l = n - 1; l >= 0; --l) {
      double acc = Q[(size_t)s * n + l];
      for (int c = l + 1; c < n; ++c) acc -= A[(size_t)l * n + c] * x[c];
      x[l] = acc / A[(size_t)l * n + l];
    }
    for (int l = 0; l < n; ++l) Op[(size_t)l * m + s] = x[l] * scale[s];
  }
  return rmin / rmax;
}

// Rows of the constrained system of one stencil of (user) cell i.
static void lsq_rows(const Mesh& m, const Basis& B, const Radon& rule, int i, const int32_t* mem,
                     int nrow, std::vector<double>& A, std::vector<double>& vol) {
  const double* X0 = &m.X[6 * (size_t)i];
  const double j00 = X0[2] - X0[0], j01 = X0[4] - X0[0];
  const double j10 = X0[3] - X0[1], j11 = X0[5] - X0[1];
  const double det = j00 * j11 - j01 * j10;
  const double i00 = j11 / det, i01 = -j01 / det, i10 = -j10 / det, i11 = j00 / det;
  A.assign((size_t)nrow * B.n, 0.0);
  vol.assign(nrow, 0.0);
  for (int s = 0; s < nrow; ++s) {
    int j = mem[s];
    double dx = m.cen[2 * (size_t)j] - m.cen[2 * (size_t)i];
    double dy = m.cen[2 * (size_t)j + 1] - m.cen[2 * (size_t)i + 1], kx, ky;
    wrap_delta(m, dx, dy, kx, ky);
    const double sx = -m.P[0] * kx, sy = -m.P[1] * ky;
    const double* Xj = &m.X[6 * (size_t)j];
    double q[3][2];
    for (int v = 0; v < 3; ++v) {
      double px = Xj[2 * v] + sx - X0[0], py = Xj[2 * v + 1] + sy - X0[1];
      q[v][0] = i00 * px + i01 * py;
      q[v][1] = i10 * px + i11 * py;
    }
    // reference-space volume: |V_s| / |det J|
    vol[s] = m.area[j] / det;
    for (int l = 0; l < B.n; ++l) {
      double acc = 0.0;
      for (int g = 0; g < 7; ++g) {
        double xi = rule.l[g][0] * q[0][0] + rule.l[g][1] * q[1][0] + rule.l[g][2] * q[2][0];
        double eta = rule.l[g][0] * q[0][1] + rule.l[g][1] * q[1][1] + rule.l[g][2] * q[2][1];
        double p = 1.0;
        for (int t = 0; t < B.ea[l]; ++t) p *= xi;
        for (int t = 0; t < B.eb[l]; ++t) p *= eta;
        acc += rule.w[g] * p;
      }
      A[(size_t)s * B.n + l] = vol[s] * (acc - B.mean[l]);
    }
  }
}

// Morton code of a point in [0,1)^2 on a 2^16 grid.
static uint32_t spread16(uint32_t x) {
  x &= 0xFFFF;
  x = (x | (x << 8)) & 0x00FF00FF;
  x = (x | (x << 4)) & 0x0F0F0F0F;
  x = (x | (x << 2)) & 0x33333333;
  x = (x | (x << 1)) & 0x55555555;
  return x;
}

int mesh_setup(Mesh& m, const teno_params& p) {
  if (p.order < 3 || p.order > 6) return fail(TENO_EARG, "order must be 3..6");
  if (p.variant < 0 || p.variant > 2) return fail(TENO_EARG, "variant must be 0, 1 or 2");
  if (p.variant == 2 && !(p.dk_prime > 1.0)) return fail(TENO_EARG, "CWENO needs dk_prime > 1");
  if (p.characteristic != 0 && p.characteristic != 1)
    return fail(TENO_EARG, "characteristic must be 0 or 1");
  if (!(p.ct >= 0.0 && p.ct <= 1.0 / 3.0)) return fail(TENO_EARG, "C_T must lie in [0, 1/3]");
  if (p.power < 1 || p.power > 16) return fail(TENO_EARG, "power must be 1..16");
  if (p.n_quad != 0 && (p.n_quad < 2 || p.n_quad > 3)) return fail(TENO_EARG, "n_quad must be 0, 2 or 3");
  m.prm = p;
  m.d = dims_for(p.order, p.n_quad, p.characteristic == 0);
  const Dims& d = m.d;
  const int nc = m.nc;
  // stencil rows are addressed as cell * 4 ceil(rows / 4) + row in 32 bits
  if ((int64_t)(nc + kTile) * d.rows4 * 4 >= (int64_t)INT32_MAX)
    return fail(TENO_EARG, "mesh too large: " + std::to_string(nc) + " cells at order " +
                               std::to_string(p.order) + " exceed 32-bit stencil-row indices");

  // ---- cell order ----
  m.perm.resize(nc);
  for (int i = 0; i < nc; ++i) m.perm[i] = i;
  if (p.reorder) {
    std::vector<uint32_t> code(nc);
    for (int i = 0; i < nc; ++i) {
      double x = bin_coord(m, 0, m.cen[2 * (size_t)i]) / (m.hi[0] - m.lo[0]);
      double y = bin_coord(m, 1, m.cen[2 * (size_t)i + 1]) / (m.hi[1] - m.lo[1]);
      x = std::min(std::max(x, 0.0), 1.0);
      y = std::min(std::max(y, 0.0), 1.0);
      uint32_t qx = std::min<uint32_t>(65535u, (uint32_t)(x * 65536.0));
      uint32_t qy = std::min<uint32_t>(65535u, (uint32_t)(y * 65536.0));
      code[i] = spread16(qx) | (spread16(qy) << 1);
    }
    std::sort(m.perm.begin(), m.perm.end(), [&](int a, int b) {
      return code[a] < code[b] || (code[a] == code[b] && a < b);
    });
  }
  m.inv.assign(nc, 0);
  for (int t = 0; t < nc; ++t) m.inv[m.perm[t]] = t;

  m.n_tiles = (nc + kTile - 1) / kTile;
  m.n_pad = m.n_tiles * kTile;
  try {
    m.idx.assign((size_t)m.n_tiles * d.rows4 * kTile * 4, 0);
    m.M.assign((size_t)m.n_tiles * d.Jp * kTile, 0.0);
  } catch (...) {
    return fail(TENO_ENOMEM, "host allocation of packed operators failed");
  }

  Bins bins;
  bins_build(m, bins);
  const Basis Bs = basis_of(2), Bl = basis_of(d.r);
  const Radon rule;
  std::mutex mu;
  int err_code = TENO_OK, err_cell = nc;
  std::string err_msg;
  double rc_min = 1.0;
  parallel_for(nc, p.n_threads, [&](int i) {
    std::vector<Hit> scratch;
    std::vector<double> A, vol, op;
    int32_t mem[64];
    const int t = m.inv[i];
    double rc_local = 1.0;
    for (int k = 0; k < 4; ++k) {
      const bool big = (k == 3);
      const Basis& B = big ? Bl : Bs;
      const int nrow = big ? d.nl : kSmallRows;
      auto report = [&](int code, const std::string& msg) {
        std::lock_guard<std::mutex> g(mu);
        if (i < err_cell) {
          err_cell = i;
          err_code = code;
          err_msg = msg;
        }
      };
      if (!find_stencil(m, bins, i, k, nrow, scratch, mem)) {
        report(TENO_ESTENCIL, "too few stencil candidates at cell " + std::to_string(i));
        return;
      }
      for (int s = 0; s < nrow; ++s) {
        double dx = m.cen[2 * (size_t)mem[s]] - m.cen[2 * (size_t)i];
        double dy = m.cen[2 * (size_t)mem[s] + 1] - m.cen[2 * (size_t)i + 1], kx, ky;
        wrap_delta(m, dx, dy, kx, ky);
        if ((m.P[0] > 0.0 && std::fabs(dx) > 0.4 * m.P[0]) ||
            (m.P[1] > 0.0 && std::fabs(dy) > 0.4 * m.P[1])) {
          report(TENO_ESTENCIL, "mesh too small for the stencil at cell " + std::to_string(i));
          return;
        }
      }
      lsq_rows(m, B, rule, i, mem, nrow, A, vol);
      op.assign((size_t)B.n * nrow, 0.0);
      double rc = pinv_scaled(nrow, B.n, A, vol.data(), op.data());
      if (rc == 0.0) {
        report(TENO_ERANK, "rank-deficient least-squares matrix at cell " + std::to_string(i));
        return;
      }
      rc_local = std::min(rc_local, rc);
      for (int s = 0; s < nrow; ++s) {
        m.idx[packed_idx_index(m, t, big ? large_row(s) : small_row(k, s))] = m.inv[mem[s]];
        for (int l = 0; l < B.n; ++l)
          m.M[packed_M_offset(d, t, k, s, l)] = op[(size_t)l * nrow + s];
      }
    }
    std::lock_guard<std::mutex> g(mu);
    rc_min = std::min(rc_min, rc_local);
  });
  if (err_code != TENO_OK) return fail(err_code, err_msg);
  m.min_rcond = rc_min;

  // ---- per-cell face data (internal order) ----
  m.nbinfo.assign((size_t)m.n_pad * 4, 0);
  m.geo.assign((size_t)m.n_pad * 10, 0.0);
  m.user_of.assign(m.n_pad, 0);
  for (int t = 0; t < m.n_pad; ++t) {
    if (t >= nc) {
      m.geo[(size_t)t * 10 + 9] = 1.0;  // padding cells: unit area, no neighbours
      continue;
    }
    int i = m.perm[t];
    m.user_of[t] = i;
    int32_t bits = 0;
    for (int e = 0; e < 3; ++e) {
      int f = m.cface[3 * (size_t)i + e];
      bool isL = (m.fL[f] == i && m.fLe[f] == e);
      int other = isL ? m.fR[f] : m.fL[f];
      int oe = isL ? m.fRe[f] : m.fLe[f];
      if (other < 0) {  // boundary face: the cell itself, as its L side
        other = i;
        oe = 0;
      }
      m.nbinfo[(size_t)t * 4 + e] = m.inv[other];
      bits |= (oe & 3) << (2 * e);
      if (isL) bits |= 1 << (6 + e);
      m.geo[(size_t)t * 10 + 3 * e + 0] = m.fnx[f];
      m.geo[(size_t)t * 10 + 3 * e + 1] = m.fny[f];
      m.geo[(size_t)t * 10 + 3 * e + 2] = m.flen[f];
    }
    m.nbinfo[(size_t)t * 4 + 3] = bits;
    m.geo[(size_t)t * 10 + 9] = m.area[i];
  }

  // ---- face-ordered data for the flux kernels ----
  {
    std::vector<int32_t> order(m.nf), rank(m.nf);
    for (int f = 0; f < m.nf; ++f) order[f] = f;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      const int la = m.inv[m.fL[a]], lb = m.inv[m.fL[b]];
      return la < lb || (la == lb && m.fLe[a] < m.fLe[b]);
    });
    m.face_cells.assign((size_t)m.nf * 4, 0);
    m.face_geo.assign((size_t)m.nf * 4, 0.0);
    std::vector<int32_t> bidx(m.nf, -1);
    for (size_t b = 0; b < m.bface.size(); ++b) bidx[m.bface[b]] = (int32_t)b;
    for (int k = 0; k < m.nf; ++k) {
      const int f = order[k];
      rank[f] = k;
      // a boundary face names its own cell on both sides (the kernel loads
      // unconditionally and replaces the outer state) and its index in .w
      const bool bnd = m.fR[f] < 0;
      m.face_cells[(size_t)k * 4 + 0] = m.inv[m.fL[f]];
      m.face_cells[(size_t)k * 4 + 1] = m.inv[bnd ? m.fL[f] : m.fR[f]];
      m.face_cells[(size_t)k * 4 + 2] = (m.fLe[f] & 3) | (((bnd ? m.fLe[f] : m.fRe[f]) & 3) << 2);
      m.face_cells[(size_t)k * 4 + 3] = bnd ? bidx[f] : -1;
      m.face_geo[(size_t)k * 4 + 0] = m.fnx[f];
      m.face_geo[(size_t)k * 4 + 1] = m.fny[f];
      m.face_geo[(size_t)k * 4 + 2] = m.flen[f];
    }
    m.bface_sorted.resize(m.bface.size());
    for (size_t b = 0; b < m.bface.size(); ++b) m.bface_sorted[b] = rank[m.bface[b]];
    m.cell_faces.assign((size_t)m.n_pad * 4, 0);
    m.vol.assign(m.n_pad, 1.0);
    for (int t = 0; t < nc; ++t) {
      const int i = m.perm[t];
      int32_t bits = 0;
      for (int e = 0; e < 3; ++e) {
        const int f = m.cface[3 * (size_t)i + e];
        m.cell_faces[(size_t)t * 4 + e] = rank[f];
        if (m.fL[f] == i && m.fLe[f] == e) bits |= 1 << e;
      }
      m.cell_faces[(size_t)t * 4 + 3] = bits;
      m.vol[t] = m.area[i];
    }
  }

  // ---- distinct stencil members per tile and their LDS slots ----
  {
    std::vector<std::vector<int32_t>> lists(m.n_tiles);
    std::atomic<int> umax{1};
    m.slot.assign(m.idx.size(), 0);
    m.aslot.assign(m.idx.size(), 0);
    m.tround.assign(m.n_tiles, 1);
    parallel_for(m.n_tiles, p.n_threads, [&](int tile) {
      std::vector<int32_t>& u = lists[tile];
      for (int c = 0; c < kTile; ++c) {
        const int t = tile * kTile + c;
        if (t >= nc) break;
        for (int r = 0; r < d.rows; ++r) u.push_back(m.idx[packed_idx_index(m, t, r)]);
      }
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      int cur = umax.load();
      while ((int)u.size() > cur && !umax.compare_exchange_weak(cur, (int)u.size())) {
      }
      for (int c = 0; c < kTile; ++c) {
        const int t = tile * kTile + c;
        if (t >= nc) break;
        for (int r = 0; r < d.rows; ++r) {
          const int64_t k = packed_idx_index(m, t, r);
          m.slot[k] = (uint16_t)(std::lower_bound(u.begin(), u.end(), m.idx[k]) - u.begin());
        }
      }
      // rounds of the adjoint's additions, so that no two lanes of one LDS
      // instruction hit the same address: a block stored rows by lane adds
      // four rows of every cell at once (rows 4j..4j+3 of the block, lane
      // order c * 4 + g), and the lanes of such a group that name the same
      // member add in lane order, one round each; a block of entry pairs
      // adds one row at a time, and the cells that name the same member in
      // that row add in cell order
      int top = 1;
      auto rounds = [&](int r0, int nrow, bool by_lane) {
        const int span = by_lane ? 4 : 1;
        for (int j = 0; j * span < nrow; ++j) {
          const int rg = std::min(span, nrow - j * span);
          for (int c = 0; c < kTile && tile * kTile + c < nc; ++c)
            for (int gq = 0; gq < rg; ++gq) {
              const int64_t k = packed_idx_index(m, tile * kTile + c, r0 + j * span + gq);
              int q = 0;
              for (int c2 = 0; c2 <= c; ++c2)
                for (int g2 = 0; g2 < rg && (c2 < c || g2 < gq); ++g2)
                  if (m.slot[packed_idx_index(m, tile * kTile + c2, r0 + j * span + g2)] == m.slot[k]) ++q;
              m.aslot[k] = (uint16_t)(m.slot[k] | q << 9);
              top = std::max(top, q + 1);
            }
        }
      };
      for (int k = 0; k < 3; ++k) rounds(small_row(k, 0), kSmallRows, lane_rows(kSmallCoef, d.dense));
      rounds(large_row(0), d.nl, large_lane_rows(d.nu, d.dense));
      m.tround[tile] = top;
    });
    if (umax.load() > kMaxTileMembers)
      return fail(TENO_ESTENCIL, "a 16-cell tile has " + std::to_string(umax.load()) +
                                     " distinct stencil members (limit " +
                                     std::to_string(kMaxTileMembers) +
                                     "); keep the default cell reordering");
    m.ustride = (umax.load() + 15) / 16 * 16;
    m.tmem.assign((size_t)m.n_tiles * m.ustride, 0);
    m.tcount.assign(m.n_tiles, 0);
    for (int tile = 0; tile < m.n_tiles; ++tile) {
      const auto& u = lists[tile];
      m.tcount[tile] = (int32_t)u.size();
      for (int k = 0; k < m.ustride; ++k)
        m.tmem[(size_t)tile * m.ustride + k] = u.empty() ? 0 : u[std::min<size_t>(k, u.size() - 1)];
    }
  }

  // ---- reverse member lists for the adjoint gather: the (tile, slot)
  //      entries naming each cell, by tile ----
  m.rev_ptr.assign(nc + 1, 0);
  for (int tile = 0; tile < m.n_tiles; ++tile)
    for (int k = 0; k < m.tcount[tile]; ++k) m.rev_ptr[m.tmem[(size_t)tile * m.ustride + k] + 1]++;
  for (int t = 0; t < nc; ++t) m.rev_ptr[t + 1] += m.rev_ptr[t];
  m.rev_ent.assign(std::max<int32_t>(1, m.rev_ptr[nc]), 0);
  {
    std::vector<int32_t> fill(m.rev_ptr.begin(), m.rev_ptr.end() - 1);
    for (int tile = 0; tile < m.n_tiles; ++tile)
      for (int k = 0; k < m.tcount[tile]; ++k) {
        const int j = m.tmem[(size_t)tile * m.ustride + k];
        m.rev_ent[fill[j]++] = tile * m.ustride + k;
      }
  }
  m.ready = true;
  return TENO_OK;
}

}  // namespace teno
