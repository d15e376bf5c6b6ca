// Host set-up of the tetrahedral path: geometry, faces, stencils,
// reference-space least squares and the device-ready packed layouts.  The
// method is the paper's written in (xi, eta, zeta) (Sec. 2.2 eqs. 02-10 with
// n_d = 3; Sec. 3.1 stencils; Sec. 5.9 runs it on tetrahedra):
//  * geometry and faces: positively oriented tetrahedra, local face e
//    opposite vertex e, one face per shared triangle, unit normal out of L
//    (the cell of lower user id) and area;
//  * stencils: the central stencil is the target and its 2 N_k - 1 nearest
//    cells by (periodic) centroid distance; directional stencil e the target
//    and the 19 nearest cells whose centroid lies in the closed cone from the
//    target centroid through the three vertices of local face e; ties by
//    lower user id; near a wall a short cone is completed with the nearest
//    cells outside it;
//  * least squares: affine map of the target onto the reference
//    tetrahedron, zero-mean monomial basis, rows A_sl = int_{V'_s} psi_l by
//    the Grundmann-Moller rule of degree 5 (exact for every basis function up
//    to order 6), Householder QR, operator M = pinv(A) diag |V'_s|;
//  * smoothness forms B_lm = sum_alpha int_{T_ref} D^alpha phi_l D^alpha phi_m
//    (each multi-index once) from the closed-form moments of T_ref;
//  * face quadrature: symmetric triangle rules whose points the two cells of
//    a face pair up through the permutation of the face's vertices.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>

#include "internal3.h"

namespace teno {

namespace {

template <class F>
void parallel_for3(int n, int threads, F&& f) {
  if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
  threads = std::min(threads, std::max(1, n / 32));
  if (threads <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int i0 = next.fetch_add(16);
        if (i0 >= n) break;
        for (int i = i0; i < std::min(n, i0 + 16); ++i) f(i);
      }
    });
  for (auto& th : pool) th.join();
}

double fact3(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

inline double det3(const double a[3], const double b[3], const double c[3]) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

inline void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// periodic minimum image of displacement d; k gets the period counts removed
inline void wrap3(const Mesh3& m, double d[3], double k[3]) {
  for (int a = 0; a < 3; ++a) {
    k[a] = 0.0;
    if (m.P[a] > 0.0) {
      k[a] = std::nearbyint(d[a] / m.P[a]);
      d[a] -= m.P[a] * k[a];
    }
  }
}

// ---- basis of degree r (graded monomials xi^a eta^b zeta^c) --------------
struct Basis3 {
  int n = 0;
  int e[55][3];
  double mean[55];  // average over the reference tetrahedron
};

Basis3 basis3_of(int r) {
  Basis3 B;
  for (int deg = 1; deg <= r; ++deg)
    for (int a = deg; a >= 0; --a)
      for (int b = deg - a; b >= 0; --b) {
        const int c = deg - a - b;
        B.e[B.n][0] = a;
        B.e[B.n][1] = b;
        B.e[B.n][2] = c;
        // int_{T_ref} xi^a eta^b zeta^c = a! b! c! / (a+b+c+3)!, volume 1/6
        B.mean[B.n] = 6.0 * fact3(a) * fact3(b) * fact3(c) / fact3(deg + 3);
        B.n++;
      }
  return B;
}

// ---- Grundmann-Moller rule of degree 2s+1 = 5 on the tetrahedron ----------
constexpr int kGM5Points = 15;  // C(5,3) + C(4,3) + C(3,3)
// (points in barycentric coordinates; weights sum to 1: the average)
struct GM5 {
  std::vector<double> l0, l1, l2, l3, w;
  GM5() {
    const int s = 2, d = 5, n = 3;
    double tot = 0.0;
    for (int i = 0; i <= s; ++i) {
      const double den = d + n - 2 * i;
      const double wi = ((i % 2) ? -1.0 : 1.0) * std::pow(2.0, -2 * s) * std::pow(den, d) /
                        (fact3(i) * fact3(d + n - i));
      const int k = s - i;
      for (int b0 = 0; b0 <= k; ++b0)
        for (int b1 = 0; b1 <= k - b0; ++b1)
          for (int b2 = 0; b2 <= k - b0 - b1; ++b2) {
            const int b3 = k - b0 - b1 - b2;
            l0.push_back((2 * b0 + 1) / den);
            l1.push_back((2 * b1 + 1) / den);
            l2.push_back((2 * b2 + 1) / den);
            l3.push_back((2 * b3 + 1) / den);
            w.push_back(wi);
            tot += wi;
          }
    }
    for (double& x : w) x /= tot;  // the rule integrates over volume 1/6
    if ((int)w.size() != kGM5Points) std::abort();
  }
};

// ---- bins for the stencil search ------------------------------------------
struct Bins3 {
  int n = 1;
  double w[3] = {1, 1, 1}, lo[3] = {0, 0, 0};
  std::vector<int32_t> start, cells;
};

inline double bin_coord3(const Mesh3& m, const Bins3& b, int a, double x) {
  if (m.P[a] > 0.0) return x - m.P[a] * std::floor(x / m.P[a]);
  return x - b.lo[a];
}

void bins3_build(const Mesh3& m, Bins3& b) {
  double hi[3];
  for (int a = 0; a < 3; ++a) {
    if (m.P[a] > 0.0) {
      b.lo[a] = 0.0;
      hi[a] = m.P[a];
    } else {
      b.lo[a] = INFINITY;
      hi[a] = -INFINITY;
      for (int i = 0; i < m.nc; ++i) {
        b.lo[a] = std::min(b.lo[a], m.cen[3 * (size_t)i + a]);
        hi[a] = std::max(hi[a], m.cen[3 * (size_t)i + a]);
      }
      hi[a] += 1e-12 * (1.0 + std::fabs(hi[a]));
    }
  }
  b.n = std::max(1, (int)std::floor(std::cbrt(m.nc / 6.0)));
  for (int a = 0; a < 3; ++a) b.w[a] = (hi[a] - b.lo[a]) / b.n;
  const int nb = b.n;
  std::vector<int32_t> id(m.nc);
  b.start.assign((size_t)nb * nb * nb + 1, 0);
  for (int i = 0; i < m.nc; ++i) {
    int c[3];
    for (int a = 0; a < 3; ++a)
      c[a] = std::min(nb - 1, std::max(0, (int)(bin_coord3(m, b, a, m.cen[3 * (size_t)i + a]) / b.w[a])));
    id[i] = (c[2] * nb + c[1]) * nb + c[0];
    b.start[id[i] + 1]++;
  }
  for (size_t k = 0; k + 1 < b.start.size(); ++k) b.start[k + 1] += b.start[k];
  b.cells.resize(m.nc);
  std::vector<int32_t> pos(b.start.begin(), b.start.end() - 1);
  for (int i = 0; i < m.nc; ++i) b.cells[pos[id[i]]++] = i;
}

struct Hit3 {
  double d2;
  int32_t id;
};
inline bool hit3_less(const Hit3& a, const Hit3& b) {
  return a.d2 < b.d2 || (a.d2 == b.d2 && a.id < b.id);
}

// closed cone of directional stencil k (k = 4: the central stencil)
inline bool cone3_ok(const Mesh3& m, int i, int k, const double d[3]) {
  if (k == 4) return true;
  const double* X = &m.X[12 * (size_t)i];
  const double* c = &m.cen[3 * (size_t)i];
  double A[3], B[3], C[3];
  for (int a = 0; a < 3; ++a) {
    A[a] = X[3 * kFaceVerts3[k][0] + a] - c[a];
    B[a] = X[3 * kFaceVerts3[k][1] + a] - c[a];
    C[a] = X[3 * kFaceVerts3[k][2] + a] - c[a];
  }
  const double D = det3(A, B, C);
  return det3(d, B, C) * D >= 0.0 && det3(A, d, C) * D >= 0.0 && det3(A, B, d) * D >= 0.0;
}

// Candidates of cell i sorted by (distance, user id): every other cell in the
// block of bins within `rad` of i's bin (all cells when the block covers the
// domain, *whole = true).  Returns the squared distance below which the list
// holds every cell of the mesh.
double candidates3(const Mesh3& m, const Bins3& b, int i, int rad, std::vector<Hit3>& out,
                   bool* whole_out, int* blo, int* bhi) {
  const double* ci = &m.cen[3 * (size_t)i];
  auto consider = [&](int j) {
    if (j == i) return;
    double d[3], kk[3];
    for (int a = 0; a < 3; ++a) d[a] = m.cen[3 * (size_t)j + a] - ci[a];
    wrap3(m, d, kk);
    out.push_back({d[0] * d[0] + d[1] * d[1] + d[2] * d[2], j});
  };
  out.clear();
  const int nb = b.n;
  int lo[3], hi[3];
  bool whole = nb < 5;
  if (!whole) {
    whole = true;
    for (int a = 0; a < 3; ++a) {
      const int c0 = std::min(nb - 1, std::max(0, (int)(bin_coord3(m, b, a, ci[a]) / b.w[a])));
      bool wa;
      if (m.P[a] > 0.0) {
        wa = 2 * rad + 1 > nb;
        lo[a] = wa ? 0 : c0 - rad;
        hi[a] = wa ? nb - 1 : c0 + rad;
      } else {
        lo[a] = std::max(0, c0 - rad);
        hi[a] = std::min(nb - 1, c0 + rad);
        wa = lo[a] == 0 && hi[a] == nb - 1;
      }
      whole = whole && wa;
    }
  }
  *whole_out = whole;
  if (!whole)
    for (int a = 0; a < 3; ++a) {
      blo[a] = lo[a];
      bhi[a] = hi[a];
    }
  if (whole) {
    for (int j = 0; j < m.nc; ++j) consider(j);
  } else {
    for (int oz = lo[2]; oz <= hi[2]; ++oz)
      for (int oy = lo[1]; oy <= hi[1]; ++oy)
        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
          const int bin = (((oz + nb) % nb) * nb + (oy + nb) % nb) * nb + (ox + nb) % nb;
          for (int t = b.start[bin]; t < b.start[bin + 1]; ++t) consider(b.cells[t]);
        }
  }
  std::sort(out.begin(), out.end(), hit3_less);
  if (whole) return INFINITY;
  // every cell outside the searched block is at least rad bin widths away
  const double reach = (rad - 0.01) * std::min(b.w[0], std::min(b.w[1], b.w[2]));
  return reach * reach;
}

// On a mesh open in every axis: true when no centroid outside the block of
// bins [blo, bhi] can lie in the closed cone of local face k of cell i.  The
// centroids fill the box of the bins, so it suffices that the cone clipped to
// that box stays inside the block; the clipped cone is the polytope
// {c + a A + b B + g C : a, b, g >= 0} within the box, and its extent along
// each axis is attained at a vertex (three of its nine planes meeting).
bool cone_inside_block3(const Mesh3& m, const Bins3& b, int i, int k, const int* blo,
                        const int* bhi) {
  const double* X = &m.X[12 * (size_t)i];
  const double* c = &m.cen[3 * (size_t)i];
  double E[3][3];  // columns A, B, C
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) E[a][j] = X[3 * kFaceVerts3[k][j] + a] - c[a];
  double bx0[3], bx1[3], scale = 0.0;
  for (int a = 0; a < 3; ++a) {
    bx0[a] = b.lo[a];
    bx1[a] = b.lo[a] + b.n * b.w[a];
    scale = std::max(scale, bx1[a] - bx0[a]);
  }
  // plane q: q < 3: x_q = 0; else axis (q-3)/2 at the box's low or high side
  auto plane = [&](int q, double row[3], double& rhs) {
    if (q < 3) {
      for (int j = 0; j < 3; ++j) row[j] = j == q ? 1.0 : 0.0;
      rhs = 0.0;
    } else {
      const int a = (q - 3) / 2;
      for (int j = 0; j < 3; ++j) row[j] = E[a][j];
      rhs = ((q - 3) % 2 ? bx1[a] : bx0[a]) - c[a];
    }
  };
  const double tol = 1e-9 * scale;
  double emin[3] = {INFINITY, INFINITY, INFINITY}, emax[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int q0 = 0; q0 < 9; ++q0)
    for (int q1 = q0 + 1; q1 < 9; ++q1)
      for (int q2 = q1 + 1; q2 < 9; ++q2) {
        double R[3][3], r[3];
        plane(q0, R[0], r[0]);
        plane(q1, R[1], r[1]);
        plane(q2, R[2], r[2]);
        const double D = det3(R[0], R[1], R[2]);
        if (std::fabs(D) < 1e-14 * (1.0 + scale * scale * scale)) continue;
        double x[3];
        for (int j = 0; j < 3; ++j) {
          double T[3][3];
          for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) T[u][v] = v == j ? r[u] : R[u][v];
          x[j] = det3(T[0], T[1], T[2]) / D;
        }
        if (x[0] < -1e-12 || x[1] < -1e-12 || x[2] < -1e-12) continue;
        double p[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) {
          p[a] = c[a] + E[a][0] * x[0] + E[a][1] * x[1] + E[a][2] * x[2];
          in = in && p[a] >= bx0[a] - tol && p[a] <= bx1[a] + tol;
        }
        if (!in) continue;
        for (int a = 0; a < 3; ++a) {
          emin[a] = std::min(emin[a], p[a]);
          emax[a] = std::max(emax[a], p[a]);
        }
      }
  for (int a = 0; a < 3; ++a) {
    if (blo[a] > 0 && !(emin[a] > b.lo[a] + blo[a] * b.w[a] + tol)) return false;
    if (bhi[a] < b.n - 1 && !(emax[a] < b.lo[a] + (bhi[a] + 1) * b.w[a] - tol)) return false;
  }
  return true;
}

// All five stencils of user cell i from one sorted candidate list: the
// central one (the nl nearest cells) and directional stencil k (the 19
// nearest cells in the closed cone of local face k; near a wall a cone left
// short is completed with the nearest cells outside it).  A list is accepted
// once its last member lies inside the searched reach; otherwise the block
// grows.  Returns false when the mesh has too few cells.
bool stencils3(const Mesh3& m, const Bins3& b, int i, int nl, std::vector<Hit3>& cand,
               int32_t* small /*[4][19]*/, int32_t* large /*[nl]*/) {
  const bool all_open = !(m.P[0] > 0.0) && !(m.P[1] > 0.0) && !(m.P[2] > 0.0);
  for (int rad = 2;; ++rad) {
    bool whole = false;
    int blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
    const double reach2 = candidates3(m, b, i, rad, cand, &whole, blo, bhi);
    const int nc = (int)cand.size();
    bool ok = nc >= nl && cand[nl - 1].d2 < reach2;
    for (int k = 0; k < 4 && ok; ++k) {
      int32_t* out = small + k * kSmall3Rows;
      auto in_cone = [&](int t) {
        double d[3], kk[3];
        for (int a = 0; a < 3; ++a)
          d[a] = m.cen[3 * (size_t)cand[t].id + a] - m.cen[3 * (size_t)i + a];
        wrap3(m, d, kk);
        return cone3_ok(m, i, k, d);
      };
      // the nearest in-cone cells, as far as the reach vouches for them
      int have = 0, t = 0;
      for (; t < nc && have < kSmall3Rows; ++t) {
        if (!in_cone(t)) continue;
        if (!whole && !(cand[t].d2 < reach2)) break;
        out[have++] = cand[t].id;
      }
      if (have == kSmall3Rows) continue;
      // fewer: go on only once no cell of the cone can lie outside the list
      // (every cell seen, or on an all-open mesh the cone clipped to the
      // domain inside the block); then the list's in-cone cells are all of
      // them, in order
      if (!(whole || (all_open && cone_inside_block3(m, b, i, k, blo, bhi)))) {
        ok = false;
        break;
      }
      for (; t < nc && have < kSmall3Rows; ++t)
        if (in_cone(t)) out[have++] = cand[t].id;
      if (have == kSmall3Rows) continue;
      // a cone left short by a wall takes the nearest cells outside it
      // (open meshes only), as far as the reach vouches for them
      if (!m.open()) return false;
      for (t = 0; t < nc && have < kSmall3Rows; ++t) {
        if (std::find(out, out + have, cand[t].id) != out + have) continue;
        if (!whole && !(cand[t].d2 < reach2)) break;
        out[have++] = cand[t].id;
      }
      if (have < kSmall3Rows) {
        if (whole) return false;
        ok = false;
        break;
      }
    }
    if (ok) {
      for (int s = 0; s < nl; ++s) large[s] = cand[s].id;
      return true;
    }
    if (whole) return false;
  }
}

// rows of stencil `mem` of user cell i: A [nrow][n] row-major, vol [nrow]
void lsq_rows3(const Mesh3& m, const Basis3& B, const GM5& rule, int i, const int32_t* mem,
               int nrow, std::vector<double>& A, std::vector<double>& vol) {
  const double* X0 = &m.X[12 * (size_t)i];
  double c0[3], c1[3], c2[3];  // columns v1-v0, v2-v0, v3-v0
  for (int a = 0; a < 3; ++a) {
    c0[a] = X0[3 + a] - X0[a];
    c1[a] = X0[6 + a] - X0[a];
    c2[a] = X0[9 + a] - X0[a];
  }
  const double det = det3(c0, c1, c2);
  double r0[3], r1[3], r2[3];  // rows of J^-1 times det
  cross3(c1, c2, r0);
  cross3(c2, c0, r1);
  cross3(c0, c1, r2);
  A.assign((size_t)nrow * B.n, 0.0);
  vol.assign(nrow, 0.0);
  const int npt = (int)rule.w.size();
  for (int s = 0; s < nrow; ++s) {
    const int j = mem[s];
    double d[3], kk[3];
    for (int a = 0; a < 3; ++a) d[a] = m.cen[3 * (size_t)j + a] - m.cen[3 * (size_t)i + a];
    wrap3(m, d, kk);
    const double* Xj = &m.X[12 * (size_t)j];
    double q[4][3];
    for (int v = 0; v < 4; ++v) {
      double p[3];
      for (int a = 0; a < 3; ++a) p[a] = Xj[3 * v + a] - m.P[a] * kk[a] - X0[a];
      q[v][0] = (r0[0] * p[0] + r0[1] * p[1] + r0[2] * p[2]) / det;
      q[v][1] = (r1[0] * p[0] + r1[1] * p[1] + r1[2] * p[2]) / det;
      q[v][2] = (r2[0] * p[0] + r2[1] * p[1] + r2[2] * p[2]) / det;
    }
    // reference-space volume: |V_s| / |det J| (|V'_0| = 1/6)
    vol[s] = m.vol[j] / det;
    // powers pw[g][a][t] = x_a^t at the rule's points
    double pw[kGM5Points][3][6];
    for (int g = 0; g < npt; ++g)
      for (int a = 0; a < 3; ++a) {
        const double x = rule.l0[g] * q[0][a] + rule.l1[g] * q[1][a] + rule.l2[g] * q[2][a] +
                         rule.l3[g] * q[3][a];
        pw[g][a][0] = 1.0;
        for (int t = 1; t < 6; ++t) pw[g][a][t] = pw[g][a][t - 1] * x;
      }
    for (int l = 0; l < B.n; ++l) {
      double acc = 0.0;
      for (int g = 0; g < npt; ++g)
        acc += rule.w[g] * (pw[g][0][B.e[l][0]] * pw[g][1][B.e[l][1]] * pw[g][2][B.e[l][2]]);
      A[(size_t)s * B.n + l] = vol[s] * (acc - B.mean[l]);
    }
  }
}

// smoothness form of degree r: B_lm = sum over alpha (1 <= |alpha| <= r,
// each once) of int_{T_ref} D^alpha phi_l D^alpha phi_m
void smooth_form3(const Basis3& B, int r, std::vector<double>& F) {
  F.assign((size_t)B.n * B.n, 0.0);
  auto falling = [](int a, int k) {
    double v = 1.0;
    for (int t = 0; t < k; ++t) v *= (a - t);
    return v;
  };
  for (int deg = 1; deg <= r; ++deg)
    for (int ax = deg; ax >= 0; --ax)
      for (int ay = deg - ax; ay >= 0; --ay) {
        const int az = deg - ax - ay;
        for (int l = 0; l < B.n; ++l) {
          if (B.e[l][0] < ax || B.e[l][1] < ay || B.e[l][2] < az) continue;
          const double fl = falling(B.e[l][0], ax) * falling(B.e[l][1], ay) * falling(B.e[l][2], az);
          for (int mm = 0; mm < B.n; ++mm) {
            if (B.e[mm][0] < ax || B.e[mm][1] < ay || B.e[mm][2] < az) continue;
            const double fm = falling(B.e[mm][0], ax) * falling(B.e[mm][1], ay) * falling(B.e[mm][2], az);
            const int p = B.e[l][0] + B.e[mm][0] - 2 * ax, q = B.e[l][1] + B.e[mm][1] - 2 * ay,
                      t = B.e[l][2] + B.e[mm][2] - 2 * az;
            F[(size_t)l * B.n + mm] += fl * fm * fact3(p) * fact3(q) * fact3(t) / fact3(p + q + t + 3);
          }
        }
      }
}

uint64_t spread21(uint64_t x) {
  x &= 0x1FFFFF;
  x = (x | (x << 32)) & 0x1F00000000FFFFull;
  x = (x | (x << 16)) & 0x1F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

}  // namespace

Dims3 dims3_for(int order) {
  Dims3 d;
  d.order = order;
  d.r = order - 1;
  const int nk = (d.r + 1) * (d.r + 2) * (d.r + 3) / 6;
  d.nu = nk - 1;
  d.nl = 2 * nk - 1;
  d.npt = order <= 4 ? 6 : 7;
  d.rsl = d.nu + (d.nu & 1);
  d.rows = 4 * kSmall3Rows + d.nl;
  d.jp = 4 * kSmall3Blk + d.nl * d.rsl;
  return d;
}

int face_rule3(int order, double (*bary)[3], double* w) {
  int n = 0;
  auto orbit = [&](double a, double wt) {
    const double b = 1.0 - 2.0 * a;
    const double p[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
    for (int k = 0; k < 3; ++k) {
      for (int j = 0; j < 3; ++j) bary[n][j] = p[k][j];
      w[n++] = wt;
    }
  };
  if (order <= 4) {
    // Dunavant (1985), degree 4
    orbit(0.445948490915965, 0.223381589678011);
    orbit(0.091576213509771, 0.109951743655322);
  } else {
    // Radon (1948), degree 5
    const double s = std::sqrt(15.0);
    bary[0][0] = bary[0][1] = bary[0][2] = 1.0 / 3.0;
    w[0] = 9.0 / 40.0;
    n = 1;
    orbit((6.0 - s) / 21.0, (155.0 - s) / 1200.0);
    orbit((6.0 + s) / 21.0, (155.0 + s) / 1200.0);
  }
  return n;
}

int mesh3_create(int32_t n_vert, const double* xyz, int32_t n_cell, const int32_t* tet,
                 const double* period, Mesh3& m) {
  if (n_vert <= 0 || n_cell <= 0 || !xyz || !tet) return fail(TENO_EARG, "empty mesh");
  m.nv = n_vert;
  m.nc = n_cell;
  for (int a = 0; a < 3; ++a) m.P[a] = period && period[a] > 0.0 ? period[a] : 0.0;
  m.tet.assign(tet, tet + 4 * (size_t)n_cell);
  m.X.assign(12 * (size_t)n_cell, 0.0);
  m.vol.assign(n_cell, 0.0);
  m.cen.assign(3 * (size_t)n_cell, 0.0);
  for (int i = 0; i < n_cell; ++i) {
    int32_t* t = &m.tet[4 * (size_t)i];
    double p[4][3];
    for (int v = 0; v < 4; ++v) {
      if (t[v] < 0 || t[v] >= n_vert) return fail(TENO_EMESH, "vertex index out of range");
      for (int a = 0; a < 3; ++a) p[v][a] = xyz[3 * (size_t)t[v] + a];
    }
    for (int v = 1; v < 4; ++v) {
      double d[3] = {p[v][0] - p[0][0], p[v][1] - p[0][1], p[v][2] - p[0][2]}, kk[3];
      wrap3(m, d, kk);
      for (int a = 0; a < 3; ++a) p[v][a] = p[0][a] + d[a];
    }
    double e1[3], e2[3], e3[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = p[1][a] - p[0][a];
      e2[a] = p[2][a] - p[0][a];
      e3[a] = p[3][a] - p[0][a];
    }
    double d6 = det3(e1, e2, e3);
    if (d6 < 0.0) {  // positive orientation: swap the last two vertices
      std::swap(t[2], t[3]);
      for (int a = 0; a < 3; ++a) std::swap(p[2][a], p[3][a]);
      d6 = -d6;
    }
    if (!(d6 > 0.0)) return fail(TENO_EMESH, "degenerate tetrahedron " + std::to_string(i));
    m.vol[i] = d6 / 6.0;
    for (int v = 0; v < 4; ++v)
      for (int a = 0; a < 3; ++a) m.X[12 * (size_t)i + 3 * v + a] = p[v][a];
    for (int a = 0; a < 3; ++a)
      m.cen[3 * (size_t)i + a] = 0.25 * (p[0][a] + p[1][a] + p[2][a] + p[3][a]);
  }
  // faces: the sorted vertex triple of every local face; a triple met twice
  // is an interior face (L = the lower user cell), once a boundary face
  struct Key {
    int32_t v[3];
    int32_t cell, face;
  };
  std::vector<Key> keys(4 * (size_t)n_cell);
  for (int i = 0; i < n_cell; ++i)
    for (int e = 0; e < 4; ++e) {
      Key& k = keys[4 * (size_t)i + e];
      for (int j = 0; j < 3; ++j) k.v[j] = m.tet[4 * (size_t)i + kFaceVerts3[e][j]];
      std::sort(k.v, k.v + 3);
      k.cell = i;
      k.face = e;
    }
  std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
    for (int j = 0; j < 3; ++j)
      if (a.v[j] != b.v[j]) return a.v[j] < b.v[j];
    return a.cell < b.cell || (a.cell == b.cell && a.face < b.face);
  });
  m.cface.assign(4 * (size_t)n_cell, -1);
  for (size_t t = 0; t < keys.size();) {
    size_t u = t + 1;
    while (u < keys.size() && std::equal(keys[u].v, keys[u].v + 3, keys[t].v)) ++u;
    if (u - t > 2) return fail(TENO_EMESH, "non-manifold face");
    const int f = m.nf++;
    const int ci = keys[t].cell, ce = keys[t].face;
    m.fL.push_back(ci);
    m.fLe.push_back(ce);
    m.cface[4 * (size_t)ci + ce] = f;
    const double* X = &m.X[12 * (size_t)ci];
    double ab[3], ac[3], nn[3];
    for (int a = 0; a < 3; ++a) {
      ab[a] = X[3 * kFaceVerts3[ce][1] + a] - X[3 * kFaceVerts3[ce][0] + a];
      ac[a] = X[3 * kFaceVerts3[ce][2] + a] - X[3 * kFaceVerts3[ce][0] + a];
    }
    cross3(ab, ac, nn);
    const double len = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    for (int a = 0; a < 3; ++a) m.fn.push_back(nn[a] / len);
    m.farea.push_back(0.5 * len);
    if (u - t == 2) {
      m.fR.push_back(keys[t + 1].cell);
      m.fRe.push_back(keys[t + 1].face);
      m.cface[4 * (size_t)keys[t + 1].cell + keys[t + 1].face] = f;
    } else {
      if (!m.open()) return fail(TENO_EMESH, "open face on a mesh periodic in all axes");
      m.fR.push_back(-1);
      m.fRe.push_back(-1);
      m.bface.push_back(f);
    }
    t = u;
  }
  m.bkind.assign(m.bface.size(), TENO_BC_TRANSMISSIVE);
  return TENO_OK;
}

int mesh3_setup(Mesh3& m, const teno_params& p) {
  if (p.order < 3 || p.order > 6) return fail(TENO_EARG, "order must be 3..6");
  if (p.variant != 0 && p.variant != 1)
    return fail(TENO_EARG, "tetrahedra: variant must be 0 (TENO) or 1 (LINEAR)");
  if (p.characteristic != 0) return fail(TENO_EARG, "tetrahedra: conservative variables only");
  if (!(p.ct >= 0.0 && p.ct <= 0.25)) return fail(TENO_EARG, "C_T must lie in [0, 1/4]");
  if (p.power < 1 || p.power > 16) return fail(TENO_EARG, "power must be 1..16");
  m.prm = p;
  m.d = dims3_for(p.order);
  const Dims3& d = m.d;
  const int nc = m.nc;
  if ((int64_t)(nc + kTile3) * d.rows >= (int64_t)INT32_MAX)
    return fail(TENO_EARG, "mesh too large for 32-bit stencil-row indices");

  // ---- cell order: Morton curve of the centroids ----
  Bins3 bins;
  bins3_build(m, bins);
  m.perm.resize(nc);
  for (int i = 0; i < nc; ++i) m.perm[i] = i;
  if (p.reorder) {
    std::vector<uint64_t> code(nc);
    for (int i = 0; i < nc; ++i) {
      uint64_t c = 0;
      for (int a = 0; a < 3; ++a) {
        double x = bin_coord3(m, bins, a, m.cen[3 * (size_t)i + a]) / (bins.w[a] * bins.n);
        x = std::min(std::max(x, 0.0), 1.0);
        const uint64_t q = std::min<uint64_t>((1u << 21) - 1, (uint64_t)(x * (1u << 21)));
        c |= spread21(q) << a;
      }
      code[i] = c;
    }
    std::sort(m.perm.begin(), m.perm.end(), [&](int a, int b) {
      return code[a] < code[b] || (code[a] == code[b] && a < b);
    });
  }
  m.inv.assign(nc, 0);
  for (int t = 0; t < nc; ++t) m.inv[m.perm[t]] = t;
  m.n_tiles = (nc + kTile3 - 1) / kTile3;
  m.n_pad = m.n_tiles * kTile3;
  try {
    m.idx.assign((size_t)m.n_tiles * d.rows * kTile3, 0);
    m.M.assign((size_t)m.n_tiles * d.jp * kTile3, 0.0);
  } catch (...) {
    return fail(TENO_ENOMEM, "host allocation of packed operators failed");
  }
  const Basis3 Bs = basis3_of(2), Bl = basis3_of(d.r);
  const GM5 rule;
  std::mutex mu;
  int err_code = TENO_OK, err_cell = nc;
  std::string err_msg;
  double rc_min = 1.0;
  parallel_for3(nc, p.n_threads, [&](int t) {
    const int i = m.perm[t];
    const int tile = t / kTile3, c = t % kTile3;
    std::vector<Hit3> scratch;
    std::vector<int32_t> small(4 * kSmall3Rows), large(d.nl);
    std::vector<double> A, vol, op;
    double rc_local = 1.0;
    if (!stencils3(m, bins, i, d.nl, scratch, small.data(), large.data())) {
      std::lock_guard<std::mutex> lk(mu);
      if (i < err_cell) {
        err_cell = i;
        err_code = TENO_ESTENCIL;
        err_msg = "too few cells for the stencils of cell " + std::to_string(i);
      }
      return;
    }
    for (int k = 0; k <= 4; ++k) {
      const bool big = k == 4;
      const Basis3& B = big ? Bl : Bs;
      const int nrow = big ? d.nl : kSmall3Rows;
      const int32_t* mem = big ? large.data() : small.data() + k * kSmall3Rows;
      for (int s = 0; s < nrow; ++s) {
        double dd[3], kk[3];
        for (int a = 0; a < 3; ++a) dd[a] = m.cen[3 * (size_t)mem[s] + a] - m.cen[3 * (size_t)i + a];
        wrap3(m, dd, kk);
        for (int a = 0; a < 3; ++a)
          if (m.P[a] > 0.0 && std::fabs(dd[a]) > 0.4 * m.P[a]) {
            std::lock_guard<std::mutex> lk(mu);
            if (i < err_cell) {
              err_cell = i;
              err_code = TENO_ESTENCIL;
              err_msg = "mesh too small: a stencil member of cell " + std::to_string(i) +
                        " lies beyond 0.4 of the period";
            }
            return;
          }
      }
      lsq_rows3(m, B, rule, i, mem, nrow, A, vol);
      op.assign((size_t)B.n * nrow, 0.0);
      const double rc = pinv_scaled(nrow, B.n, A, vol.data(), op.data());
      if (!(rc > 0.0)) {
        std::lock_guard<std::mutex> lk(mu);
        if (i < err_cell) {
          err_cell = i;
          err_code = TENO_ERANK;
          err_msg = "rank-deficient least-squares matrix at cell " + std::to_string(i);
        }
        return;
      }
      rc_local = std::min(rc_local, rc);
      const int row0 = big ? 4 * kSmall3Rows : k * kSmall3Rows;
      const int rs = big ? d.rsl : kSmall3Stored;
      const int j0 = big ? 4 * kSmall3Blk : k * kSmall3Blk;
      for (int s = 0; s < nrow; ++s) {
        m.idx[((size_t)tile * d.rows + row0 + s) * kTile3 + c] = m.inv[mem[s]];
        for (int l = 0; l < B.n; ++l) {
          const int j = j0 + s * rs + l;
          m.M[(((size_t)tile * (d.jp / 2) + j / 2) * kTile3 + c) * 2 + (j & 1)] =
              op[(size_t)l * nrow + s];
        }
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    rc_min = std::min(rc_min, rc_local);
  });
  if (err_code != TENO_OK) return fail(err_code, err_msg);
  m.min_rcond = rc_min;
  // padding cells of the last tile name themselves... name the tile's first
  // cell, whose loads are valid
  for (int t = nc; t < m.n_pad; ++t) {
    const int tile = t / kTile3, c = t % kTile3;
    for (int r = 0; r < d.rows; ++r)
      m.idx[((size_t)tile * d.rows + r) * kTile3 + c] = m.idx[((size_t)tile * d.rows + r) * kTile3];
  }

  // ---- universal tables: smoothness forms and the face basis ----
  smooth_form3(Bs, 2, m.Bsmall);
  smooth_form3(Bl, d.r, m.Blarge);
  double bary[7][3], wq[7];
  const int npt = face_rule3(p.order, bary, wq);
  static const double V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  m.psi.assign((size_t)4 * npt * d.nu, 0.0);
  for (int e = 0; e < 4; ++e)
    for (int q = 0; q < npt; ++q) {
      double x[3] = {0, 0, 0};
      for (int j = 0; j < 3; ++j)
        for (int a = 0; a < 3; ++a) x[a] += bary[q][j] * V[kFaceVerts3[e][j]][a];
      for (int l = 0; l < Bl.n; ++l) {
        double v = 1.0;
        for (int a = 0; a < 3; ++a)
          for (int t = 0; t < Bl.e[l][a]; ++t) v *= x[a];
        m.psi[((size_t)e * npt + q) * d.nu + l] = v - Bl.mean[l];
      }
    }

  // ---- faces in the order of their L cell, with the point pairing ----
  m.fpair.assign(m.nf, 0);
  for (int f = 0; f < m.nf; ++f) {
    if (m.fR[f] < 0) continue;
    int vl[3], vr[3];
    for (int j = 0; j < 3; ++j) {
      vl[j] = m.tet[4 * (size_t)m.fL[f] + kFaceVerts3[m.fLe[f]][j]];
      vr[j] = m.tet[4 * (size_t)m.fR[f] + kFaceVerts3[m.fRe[f]][j]];
    }
    int packed = 0;
    for (int k = 0; k < npt; ++k) {
      // the point in the neighbour's vertex order
      double want[3];
      for (int j = 0; j < 3; ++j) {
        int jl = 0;
        while (vl[jl] != vr[j]) ++jl;
        want[j] = bary[k][jl];
      }
      int q = 0;
      while (q < npt && !(std::fabs(bary[q][0] - want[0]) < 1e-12 &&
                          std::fabs(bary[q][1] - want[1]) < 1e-12 &&
                          std::fabs(bary[q][2] - want[2]) < 1e-12))
        ++q;
      if (q == npt) return fail(TENO_EMESH, "face points do not pair up");
      packed |= q << (3 * k);
    }
    m.fpair[f] = packed;
  }
  std::vector<int32_t> order(m.nf);
  for (int f = 0; f < m.nf; ++f) order[f] = f;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const int la = m.inv[m.fL[a]], lb = m.inv[m.fL[b]];
    return la < lb || (la == lb && m.fLe[a] < m.fLe[b]);
  });
  std::vector<int32_t> rank(m.nf), bidx(m.nf, -1);
  for (int r = 0; r < m.nf; ++r) rank[order[r]] = r;
  for (size_t b = 0; b < m.bface.size(); ++b) bidx[m.bface[b]] = (int)b;
  m.face_cells.assign(4 * (size_t)m.nf, 0);
  m.face_geo.assign(4 * (size_t)m.nf, 0.0);
  for (int r = 0; r < m.nf; ++r) {
    const int f = order[r];
    const int L = m.inv[m.fL[f]];
    const bool bnd = m.fR[f] < 0;
    m.face_cells[4 * (size_t)r] = L;
    m.face_cells[4 * (size_t)r + 1] = bnd ? -1 - bidx[f] : m.inv[m.fR[f]];
    m.face_cells[4 * (size_t)r + 2] = m.fLe[f] | ((bnd ? 0 : m.fRe[f]) << 2);
    m.face_cells[4 * (size_t)r + 3] = m.fpair[f];
    for (int a = 0; a < 3; ++a) m.face_geo[4 * (size_t)r + a] = m.fn[3 * (size_t)f + a];
    m.face_geo[4 * (size_t)r + 3] = m.farea[f];
  }
  m.bkind_sorted = m.bkind;
  m.cell_faces.assign(4 * (size_t)m.n_pad, 0);
  m.cell_side.assign(m.n_pad, 0);
  m.geo.assign(17 * (size_t)m.n_pad, 0.0);
  m.user_of.assign(m.n_pad, -1);
  for (int t = 0; t < m.n_pad; ++t) {
    const int i = m.perm[t < nc ? t : 0];
    m.user_of[t] = t < nc ? i : -1;
    int bits = 0;
    for (int e = 0; e < 4; ++e) {
      const int f = m.cface[4 * (size_t)i + e];
      m.cell_faces[4 * (size_t)t + e] = rank[f];
      const bool isL = m.fL[f] == i && m.fLe[f] == e;
      if (isL) bits |= 1 << e;
      const double s = isL ? 1.0 : -1.0;
      for (int a = 0; a < 3; ++a) m.geo[17 * (size_t)t + 4 * e + a] = s * m.fn[3 * (size_t)f + a];
      m.geo[17 * (size_t)t + 4 * e + 3] = m.farea[f];
    }
    m.cell_side[t] = bits;
    m.geo[17 * (size_t)t + 16] = t < nc ? m.vol[i] : 1.0;
  }
  m.ready = true;
  return TENO_OK;
}

}  // namespace teno
