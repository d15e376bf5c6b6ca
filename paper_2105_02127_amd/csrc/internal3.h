// Library-internal data of the tetrahedral path (three-dimensional TENO):
// host set-up (setup3.cpp) and device launches (teno3_api.hip).
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"

namespace teno {

// Cells per wavefront tile: five lanes per cell (one per conservative
// variable), twelve cells in the 64 lanes (the last four lanes idle).
constexpr int kTile3 = 12;
constexpr int kVars3 = 5;
constexpr int kSmall3Rows = 19;  // 2 N_k - 1 with N_k = 10 (degree 2, n_d = 3)
constexpr int kSmall3Coef = 9;
constexpr int kSmall3Stored = 10;  // stored row length (whole 16-byte pairs)
constexpr int kSmall3Blk = kSmall3Rows * kSmall3Stored;

// local face e of a tetrahedron: the face opposite vertex e, vertices in the
// order that makes (b - a) x (c - a) point out of a positively oriented cell
constexpr int kFaceVerts3[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

// Sizes of one order (Sec. 2.2 eq. 03 with n_d = 3: N_k = C(r+3, 3) counting
// the constant; N_s = 2 N_k cells including the target, 2 N_k - 1 rows).
struct Dims3 {
  int order = 0, r = 0;
  int nu = 0;    // unknowns of the large stencil
  int nl = 0;    // rows of the large stencil
  int npt = 0;   // quadrature points per triangular face (6 or 7)
  int rsl = 0;   // stored row length of the large stencil (nu rounded up to even)
  int rows = 0;  // all rows: 4 x 19 small + nl
  int jp = 0;    // stored operator entries per cell: 4 small blocks + nl * rsl
};

Dims3 dims3_for(int order);

// Face rule of an order (symmetric triangle rules, barycentric coordinates
// in the cell's local face order): Dunavant's 6 points of degree 4 at orders
// 3-4, Radon's 7 points of degree 5 at orders 5-6.
int face_rule3(int order, double (*bary)[3], double* w);

struct Mesh3 {
  int nv = 0, nc = 0, nf = 0;
  double P[3] = {0, 0, 0};        // period per axis, 0 = open
  std::vector<double> X;          // [nc][4][3] vertices unwrapped about v0
  std::vector<int32_t> tet;       // [nc][4] positively oriented
  std::vector<double> vol, cen;   // [nc], [nc][3]
  std::vector<int32_t> fL, fR, fLe, fRe;  // user ids; fR = -1 on a boundary face
  std::vector<double> fn, farea;          // [nf][3] unit normal out of L, area
  std::vector<int32_t> cface;             // [nc][4]
  std::vector<int32_t> fpair;             // [nf] R's point of L's point k, 3 bits each
  std::vector<int32_t> bface, bkind;      // boundary faces, kind (1 or 2)
  bool open() const { return !(P[0] > 0 && P[1] > 0 && P[2] > 0); }

  bool ready = false;
  teno_params prm{};
  Dims3 d;
  std::vector<int32_t> perm, inv;  // perm[internal] = user
  double min_rcond = 1.0;

  // packed device images (internal order, tiles of kTile3 cells)
  int n_pad = 0, n_tiles = 0;
  std::vector<int32_t> idx;       // [n_tiles][rows][kTile3] member (internal)
  std::vector<double> M;          // [n_tiles][jp/2][kTile3][2]
  std::vector<double> Bsmall, Blarge;  // smoothness forms [9][9], [nu][nu]
  std::vector<double> psi;        // [4][npt][nu] basis at the face points
  // faces sorted by their L cell's internal index
  std::vector<int32_t> face_cells;  // [nf][4]: L, R (-1 - b on boundary face b), eL | eR << 2, pairing
  std::vector<double> face_geo;     // [nf][4]: nx, ny, nz, |A|
  std::vector<int32_t> cell_faces;  // [n_pad][4]: sorted face of local faces 0..3
  std::vector<int32_t> cell_side;   // [n_pad]: bit e set when the cell is the face's L
  std::vector<double> geo;          // [n_pad][17]: (n, |A|) out of the cell per face, |V|
  std::vector<int32_t> user_of;     // [n_pad]
  std::vector<int32_t> bkind_sorted;  // [n_bface] kind of boundary face b
};

int mesh3_create(int32_t n_vert, const double* xyz, int32_t n_cell, const int32_t* tet,
                 const double* period, Mesh3& m);
int mesh3_setup(Mesh3& m, const teno_params& p);

// Householder QR of the m x n row-major matrix A (overwritten), then
// Op[l][s] = pinv(A)[l][s] * scale[s]; returns min|R_jj| / max|R_jj|.
double pinv_scaled(int m, int n, std::vector<double>& A, const double* scale, double* Op);

}  // namespace teno

struct teno3_mesh {
  teno::Mesh3 m;
};
