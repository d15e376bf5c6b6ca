// Library-internal data shared by the host set-up and the device launches.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/teno.h"

namespace teno {

// Cells per wavefront tile of the reconstruction kernel (16 or 8): the 64
// lanes of a wavefront give each cell 64 / kTile lanes.  Host packing and
// device kernels must agree, so both compilers see the same macro.
#ifndef TENO_TILE
#define TENO_TILE 16
#endif
constexpr int kTile = TENO_TILE;
constexpr int kLanesPerCell = 64 / kTile;
static_assert(kTile == 16 || kTile == 8, "tile must hold 16 or 8 cells");

// Sizes of one order (Sec. 2.2 eq. 03 with N_k counting the constant term;
// N_s = 2 N_k cells including the target, so 2 N_k - 1 least-squares rows).
struct Dims {
  int order = 0, r = 0;
  int nu = 0;      // unknowns of the large stencil, N_k - 1
  int nl = 0;      // rows of the large stencil
  int nq = 0;      // Gauss points per face
  int rows = 0;    // all stencil rows: 3 * 11 small + nl
  int rows4 = 0;   // rows rounded up to a multiple of 4 (int4 loads)
  int J = 0;       // operator entries per cell: 3 * 5 * 11 + nu * nl
  int lblk = 0;    // stored entries of the large stencil (see block_entries)
  int Jp = 0;      // stored entries per cell: 3 small blocks + lblk
  bool dense = true;  // operator blocks of odd row length stored rows by lane
};

Dims dims_for(int order, int nq_req, bool dense);

// Largest number of distinct stencil members a 16-cell tile may have (their
// states are staged in LDS, 32 bytes each).
constexpr int kMaxTileMembers = 384;
static_assert(kMaxTileMembers <= 512, "member slots take 9 bits of the adjoint's slot word");

constexpr int kSmallRows = 11;
constexpr int kSmallCoef = 5;

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

struct Mesh {
  // ---- geometry, user order ----
  int nv = 0, nc = 0, nf = 0;
  double P[2] = {0.0, 0.0};           // period per axis, 0 = open axis
  double lo[2] = {0.0, 0.0}, hi[2] = {1.0, 1.0};  // box of the centroids (open axes)
  std::vector<int32_t> tri;           // [nc][3] counter-clockwise
  std::vector<double> X;              // [nc][3][2] vertices unwrapped about v0
  std::vector<double> area, cen;      // [nc], [nc][2]
  std::vector<int32_t> fL, fR, fLe, fRe;  // face -> L/R cell (user id), local edges
  std::vector<double> fnx, fny, flen;     // unit normal out of L, edge length
  std::vector<int32_t> cface;         // [nc][3] face of each local edge
  // boundary faces (an edge with one cell, on an open axis): fR = fRe = -1
  std::vector<int32_t> bface;         // [n_bface] face id, in creation order
  std::vector<int32_t> bkind;         // [n_bface] TENO_BC_* (default transmissive)
  std::vector<double> bstate;         // [n_bface][4] prescribed states
  bool open() const { return !(P[0] > 0.0 && P[1] > 0.0); }

  // ---- set-up ----
  bool ready = false;
  teno_params prm{};
  Dims d;
  std::vector<int32_t> perm, inv;     // perm[internal] = user, inv[user] = internal
  double min_rcond = 1.0;

  // ---- packed device images, internal order, tile-major ----
  int n_pad = 0, n_tiles = 0;
  std::vector<int32_t> idx;     // [n_tiles][rows4][16][4] stencil members (internal; host)
  // distinct stencil members of each tile, staged in LDS by the kernel
  int ustride = 0;              // list length per tile (largest count, rounded up)
  std::vector<int32_t> tmem;    // [n_tiles][ustride] sorted, padded with the last
  std::vector<int32_t> tcount;  // [n_tiles] distinct members of each tile (unpadded)
  std::vector<uint16_t> slot;   // [n_tiles][rows4][16][4] position of each member in its
                                // tile's list (packed like idx)
  std::vector<double> M;        // [n_tiles][Jp/2][kTile][2] operator entries (pairs)
  std::vector<int32_t> nbinfo;  // [n_pad][4]: 3 neighbours + packed edge/side bits
  std::vector<double> geo;      // [n_pad][10]: (nx, ny, len) x 3 edges, area
  std::vector<int32_t> user_of; // [n_pad] user id (diagnostics)
  // face-ordered flux data: faces sorted by their L cell's internal index
  std::vector<int32_t> face_cells;  // [nf][4]: L, R (internal; L again on a boundary
                                    //   face), eL | eR << 2, boundary index or -1
  std::vector<double> face_geo;     // [nf][4]: nx, ny (out of L), |A|, 0
  std::vector<int32_t> bface_sorted; // [n_bface]: face-ordered index of boundary face b
  std::vector<int32_t> cell_faces;  // [n_pad][4]: sorted face of local edges 0..2;
                                    //   bit e of [3] set when the cell is that face's L
  std::vector<double> vol;          // [n_pad] |V| (1 for padding cells)
  // adjoint accumulation order: aslot[tile][rows4][16][4] = slot | round << 9,
  // where round = how many earlier cells of the tile name the same member
  // in that row; tround[tile] = the tile's largest round plus one
  std::vector<uint16_t> aslot;
  std::vector<int32_t> tround;
  // reverse member lists (adjoint gather): the tile member slots naming cell j
  std::vector<int32_t> rev_ptr; // [n_cell + 1]
  std::vector<int32_t> rev_ent; // tile * ustride + slot, by tile
};

// Stencil row order of a cell: rows 0..32 hold the three small stencils
// (row s of small stencil k is row 11k + s), then the nl large-stencil rows.
constexpr int small_row(int k, int s) { return kSmallRows * k + s; }
constexpr int large_row(int s) { return 3 * kSmallRows + s; }

// Stored operator entries of one stencil (M^T: nrow rows of L
// coefficients), in one of two block layouts (offsets in doubles within the
// block of a tile of kTile cells):
//  * rows by lane (dense meshes, odd L: the small stencils and the large one
//    at orders 3 and 4): the rows come in groups of four; lane g of a cell
//    owns row 4j + g of group j and reads its L entries from L planes, each
//    holding entry l of the group's rows for every cell (cell-major,
//    row-minor).  The last group may hold fewer rows.  Nothing is padded,
//    and a wavefront's load of one plane covers 16 cells x 4 rows
//    contiguously.
//  * entry pairs (even L, or any L on meshes that are not dense): M^T row by
//    row as 16-byte pairs, [pair][cell][2], odd rows padded with a zero to
//    even length; lane g of a cell reads pairs g, g + 4, ... of each row.
// Meshes reconstructed in conservative variables are dense; the
// characteristic-variable kernel holds more values across its streams and
// measured faster on entry pairs.  TENO_DENSE=0 makes no mesh dense.
#ifndef TENO_DENSE
#define TENO_DENSE 1
#endif
#ifndef TENO_LARGE_LANES
#define TENO_LARGE_LANES 1
#endif
constexpr bool lane_rows(int L, bool dense) { return TENO_DENSE && dense && (L & 1) && kTile == 16; }
// the large stencil's block (its rows are longer than the small ones')
constexpr bool large_lane_rows(int L, bool dense) { return TENO_LARGE_LANES && lane_rows(L, dense); }
constexpr int stored_row(int L) { return L + (L & 1); }
constexpr int block_entries(int nrow, int L, bool dense) {
  return lane_rows(L, dense) ? nrow * L : nrow * stored_row(L);
}
constexpr int group_rows(int nrow, int j) { return nrow - 4 * j < 4 ? nrow - 4 * j : 4; }
constexpr int block_offset(int nrow, int L, bool dense, int c, int s, int l) {
  return lane_rows(L, dense)
             ? 4 * kTile * L * (s / 4) + (l * kTile + c) * group_rows(nrow, s / 4) + (s % 4)
             : (((s * stored_row(L) + l) >> 1) * kTile + c) * 2 + ((s * stored_row(L) + l) & 1);
}
constexpr int small_block(bool dense) { return block_entries(kSmallRows, kSmallCoef, dense); }
constexpr int large_block(int nrow, int L, bool dense) {
  return block_entries(nrow, L, large_lane_rows(L, dense));
}
constexpr int large_block_offset(int nrow, int L, bool dense, int c, int s, int l) {
  return block_offset(nrow, L, large_lane_rows(L, dense), c, s, l);
}

// The operator stream of a tile: the three small stencils' blocks, then the
// large stencil's, Jp * kTile doubles in all.  Block k (3 = large) starts at
// block_start(k, dense) * kTile.
constexpr int block_start(int k, bool dense) { return small_block(dense) * k; }
inline int64_t packed_M_offset(const Dims& d, int internal, int k, int s, int l) {
  const int t = internal / kTile, c = internal % kTile;
  const bool big = k == 3;
  return ((int64_t)t * d.Jp + block_start(k, d.dense)) * kTile +
         (big ? large_block_offset(d.nl, d.nu, d.dense, c, s, l)
              : block_offset(kSmallRows, kSmallCoef, d.dense, c, s, l));
}

inline int64_t packed_idx_index(const Mesh& m, int internal, int row) {
  int t = internal / kTile, c = internal % kTile;
  return (((int64_t)t * m.d.rows4 + (row >> 2)) * kTile + c) * 4 + (row & 3);
}

int mesh_create(int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri,
                const double* period, Mesh& m);
int mesh_setup(Mesh& m, const teno_params& p);

}  // namespace teno

struct teno_mesh {
  teno::Mesh m;
};
