// C ABI of libteno (include/teno.h): argument checks, device buffers and
// kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "kernels.hpp"

namespace teno {
const char* last_error();
}

using namespace teno;

namespace {

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<P>, IC<NQ>) for the supported (order, face points) pairs.
template <class F>
bool dispatch(int P, int NQ, F&& f) {
  switch (P * 10 + NQ) {
    case 32: f(IC<3>{}, IC<2>{}); return true;
    case 33: f(IC<3>{}, IC<3>{}); return true;
    case 42: f(IC<4>{}, IC<2>{}); return true;
    case 43: f(IC<4>{}, IC<3>{}); return true;
    case 52: f(IC<5>{}, IC<2>{}); return true;
    case 53: f(IC<5>{}, IC<3>{}); return true;
    case 62: f(IC<6>{}, IC<2>{}); return true;
    case 63: f(IC<6>{}, IC<3>{}); return true;
    default: return false;
  }
}

struct DeviceScope {
  int prev = -1;
  bool ok = true;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int hip_fail(hipError_t e, const char* what) {
  return fail(TENO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

// SSP-RK3 stage k: U^(k+1) = A[k] U^n + B[k] U^(k) + C[k] dt R(U^(k)).
static const double kStageA[3] = {1.0, 0.75, 1.0 / 3.0};
static const double kStageB[3] = {0.0, 0.25, 2.0 / 3.0};
static const double kStageC[3] = {1.0, 0.25, 2.0 / 3.0};

struct teno_solver {
  int device = 0;
  Dims d;
  teno_params prm{};
  int n_cell = 0, n_pad = 0, n_tiles = 0;
  int4* slot = nullptr;     // member slots of each tile's stencil rows (uint16)
  int4* aslot = nullptr;    // adjoint: member slot and accumulation round per row
  int* tround = nullptr;    // adjoint: rounds per tile
  int* tmem = nullptr;      // distinct stencil members of each tile
  int ustride = 0;
  double2* M = nullptr;
  int4* nbinfo = nullptr;
  double* geo = nullptr;
  int4* fcell = nullptr;    // face-ordered flux data
  double2* fgeo = nullptr;
  int4* cfaces = nullptr;
  double* vol = nullptr;
  double* phi = nullptr;    // face fluxes of the last stage
  int n_face = 0;
  int n_bface = 0;
  int* bkind = nullptr;     // boundary conditions (meshes with an open axis)
  double* bstate = nullptr;
  int* bface = nullptr;     // face-ordered index of each boundary face
  int32_t* user_of = nullptr;
  int32_t* rev_ptr = nullptr;
  int32_t* rev_ent = nullptr;
  double* fp = nullptr;
  double* fpbar = nullptr;
  double* tbar = nullptr;   // adjoint: per-tile member sums [n_tiles][ustride][4]
  double* own = nullptr;
  double* W1 = nullptr;
  double* W2 = nullptr;
  double* T0 = nullptr;
  double* T1 = nullptr;
  double* T2 = nullptr;
  double* dtpart = nullptr;
  int n_dtblk = 0;
  DevDiag* diag = nullptr;
  std::vector<void*> allocs;
  int64_t bytes = 0;
  // profiling
  unsigned prof = 0;  // bit k: time kernels of kind k
  struct Ev {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Ev> evs;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  double prof_ms[4] = {0, 0, 0, 0};
  int64_t prof_n[4] = {0, 0, 0, 0};

  template <class T>
  int alloc(T*& p, size_t count) {
    void* q = nullptr;
    size_t nb = std::max<size_t>(count * sizeof(T), 256);
    hipError_t e = hipMalloc(&q, nb);
    if (e != hipSuccess) return fail(TENO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(q);
    bytes += (int64_t)nb;
    p = (T*)q;
    return TENO_OK;
  }
  ~teno_solver() {
    for (auto& e : evs) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (auto& e : pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    for (void* q : allocs) (void)hipFree(q);
  }
};

namespace {

// Records kernel timing around `launch` when profiling is on for `kind`.
template <class F>
int timed(teno_solver* s, int kind, hipStream_t st, F&& launch) {
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  const bool on = (s->prof >> kind) & 1;
  if (on) {
    if (!s->pool.empty()) {
      ev = s->pool.back();
      s->pool.pop_back();
    } else {
      if (hipEventCreate(&ev.first) != hipSuccess) return fail(TENO_EHIP, "hipEventCreate failed");
      if (hipEventCreate(&ev.second) != hipSuccess) {
        (void)hipEventDestroy(ev.first);
        return fail(TENO_EHIP, "hipEventCreate failed");
      }
    }
    (void)hipEventRecord(ev.first, st);
  }
  launch();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  if (on) {
    (void)hipEventRecord(ev.second, st);
    s->evs.push_back({kind, ev.first, ev.second});
  }
  return TENO_OK;
}

// chi counts as a near tie when |chi / C_T - 1| <= tie_rel; an empty window
// when C_T = 0 (the linear scheme has no ties).
static void set_tie_window(ReconArgs& a) {
  if (a.ct > 0.0) {
    a.tie_lo = a.ct * (1.0 - a.tie_rel);
    a.tie_hi = a.ct * (1.0 + a.tie_rel);
  } else {
    a.tie_lo = 1.0;
    a.tie_hi = 0.0;
  }
}

// Doubles of one stage's face states in the library layout [3 nq][n_pad][4].
static size_t face_state_doubles(const teno_solver* s) { return (size_t)3 * s->d.nq * s->n_pad * 4; }

// fp: face-state buffer of the launch (library layout), nullptr = the
// solver's own.
int launch_reconstruct(teno_solver* s, const double* U, uint16_t* flags, bool frozen,
                       hipStream_t st, double* fp = nullptr) {
  ReconArgs a;
  a.U = U;
  a.slot = s->slot;
  a.tmem = s->tmem;
  a.ustride = s->ustride;
  a.lds_stride = stage_int4(s->d.rows4, s->ustride);
  if (s->prm.characteristic != 0) a.lds_stride = std::max(a.lds_stride, char_gram_int4());
  a.M = s->M;
  a.fp = fp ? fp : s->fp;
  a.flags = flags;
  a.user_of = s->user_of;
  a.geo = s->geo;
  a.nbinfo = s->nbinfo;
  a.diag = s->diag;
  a.n_cell = s->n_cell;
  a.n_tiles = s->n_tiles;
  a.n_pad = s->n_pad;
  a.frozen = frozen ? 1 : 0;
  a.variant = s->prm.variant;
  a.fallback = s->prm.fallback;
  a.power = s->prm.power;
  a.ct = s->prm.ct;
  a.eps = s->prm.eps;
  a.gamma = s->prm.gamma;
  a.tie_rel = s->prm.tie_rel;
  set_tie_window(a);
  a.cw_dK = 1.0 - 1.0 / s->prm.dk_prime;
  a.cw_ds = (1.0 - a.cw_dK) / 3.0;
  const int blocks = (s->n_tiles + kReconBlockWaves - 1) / kReconBlockWaves;
  const dim3 threads(64 * kReconBlockWaves);
  const size_t lds = (size_t)kReconBlockWaves * a.lds_stride * sizeof(int4);
  const bool cw = s->prm.variant == 2, ch = s->prm.characteristic != 0;
  int rc = TENO_OK;
  dispatch(s->d.order, s->d.nq, [&](auto P, auto NQ) {
    constexpr int p = decltype(P)::value, nq = decltype(NQ)::value;
    rc = timed(s, 0, st, [&]() {
      if (ch && cw)
        hipLaunchKernelGGL((k_reconstruct_char<p, nq, true>), dim3(blocks), threads, lds, st, a);
      else if (ch)
        hipLaunchKernelGGL((k_reconstruct_char<p, nq, false>), dim3(blocks), threads, lds, st, a);
      else if (cw)
        hipLaunchKernelGGL((k_reconstruct<p, nq, true>), dim3(blocks), threads, lds, st, a);
      else
        hipLaunchKernelGGL((k_reconstruct<p, nq, false>), dim3(blocks), threads, lds, st, a);
    });
  });
  return rc;
}

// next_dt (nullable, last stage only): the update also forms the CFL step of
// the state it produces (k_cell_update_dt, then k_dt_final) into *next_dt,
// with cfl next_cfl.
int launch_flux(teno_solver* s, const double* Un, const double* Uk, double* out,
                const double* dt, double ca, double cb, double cc, bool rk, hipStream_t st,
                const double* fp = nullptr, double* next_dt = nullptr, double next_cfl = 0.0) {
  FaceFluxArgs f;
  f.fp = fp ? fp : s->fp;
  f.fcell = s->fcell;
  f.fgeo = s->fgeo;
  f.phi = s->phi;
  f.bkind = s->bkind;
  f.bstate = s->bstate;
  f.gamma = s->prm.gamma;
  f.n_face = s->n_face;
  f.n_pad = s->n_pad;
  CellUpdateArgs c;
  c.cfaces = s->cfaces;
  c.vol = s->vol;
  c.phi = s->phi;
  c.Un = Un;
  c.Uk = Uk;
  c.out = out;
  c.dt = dt;
  c.ca = ca;
  c.cb = cb;
  c.cc = cc;
  c.n_cell = s->n_cell;
  const int fblocks = (s->n_face + 255) / 256;
  const int cblocks = (s->n_cell + 255) / 256;
  int rc = TENO_OK;
  auto go = [&](auto NQ) {
    rc = timed(s, 1, st, [&]() {
      hipLaunchKernelGGL((k_face_flux<decltype(NQ)::value>), dim3(fblocks), dim3(256), 0, st, f);
      if (s->n_bface > 0)
        hipLaunchKernelGGL((k_boundary_flux<decltype(NQ)::value>), dim3((s->n_bface + 255) / 256),
                           dim3(256), 0, st, f, (const int*)s->bface, s->n_bface);
      if (rk && next_dt) {
        hipLaunchKernelGGL(k_cell_update_dt, dim3(cblocks), dim3(256), 0, st, c,
                           (const double*)s->geo, s->prm.gamma, s->dtpart);
        hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, st, (const double*)s->dtpart,
                           cblocks, next_cfl, next_dt);
      } else if (rk)
        hipLaunchKernelGGL((k_cell_update<true>), dim3(cblocks), dim3(256), 0, st, c);
      else
        hipLaunchKernelGGL((k_cell_update<false>), dim3(cblocks), dim3(256), 0, st, c);
    });
  };
  if (s->d.nq == 2) go(IC<2>{});
  else go(IC<3>{});
  return rc;
}

int launch_dt(teno_solver* s, const double* U, double cfl, double* dt, hipStream_t st) {
  return timed(s, 2, st, [&]() {
    hipLaunchKernelGGL(k_dt_partial, dim3(s->n_dtblk), dim3(256), 0, st, U, s->geo, s->n_cell,
                       s->prm.gamma, s->dtpart);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, st, s->dtpart, s->n_dtblk, cfl, dt);
  });
}

// U_bar = scale * dt_scale * (dR/dU)^T lam + beta * extra, selection frozen.
// fp_in: the face states of U under `flags` (library layout) when the caller
// kept them from the forward pass; nullptr reconstructs them here.
int launch_vjp(teno_solver* s, const double* U, const uint16_t* flags, const double* lam,
               const double* scale_dev, double scale, const double* extra, double beta,
               double* out, hipStream_t st, const double* fp_in = nullptr) {
  int rc = TENO_OK;
  if (!fp_in) {
    rc = launch_reconstruct(s, U, const_cast<uint16_t*>(flags), true, st);
    if (rc) return rc;
  }
  AdjFaceArgs ff;
  ff.fp = fp_in ? fp_in : s->fp;
  ff.fcell = s->fcell;
  ff.fgeo = s->fgeo;
  ff.vol = s->vol;
  ff.lam = lam;
  ff.scale_dev = scale_dev;
  ff.scale = scale;
  ff.fpbar = s->fpbar;
  ff.bkind = s->bkind;
  ff.bstate = s->bstate;
  ff.gamma = s->prm.gamma;
  ff.n_face = s->n_face;
  ff.n_pad = s->n_pad;
  const int fblocks = (s->n_face + 255) / 256;
  AdjReconArgs ra;
  ra.fpbar = s->fpbar;
  ra.flags = flags;
  ra.M = s->M;
  ra.aslot = s->aslot;
  ra.tround = s->tround;
  ra.tbar = s->tbar;
  ra.ustride = s->ustride;
  ra.own = s->own;
  ra.n_cell = s->n_cell;
  ra.n_tiles = s->n_tiles;
  ra.n_pad = s->n_pad;
  const int tblocks = (s->n_tiles + kAdjBlockWaves - 1) / kAdjBlockWaves;
  const int qblocks = (int)(((int64_t)s->n_cell * 4 + 255) / 256);
  dispatch(s->d.order, s->d.nq, [&](auto P, auto NQ) {
    rc = timed(s, 3, st, [&]() {
      hipLaunchKernelGGL((k_adj_faces<decltype(NQ)::value>), dim3(fblocks), dim3(256), 0, st, ff);
      if (s->n_bface > 0)
        hipLaunchKernelGGL((k_adj_boundary<decltype(NQ)::value>), dim3((s->n_bface + 255) / 256),
                           dim3(256), 0, st, ff, (const int*)s->bface, s->n_bface);
      hipLaunchKernelGGL((k_adj_recon<decltype(P)::value, decltype(NQ)::value>), dim3(tblocks),
                         dim3(64 * kAdjBlockWaves),
                         (size_t)kAdjBlockWaves * s->ustride * 4 * sizeof(double), st, ra);
      hipLaunchKernelGGL(k_adj_gather, dim3(qblocks), dim3(256), 0, st, s->own, s->tbar,
                         s->rev_ptr, s->rev_ent, s->n_cell, extra, beta, out);
    });
  });
  return rc;
}

int lincomb(teno_solver* s, double* out, double a1, const double* x1, double a2, const double* x2,
            double a3, const double* x3, hipStream_t st) {
  const long n = (long)s->n_cell * 4;
  return timed(s, 3, st, [&]() {
    hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, a1,
                       x1, a2, x2, a3, x3, n);
  });
}

int check_solver(teno_solver* s) {
  if (!s) return fail(TENO_EARG, "null solver");
  return TENO_OK;
}

// CWENO (variant 2) has no selection to freeze and hence no adjoint; the
// frozen and adjoint paths work in conservative variables only.
int needs_selection(const teno_solver* s, const char* what) {
  if (s->prm.variant == 2)
    return fail(TENO_EARG, std::string(what) + " needs a stencil selection (TENO or LINEAR), not CWENO");
  if (s->prm.characteristic)
    return fail(TENO_EARG, std::string(what) + " works in conservative variables only");
  return TENO_OK;
}

}  // namespace

extern "C" {

const char* teno_last_error(void) { return teno::last_error(); }

void teno_default_params(teno_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->order = 5;
  p->n_quad = 0;
  p->variant = 0;
  p->power = 6;
  p->ct = 1e-6;
  p->eps = 1e-12;
  p->gamma = 1.4;
  p->tie_rel = 1e-10;
  p->fallback = 0;
  p->reorder = 1;
  p->n_threads = 0;
  p->dk_prime = 1e4;
}

int teno_mesh_create(int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri,
                     const double* period, teno_mesh** out) {
  if (!out) return fail(TENO_EARG, "null output");
  *out = nullptr;
  teno_mesh* m = new (std::nothrow) teno_mesh();
  if (!m) return fail(TENO_ENOMEM, "host allocation failed");
  int rc = mesh_create(n_vert, xy, n_cell, tri, period, m->m);
  if (rc) {
    delete m;
    return rc;
  }
  *out = m;
  return TENO_OK;
}

int teno_mesh_setup(teno_mesh* m, const teno_params* p) {
  if (!m || !p) return fail(TENO_EARG, "null argument");
  try {
    return mesh_setup(m->m, *p);
  } catch (const std::bad_alloc&) {
    return fail(TENO_ENOMEM, "host allocation failed during set-up");
  }
}

int teno_mesh_info(const teno_mesh* m, teno_info* out) {
  if (!m || !out) return fail(TENO_EARG, "null argument");
  const Mesh& x = m->m;
  std::memset(out, 0, sizeof(*out));
  out->n_cell = x.nc;
  out->n_face = x.nf;
  if (x.ready) {
    out->order = x.d.order;
    out->n_quad = x.d.nq;
    out->n_coef_large = x.d.nu;
    out->rows_large = x.d.nl;
    out->n_coef_small = kSmallCoef;
    out->rows_small = kSmallRows;
    out->matrix_doubles_per_cell = x.d.J;
    out->min_rcond = x.min_rcond;
    out->face_state_doubles = (int64_t)3 * x.d.nq * x.n_pad * 4;
  }
  out->n_bface = (int64_t)x.bface.size();
  return TENO_OK;
}

int teno_mesh_boundary_count(const teno_mesh* m, int32_t* n_bface) {
  if (!m || !n_bface) return fail(TENO_EARG, "null argument");
  *n_bface = (int32_t)m->m.bface.size();
  return TENO_OK;
}

int teno_mesh_boundary_faces(const teno_mesh* m, int32_t* verts, int32_t* cell) {
  if (!m || !verts) return fail(TENO_EARG, "null argument");
  const Mesh& x = m->m;
  for (size_t b = 0; b < x.bface.size(); ++b) {
    const int f = x.bface[b], i = x.fL[f], e = x.fLe[f];
    verts[2 * b] = x.tri[3 * (size_t)i + e];
    verts[2 * b + 1] = x.tri[3 * (size_t)i + (e + 1) % 3];
    if (cell) cell[b] = i;
  }
  return TENO_OK;
}

int teno_mesh_set_boundary(teno_mesh* m, const int32_t* kind, const double* state) {
  if (!m) return fail(TENO_EARG, "null argument");
  Mesh& x = m->m;
  const size_t nb = x.bface.size();
  if (nb == 0) return TENO_OK;
  if (!kind) return fail(TENO_EARG, "null argument");
  for (size_t b = 0; b < nb; ++b) {
    if (kind[b] < TENO_BC_TRANSMISSIVE || kind[b] > TENO_BC_PRESCRIBED)
      return fail(TENO_EARG, "boundary kind must be 1, 2 or 3 (face " + std::to_string(b) + ")");
    if (kind[b] == TENO_BC_PRESCRIBED && !state)
      return fail(TENO_EARG, "prescribed boundary faces need states");
  }
  x.bkind.assign(kind, kind + nb);
  x.bstate.assign(4 * nb, 0.0);
  if (state) std::copy(state, state + 4 * nb, x.bstate.begin());
  return TENO_OK;
}

int teno_mesh_permutation(const teno_mesh* m, int32_t* perm) {
  if (!m || !perm) return fail(TENO_EARG, "null argument");
  if (!m->m.ready) return fail(TENO_EARG, "teno_mesh_setup not called");
  std::memcpy(perm, m->m.perm.data(), sizeof(int32_t) * m->m.nc);
  return TENO_OK;
}

int teno_mesh_stencil(const teno_mesh* m, int32_t cell, int32_t k, int32_t* members) {
  if (!m || !members) return fail(TENO_EARG, "null argument");
  const Mesh& x = m->m;
  if (!x.ready) return fail(TENO_EARG, "teno_mesh_setup not called");
  if (cell < 0 || cell >= x.nc || k < 0 || k > 3) return fail(TENO_EARG, "cell or stencil out of range");
  const int t = x.inv[cell];
  const int nrow = k == 3 ? x.d.nl : kSmallRows;
  for (int s = 0; s < nrow; ++s)
    members[s] = x.perm[x.idx[packed_idx_index(x, t, k == 3 ? large_row(s) : small_row(k, s))]];
  return nrow;
}

int teno_mesh_lsq_operator(const teno_mesh* m, int32_t cell, int32_t k, double* M) {
  if (!m || !M) return fail(TENO_EARG, "null argument");
  const Mesh& x = m->m;
  if (!x.ready) return fail(TENO_EARG, "teno_mesh_setup not called");
  if (cell < 0 || cell >= x.nc || k < 0 || k > 3) return fail(TENO_EARG, "cell or stencil out of range");
  const int t = x.inv[cell];
  const bool big = k == 3;
  const int nrow = big ? x.d.nl : kSmallRows, nco = big ? x.d.nu : kSmallCoef;
  for (int l = 0; l < nco; ++l)
    for (int s = 0; s < nrow; ++s)
      M[(size_t)l * nrow + s] = x.M[packed_M_offset(x.d, t, k, s, l)];
  return nrow;
}

void teno_mesh_destroy(teno_mesh* m) { delete m; }

int teno_solver_create(const teno_mesh* mesh, int32_t device, teno_solver** out) {
  if (!mesh || !out) return fail(TENO_EARG, "null argument");
  *out = nullptr;
  const Mesh& m = mesh->m;
  if (!m.ready) return fail(TENO_EARG, "teno_mesh_setup not called");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(TENO_EHIP, "no HIP device");
  if (device < 0 || device >= ndev) return fail(TENO_EARG, "device out of range");
  bool ok_combo = dispatch(m.d.order, m.d.nq, [](auto, auto) {});
  if (!ok_combo) return fail(TENO_EARG, "unsupported order / face-point count");
  DeviceScope ds(device);
  if (!ds.ok) return fail(TENO_EHIP, "hipSetDevice failed");
  teno_solver* s = new (std::nothrow) teno_solver();
  if (!s) return fail(TENO_ENOMEM, "host allocation failed");
  s->device = device;
  s->d = m.d;
  s->prm = m.prm;
  s->n_cell = m.nc;
  s->n_pad = m.n_pad;
  s->n_tiles = m.n_tiles;
  s->n_dtblk = (m.nc + 255) / 256;
  const size_t np = m.n_pad, nc = m.nc;
  int rc = TENO_OK;
  auto A = [&](auto& p, size_t n) {
    if (rc == TENO_OK) rc = s->alloc(p, n);
  };
  s->ustride = m.ustride;
  A(s->slot, m.slot.size() / 8);
  A(s->aslot, m.aslot.size() / 8);
  A(s->tround, m.tround.size());
  A(s->tmem, m.tmem.size());
  A(s->M, m.M.size() / 2);
  A(s->nbinfo, np);
  s->n_face = m.nf;
  s->n_bface = (int)m.bface.size();
  A(s->bkind, std::max<size_t>(1, m.bkind.size()));
  A(s->bface, std::max<size_t>(1, m.bface_sorted.size()));
  A(s->bstate, std::max<size_t>(4, m.bstate.size()));
  A(s->fcell, (size_t)m.nf);
  A(s->fgeo, (size_t)m.nf * 2);
  A(s->cfaces, np);
  A(s->vol, np);
  A(s->phi, (size_t)m.nf * 4);
  A(s->geo, np * 10);
  A(s->user_of, np);
  A(s->rev_ptr, nc + 1);
  A(s->rev_ent, std::max<size_t>(1, m.rev_ent.size()));
  A(s->fp, (size_t)3 * m.d.nq * np * 4);
  A(s->fpbar, (size_t)3 * m.d.nq * np * 4);
  A(s->tbar, (size_t)m.n_tiles * m.ustride * 4);
  A(s->own, np * 4);
  A(s->W1, nc * 4);
  A(s->W2, nc * 4);
  A(s->T0, nc * 4);
  A(s->T1, nc * 4);
  A(s->T2, nc * 4);
  A(s->dtpart, (size_t)s->n_dtblk);
  A(s->diag, 1);
  if (rc) {
    delete s;
    return rc;
  }
  struct Up {
    void* dst;
    const void* src;
    size_t n;
  } ups[] = {{s->slot, m.slot.data(), m.slot.size() * sizeof(uint16_t)},
             {s->aslot, m.aslot.data(), m.aslot.size() * sizeof(uint16_t)},
             {s->tround, m.tround.data(), m.tround.size() * sizeof(int32_t)},
             {s->tmem, m.tmem.data(), m.tmem.size() * sizeof(int32_t)},
             {s->M, m.M.data(), m.M.size() * sizeof(double)},
             {s->nbinfo, m.nbinfo.data(), m.nbinfo.size() * sizeof(int32_t)},
             {s->bkind, m.bkind.data(), m.bkind.size() * sizeof(int32_t)},
             {s->bface, m.bface_sorted.data(), m.bface_sorted.size() * sizeof(int32_t)},
             {s->bstate, m.bstate.data(), m.bstate.size() * sizeof(double)},
             {s->fcell, m.face_cells.data(), m.face_cells.size() * sizeof(int32_t)},
             {s->fgeo, m.face_geo.data(), m.face_geo.size() * sizeof(double)},
             {s->cfaces, m.cell_faces.data(), m.cell_faces.size() * sizeof(int32_t)},
             {s->vol, m.vol.data(), m.vol.size() * sizeof(double)},
             {s->geo, m.geo.data(), m.geo.size() * sizeof(double)},
             {s->user_of, m.user_of.data(), m.user_of.size() * sizeof(int32_t)},
             {s->rev_ptr, m.rev_ptr.data(), m.rev_ptr.size() * sizeof(int32_t)},
             {s->rev_ent, m.rev_ent.data(), m.rev_ent.size() * sizeof(int32_t)}};
  for (auto& u : ups) {
    if (u.n == 0) continue;
    hipError_t e = hipMemcpy(u.dst, u.src, u.n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      delete s;
      return hip_fail(e, "hipMemcpy upload");
    }
  }
  hipLaunchKernelGGL(k_diag_reset, dim3(1), dim3(64), 0, 0, s->diag);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "solver initialisation");
  }
  *out = s;
  return TENO_OK;
}

void teno_solver_destroy(teno_solver* s) {
  if (!s) return;
  DeviceScope ds(s->device);
  delete s;
}

int teno_reconstruct(teno_solver* s, const double* U, double* face_states, uint16_t* flags,
                     void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (!U) return fail(TENO_EARG, "null state");
  DeviceScope ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = launch_reconstruct(s, U, flags, false, st);
  if (rc) return rc;
  if (face_states) {
    hipError_t e = hipMemcpy2DAsync(face_states, (size_t)s->n_cell * 32, s->fp,
                                    (size_t)s->n_pad * 32, (size_t)s->n_cell * 32,
                                    (size_t)3 * s->d.nq, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync");
  }
  return TENO_OK;
}

int teno_residual(teno_solver* s, const double* U, double* R, uint16_t* flags, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (!U || !R) return fail(TENO_EARG, "null state");
  DeviceScope ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = launch_reconstruct(s, U, flags, false, st);
  if (rc) return rc;
  return launch_flux(s, U, U, R, nullptr, 0, 0, 0, false, st);
}

int teno_residual_frozen(teno_solver* s, const double* U, double* R, const uint16_t* flags,
                         void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (int rc = needs_selection(s, "residual_frozen")) return rc;
  if (!U || !R || !flags) return fail(TENO_EARG, "null argument");
  DeviceScope ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = launch_reconstruct(s, U, const_cast<uint16_t*>(flags), true, st);
  if (rc) return rc;
  return launch_flux(s, U, U, R, nullptr, 0, 0, 0, false, st);
}

int teno_max_dt(teno_solver* s, const double* U, double cfl, double* dt_dev, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (!U || !dt_dev) return fail(TENO_EARG, "null argument");
  if (!(cfl > 0.0)) return fail(TENO_EARG, "cfl must be positive");
  DeviceScope ds(s->device);
  return launch_dt(s, U, cfl, dt_dev, (hipStream_t)stream);
}

static int stage_impl(teno_solver* s, int k, const double* Un, const double* Uk, double* Uk1,
                      const double* dt, uint16_t* flags, bool frozen, hipStream_t st,
                      double* fp = nullptr, double* next_dt = nullptr, double next_cfl = 0.0) {
  int rc = launch_reconstruct(s, Uk, flags, frozen, st, fp);
  if (rc) return rc;
  return launch_flux(s, Un, Uk, Uk1, dt, kStageA[k], kStageB[k], kStageC[k], true, st, fp,
                     next_dt, next_cfl);
}

int teno_rk_stage(teno_solver* s, int32_t k, const double* Un, const double* Uk, double* Uk1,
                  const double* dt_dev, uint16_t* flags, int32_t frozen, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (k < 0 || k > 2) return fail(TENO_EARG, "stage must be 0, 1 or 2");
  if (!Un || !Uk || !Uk1 || !dt_dev) return fail(TENO_EARG, "null argument");
  if (frozen && !flags) return fail(TENO_EARG, "frozen selection needs flags");
  if (frozen)
    if (int rc = needs_selection(s, "a frozen stage")) return rc;
  if (k == 0 && Uk != Un) return fail(TENO_EARG, "stage 0 needs Uk == Un");
  if (Uk1 == Uk && Uk != Un) return fail(TENO_EARG, "Uk1 must not alias Uk");
  DeviceScope ds(s->device);
  return stage_impl(s, k, Un, Uk, Uk1, dt_dev, flags, frozen != 0, (hipStream_t)stream);
}

int teno_rk_step(teno_solver* s, double* U, const double* dt_dev, uint16_t* flags3,
                 int32_t frozen, double* stages, double* face_states3, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (!U || !dt_dev) return fail(TENO_EARG, "null argument");
  if (frozen && !flags3) return fail(TENO_EARG, "frozen selection needs flags3");
  if (frozen)
    if (int rc = needs_selection(s, "a frozen step")) return rc;
  DeviceScope ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)s->n_cell;
  const size_t nb = n * 4 * sizeof(double);
  const size_t nfl = n * (s->prm.characteristic ? 3 : 1);  // flag words per stage
  auto fl = [&](int k) { return flags3 ? flags3 + (size_t)k * nfl : nullptr; };
  const size_t fsz = face_state_doubles(s);
  auto fs = [&](int k) { return face_states3 ? face_states3 + (size_t)k * fsz : nullptr; };
  if (stages) {
    hipError_t e = hipMemcpyAsync(stages, U, nb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  int rc = stage_impl(s, 0, U, U, s->W1, dt_dev, fl(0), frozen != 0, st, fs(0));
  if (rc) return rc;
  if (stages) {
    hipError_t e = hipMemcpyAsync(stages + n * 4, s->W1, nb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  rc = stage_impl(s, 1, U, s->W1, s->W2, dt_dev, fl(1), frozen != 0, st, fs(1));
  if (rc) return rc;
  if (stages) {
    hipError_t e = hipMemcpyAsync(stages + 2 * n * 4, s->W2, nb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  return stage_impl(s, 2, U, s->W2, U, dt_dev, fl(2), frozen != 0, st, fs(2));
}

int teno_rk_step_dt(teno_solver* s, double* U, double* dt_dev, double cfl, uint16_t* flags3,
                    void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (!U || !dt_dev) return fail(TENO_EARG, "null argument");
  if (!(cfl > 0.0)) return fail(TENO_EARG, "cfl must be positive");
  DeviceScope ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t nfl = (size_t)s->n_cell * (s->prm.characteristic ? 3 : 1);
  auto fl = [&](int k) { return flags3 ? flags3 + (size_t)k * nfl : nullptr; };
  int rc = stage_impl(s, 0, U, U, s->W1, dt_dev, fl(0), false, st);
  if (rc) return rc;
  rc = stage_impl(s, 1, U, s->W1, s->W2, dt_dev, fl(1), false, st);
  if (rc) return rc;
  return stage_impl(s, 2, U, s->W2, U, dt_dev, fl(2), false, st, nullptr, dt_dev, cfl);
}

int teno_vjp_residual(teno_solver* s, const double* U, const uint16_t* flags, const double* lam,
                      double* U_bar, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (int rc = needs_selection(s, "vjp_residual")) return rc;
  if (!U || !flags || !lam || !U_bar) return fail(TENO_EARG, "null argument");
  if (U_bar == lam) return fail(TENO_EARG, "U_bar must not alias lam");
  DeviceScope ds(s->device);
  return launch_vjp(s, U, flags, lam, nullptr, 1.0, nullptr, 0.0, U_bar, (hipStream_t)stream);
}

int teno_vjp_rk_step(teno_solver* s, const double* stages, const uint16_t* flags3,
                     const double* face_states3, const double* dt_dev, const double* lam_out,
                     double* lam_in, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (int rc = needs_selection(s, "vjp_rk_step")) return rc;
  if (!stages || !flags3 || !dt_dev || !lam_out || !lam_in) return fail(TENO_EARG, "null argument");
  DeviceScope ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)s->n_cell;
  const double* U0 = stages;
  const double* U1 = stages + n * 4;
  const double* U2 = stages + 2 * n * 4;
  const size_t fsz = face_state_doubles(s);
  auto fs = [&](int k) { return face_states3 ? face_states3 + (size_t)k * fsz : nullptr; };
  // U' = 1/3 U0 + 2/3 U2 + 2/3 dt R(U2)   ->  T2 = lam_2 (adjoint of U2)
  int rc = launch_vjp(s, U2, flags3 + 2 * n, lam_out, dt_dev, 2.0 / 3.0, lam_out, 2.0 / 3.0,
                      s->T2, st, fs(2));
  if (rc) return rc;
  // U2 = 3/4 U0 + 1/4 U1 + 1/4 dt R(U1)  ->  T1 = lam_1
  rc = launch_vjp(s, U1, flags3 + n, s->T2, dt_dev, 0.25, s->T2, 0.25, s->T1, st, fs(1));
  if (rc) return rc;
  // U1 = U0 + dt R(U0)                   ->  T0 = lam_1 + dt R'(U0)^T lam_1
  rc = launch_vjp(s, U0, flags3, s->T1, dt_dev, 1.0, s->T1, 1.0, s->T0, st, fs(0));
  if (rc) return rc;
  return lincomb(s, lam_in, 1.0 / 3.0, lam_out, 0.75, s->T2, 1.0, s->T0, st);
}

int teno_solver_set_boundary_states(teno_solver* s, const double* state_dev, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (s->n_bface == 0) return TENO_OK;
  if (!state_dev) return fail(TENO_EARG, "null argument");
  DeviceScope ds(s->device);
  hipError_t e = hipMemcpyAsync(s->bstate, state_dev, (size_t)s->n_bface * 4 * sizeof(double),
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  return TENO_OK;
}

int teno_diagnostics(teno_solver* s, teno_diag* out, int32_t reset, void* stream) {
  if (int rc = check_solver(s)) return rc;
  if (!out) return fail(TENO_EARG, "null argument");
  DeviceScope ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  DevDiag h;
  hipError_t e = hipMemcpyAsync(&h, s->diag, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "diagnostics read");
  out->nonphysical = (int64_t)h.nonphysical;
  out->near_ties = (int64_t)h.near_ties;
  out->fallbacks = (int64_t)h.fallbacks;
  out->first_bad_cell = h.first_bad == LLONG_MAX ? -1 : (int64_t)h.first_bad;
  if (reset) {
    hipLaunchKernelGGL(k_diag_reset, dim3(1), dim3(64), 0, st, s->diag);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "diagnostics reset");
  }
  return TENO_OK;
}

int teno_profile_enable(teno_solver* s, int32_t kinds) {
  if (int rc = check_solver(s)) return rc;
  s->prof = (unsigned)kinds & 0xFu;
  return TENO_OK;
}

int teno_profile_read(teno_solver* s, double* ms, int64_t* launches, int32_t reset) {
  if (int rc = check_solver(s)) return rc;
  DeviceScope ds(s->device);
  for (auto& e : s->evs) {
    hipError_t r = hipEventSynchronize(e.b);
    if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e.a, e.b);
    s->prof_ms[e.kind] += t;
    s->prof_n[e.kind] += 1;
    s->pool.push_back({e.a, e.b});
  }
  s->evs.clear();
  for (int k = 0; k < 4; ++k) {
    if (ms) ms[k] = s->prof_ms[k];
    if (launches) launches[k] = s->prof_n[k];
    if (reset) {
      s->prof_ms[k] = 0;
      s->prof_n[k] = 0;
    }
  }
  return TENO_OK;
}

// ===========================================================================
// batches
// ===========================================================================
}  // extern "C"

struct teno_batch {
  int device = 0;
  int n = 0;
  int n_cu = 256;
  std::vector<teno_solver*> sv;
  teno_batch_tuning tune{0, 8, 1, 1};
  // device data
  BatchMeshDev* meshes = nullptr;
  int2* items_r = nullptr;     // reconstruction items, all orders
  int* start_r = nullptr;      // wave starts per launch, concatenated
  int2* items_f = nullptr;     // face items (64-face chunks)
  int* start_f = nullptr;
  int2* items_c = nullptr;     // cell items (64-cell chunks)
  int* start_c = nullptr;
  int2* items_dt = nullptr;
  int* start_dt = nullptr;     // per mesh
  int2* items_b = nullptr;     // boundary-face items (64-face chunks)
  double* partial = nullptr;
  // launch plan: per reconstruction launch (pq, item offset, wave offset, waves)
  struct RLaunch {
    int pq, item0, wave0, n_waves;
    int lds_stride;  // LDS per wavefront in int4, the largest of the launch's meshes
  };
  std::vector<RLaunch> rplan;
  int n_waves_f = 0, n_waves_c = 0, n_items_dt = 0, n_items_b = 0;
  // graph of one step: its kernels read every pointer from the device
  // descriptors, so it stays valid while only the descriptors change
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // what the device descriptors were last written for
  bool desc_valid = false;
  std::vector<double*> desc_U;
  const double* desc_dt = nullptr;
  std::vector<uint16_t*> flags3;  // per mesh [3][n_cell] stage flags, or empty
  teno_batch_stats stats{0, 0, 0};
  std::vector<void*> allocs;

  template <class T>
  int alloc(T*& p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 256));
    if (e != hipSuccess) return fail(TENO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(q);
    p = (T*)q;
    return TENO_OK;
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  void free_plan() {
    for (void* q : allocs) (void)hipFree(q);
    allocs.clear();
    meshes = nullptr;
    desc_valid = false;
  }
  ~teno_batch() {
    drop_graph();
    free_plan();
  }
};

namespace {

// Splits items [0, n) with costs into `waves` contiguous ranges of nearly
// equal total cost; writes waves+1 starts.
// Splits items 0..n-1 into `waves` contiguous ranges of about equal cost;
// waves == 0 gives every item its own wavefront (the hardware then balances
// the load).  Returns the number of wavefronts.
int balanced_starts(const std::vector<double>& cost, int waves, std::vector<int>& starts) {
  const int n = (int)cost.size();
  if (waves == 0) {
    starts.resize(n + 1);
    for (int i = 0; i <= n; ++i) starts[i] = i;
    return n;
  }
  double total = 0.0;
  for (double c : cost) total += c;
  starts.assign(waves + 1, n);
  starts[0] = 0;
  double acc = 0.0;
  int w = 1;
  for (int i = 0; i < n && w < waves; ++i) {
    acc += cost[i];
    while (w < waves && acc >= total * w / waves) starts[w++] = i + 1;
  }
  for (; w < waves; ++w) starts[w] = n;
  starts[waves] = n;
  return waves;
}

int batch_plan(teno_batch* b) {
  b->drop_graph();
  b->free_plan();
  const int n = b->n;
  const teno_batch_tuning& T = b->tune;
  const int waves = T.waves_per_cu * b->n_cu;  // 0: one wavefront per item
  // mesh order for the work list
  std::vector<int> morder(n);
  for (int m = 0; m < n; ++m) morder[m] = m;
  if (T.item_order == 1)
    std::stable_sort(morder.begin(), morder.end(), [&](int x, int y) {
      return b->sv[x]->d.Jp > b->sv[y]->d.Jp;
    });
  // reconstruction items, grouped per launch
  std::vector<int2> items;
  std::vector<int> starts_all;
  b->rplan.clear();
  std::vector<int> pqs;
  if (T.order_mode == 1) {
    for (int m : morder) {
      int pq = b->sv[m]->d.order * 10 + b->sv[m]->d.nq;
      if (std::find(pqs.begin(), pqs.end(), pq) == pqs.end()) pqs.push_back(pq);
    }
  } else {
    pqs.push_back(0);
  }
  for (int pq : pqs) {
    std::vector<double> cost;
    const int item0 = (int)items.size();
    int lds_stride = 0;
    for (int m : morder) {
      const teno_solver* s = b->sv[m];
      const int mpq = s->d.order * 10 + s->d.nq;
      if (pq != 0 && mpq != pq) continue;
      lds_stride = std::max(lds_stride, stage_int4(s->d.rows4, s->ustride));
      for (int t = 0; t < s->n_tiles; ++t) {
        items.push_back(make_int2(m, t));
        cost.push_back((double)s->d.Jp + 4.0 * s->d.rows4 * 4);
      }
    }
    std::vector<int> st;
    const int nw = balanced_starts(cost, waves, st);
    for (int& x : st) x += item0;
    b->rplan.push_back({pq, item0, (int)starts_all.size(), nw, lds_stride});
    starts_all.insert(starts_all.end(), st.begin(), st.end());
  }
  // face items (64-face chunks), cell items (64-cell chunks) and dt items
  // (256-cell blocks)
  std::vector<int2> fitems, citems, ditems;
  std::vector<double> fcost, ccost;
  std::vector<int> dstart(n + 1, 0);
  for (int m : morder) {
    const teno_solver* s = b->sv[m];
    for (int u = 0; u < (s->n_face + 63) / 64; ++u) {
      fitems.push_back(make_int2(m, u));
      fcost.push_back((double)s->d.nq);
    }
    for (int u = 0; u < (s->n_cell + 63) / 64; ++u) {
      citems.push_back(make_int2(m, u));
      ccost.push_back(1.0);
    }
  }
  std::vector<int2> bitems;
  for (int m : morder)
    for (int u = 0; u < (b->sv[m]->n_bface + 63) / 64; ++u) bitems.push_back(make_int2(m, u));
  b->n_items_b = (int)bitems.size();
  for (int m = 0; m < n; ++m) {
    dstart[m] = (int)ditems.size();
    for (int u = 0; u < (b->sv[m]->n_cell + 255) / 256; ++u) ditems.push_back(make_int2(m, u));
  }
  dstart[n] = (int)ditems.size();
  std::vector<int> fstart, cstart;
  b->n_waves_f = balanced_starts(fcost, waves, fstart);
  b->n_waves_c = balanced_starts(ccost, waves, cstart);
  b->n_items_dt = (int)ditems.size();
  int rc = TENO_OK;
  auto A = [&](auto& p, size_t c) {
    if (rc == TENO_OK) rc = b->alloc(p, c);
  };
  A(b->meshes, (size_t)n);
  A(b->items_r, items.size());
  A(b->start_r, starts_all.size());
  A(b->items_f, fitems.size());
  A(b->start_f, fstart.size());
  A(b->items_c, citems.size());
  A(b->start_c, cstart.size());
  A(b->items_dt, ditems.size());
  A(b->start_dt, dstart.size());
  A(b->partial, ditems.size());
  A(b->items_b, bitems.size());
  if (rc) return rc;
  struct Up {
    void* d;
    const void* h;
    size_t bytes;
  } ups[] = {{b->items_r, items.data(), items.size() * sizeof(int2)},
             {b->start_r, starts_all.data(), starts_all.size() * sizeof(int)},
             {b->items_f, fitems.data(), fitems.size() * sizeof(int2)},
             {b->start_f, fstart.data(), fstart.size() * sizeof(int)},
             {b->items_c, citems.data(), citems.size() * sizeof(int2)},
             {b->start_c, cstart.data(), cstart.size() * sizeof(int)},
             {b->items_dt, ditems.data(), ditems.size() * sizeof(int2)},
             {b->start_dt, dstart.data(), dstart.size() * sizeof(int)},
             {b->items_b, bitems.data(), bitems.size() * sizeof(int2)}};
  for (auto& u : ups) {
    if (u.bytes == 0) continue;
    hipError_t e = hipMemcpy(u.d, u.h, u.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
  }
  return TENO_OK;
}

// Makes the per-mesh descriptors describe state pointers U[m] and steps
// dt[m].  They are rewritten (a host-to-device copy and a wait on the
// stream) only when these pointers, the flag buffers or the plan changed
// since the last write; a step loop over the same buffers writes them once.
int batch_descriptors(teno_batch* b, double* const* U, const double* dt, hipStream_t st) {
  if (b->desc_valid && b->desc_dt == dt && (int)b->desc_U.size() == b->n &&
      std::equal(U, U + b->n, b->desc_U.begin()))
    return TENO_OK;
  std::vector<BatchMeshDev> h(b->n);
  for (int m = 0; m < b->n; ++m) {
    teno_solver* s = b->sv[m];
    BatchMeshDev& d = h[m];
    std::memset(&d, 0, sizeof(d));
    const double* in[3] = {U[m], s->W1, s->W2};
    double* out[3] = {s->W1, s->W2, U[m]};
    for (int k = 0; k < 3; ++k) {
      ReconArgs& a = d.r[k];
      a.U = in[k];
      a.slot = s->slot;
      a.tmem = s->tmem;
      a.ustride = s->ustride;
      a.lds_stride = stage_int4(s->d.rows4, s->ustride);
      a.M = s->M;
      a.fp = s->fp;
      a.flags = nullptr;
      a.user_of = s->user_of;
      a.geo = s->geo;
      a.nbinfo = s->nbinfo;
      a.diag = s->diag;
      a.n_cell = s->n_cell;
      a.n_tiles = s->n_tiles;
      a.n_pad = s->n_pad;
      a.flags = b->flags3.empty() ? nullptr : b->flags3[m] + (size_t)k * s->n_cell;
      a.frozen = 0;
      a.variant = s->prm.variant;
      a.fallback = s->prm.fallback;
      a.power = s->prm.power;
      a.ct = s->prm.ct;
      a.eps = s->prm.eps;
      a.gamma = s->prm.gamma;
      a.tie_rel = s->prm.tie_rel;
      set_tie_window(a);
      CellUpdateArgs& c = d.cu[k];
      c.cfaces = s->cfaces;
      c.vol = s->vol;
      c.phi = s->phi;
      c.Un = U[m];
      c.Uk = in[k];
      c.out = out[k];
      c.dt = dt ? dt + m : nullptr;
      c.ca = kStageA[k];
      c.cb = kStageB[k];
      c.cc = kStageC[k];
      c.n_cell = s->n_cell;
    }
    FaceFluxArgs& f = d.ff;
    f.fp = s->fp;
    f.fcell = s->fcell;
    f.fgeo = s->fgeo;
    f.phi = s->phi;
    f.bkind = s->bkind;
    f.bstate = s->bstate;
    f.gamma = s->prm.gamma;
    f.n_face = s->n_face;
    f.n_pad = s->n_pad;
    d.U = U[m];
    d.geo = s->geo;
    d.dt = dt ? const_cast<double*>(dt) + m : nullptr;
    d.gamma = s->prm.gamma;
    d.pq = s->d.order * 10 + s->d.nq;
    d.n_cell = s->n_cell;
    d.bface = s->bface;
    d.n_bface = s->n_bface;
  }
  // the host copy is freed on return, so the stream waits for the copy
  hipError_t e = hipMemcpyAsync(b->meshes, h.data(), h.size() * sizeof(BatchMeshDev),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    b->desc_valid = false;
    return hip_fail(e, "batch descriptors");
  }
  b->desc_U.assign(U, U + b->n);
  b->desc_dt = dt;
  b->desc_valid = true;
  b->stats.descriptor_writes++;
  return TENO_OK;
}

void batch_launch_recon(teno_batch* b, int k, hipStream_t st) {
  for (const auto& L : b->rplan) {
    // one wavefront per item: the loop-free kernel over this launch's items,
    // in blocks of kReconBlockWaves wavefronts; the persistent kernel in
    // blocks of four
    const bool one = b->tune.waves_per_cu == 0;
    const int bw = one ? kReconBlockWaves : 4;
    const int blocks = (L.n_waves + bw - 1) / bw;
    const int* ws = b->start_r + L.wave0;
    const size_t lds = (size_t)bw * L.lds_stride * sizeof(int4);
    const int2* its = b->items_r + L.item0;
    switch (L.pq) {
#define TENO_BATCH_CASE(PQ)                                                                  \
  case PQ:                                                                                   \
    if (one)                                                                                 \
      hipLaunchKernelGGL((k_batch_reconstruct_one<PQ>), dim3(blocks), dim3(64 * bw), lds, st, \
                         b->meshes, its, L.n_waves, k, L.lds_stride);                        \
    else                                                                                     \
      hipLaunchKernelGGL((k_batch_reconstruct<PQ>), dim3(blocks), dim3(256), lds, st,        \
                         b->meshes, b->items_r, ws, L.n_waves, k, L.lds_stride);             \
    break;
      TENO_BATCH_CASE(0)
      TENO_BATCH_CASE(32)
      TENO_BATCH_CASE(33)
      TENO_BATCH_CASE(42)
      TENO_BATCH_CASE(43)
      TENO_BATCH_CASE(52)
      TENO_BATCH_CASE(53)
      TENO_BATCH_CASE(62)
      TENO_BATCH_CASE(63)
#undef TENO_BATCH_CASE
      default: break;
    }
  }
}

void batch_launch_step(teno_batch* b, hipStream_t st) {
  const int fblocks = (b->n_waves_f + 3) / 4;
  const int cblocks = (b->n_waves_c + 3) / 4;
  for (int k = 0; k < 3; ++k) {
    batch_launch_recon(b, k, st);
    hipLaunchKernelGGL(k_batch_face_flux, dim3(fblocks), dim3(256), 0, st, b->meshes, b->items_f,
                       b->start_f, b->n_waves_f);
    if (b->n_items_b > 0)
      hipLaunchKernelGGL(k_batch_boundary_flux, dim3((b->n_items_b + 3) / 4), dim3(256), 0, st,
                         b->meshes, b->items_b, b->n_items_b);
    hipLaunchKernelGGL(k_batch_cell_update, dim3(cblocks), dim3(256), 0, st, b->meshes,
                       b->items_c, b->start_c, b->n_waves_c, k);
  }
}

}  // namespace

extern "C" {

int teno_batch_create(teno_solver* const* solvers, int32_t n, teno_batch** out) {
  if (!solvers || !out || n <= 0) return fail(TENO_EARG, "empty batch");
  *out = nullptr;
  for (int m = 0; m < n; ++m) {
    if (!solvers[m]) return fail(TENO_EARG, "null solver in batch");
    if (solvers[m]->device != solvers[0]->device) return fail(TENO_EARG, "batch solvers must share a device");
    for (int k = 0; k < m; ++k)
      if (solvers[k] == solvers[m]) return fail(TENO_EARG, "a solver appears twice in the batch");
    if (solvers[m]->prm.variant == 2) return fail(TENO_EARG, "CWENO meshes cannot be batched");
    if (solvers[m]->prm.characteristic)
      return fail(TENO_EARG, "meshes in characteristic variables cannot be batched");
  }
  DeviceScope ds(solvers[0]->device);
  teno_batch* b = new (std::nothrow) teno_batch();
  if (!b) return fail(TENO_ENOMEM, "host allocation failed");
  b->device = solvers[0]->device;
  b->n = n;
  b->sv.assign(solvers, solvers + n);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess &&
      cus > 0)
    b->n_cu = cus;
  int rc = batch_plan(b);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return TENO_OK;
}

int teno_batch_set_tuning(teno_batch* b, const teno_batch_tuning* t) {
  if (!b || !t) return fail(TENO_EARG, "null argument");
  if (t->order_mode < 0 || t->order_mode > 1 || t->item_order < 0 || t->item_order > 1 ||
      t->waves_per_cu < 0 || t->waves_per_cu > 32 || t->use_graph < 0 || t->use_graph > 1)
    return fail(TENO_EARG, "tuning out of range");
  DeviceScope ds(b->device);
  b->tune = *t;
  return batch_plan(b);
}

int teno_batch_get_tuning(const teno_batch* b, teno_batch_tuning* t) {
  if (!b || !t) return fail(TENO_EARG, "null argument");
  *t = b->tune;
  return TENO_OK;
}

int teno_batch_max_dt(teno_batch* b, double* const* U, double cfl, double* dt_dev, void* stream) {
  if (!b || !U || !dt_dev) return fail(TENO_EARG, "null argument");
  if (!(cfl > 0.0)) return fail(TENO_EARG, "cfl must be positive");
  for (int m = 0; m < b->n; ++m)
    if (!U[m]) return fail(TENO_EARG, "null state pointer");
  DeviceScope ds(b->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = batch_descriptors(b, U, dt_dev, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_batch_dt_partial, dim3(b->n_items_dt), dim3(256), 0, st, b->meshes,
                     b->items_dt, b->partial);
  hipLaunchKernelGGL(k_batch_dt_final, dim3(b->n), dim3(256), 0, st, b->meshes, b->start_dt,
                     b->partial, cfl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "batch dt launch");
  return TENO_OK;
}

int teno_batch_rk_step(teno_batch* b, double* const* U, const double* dt_dev, void* stream) {
  if (!b || !U || !dt_dev) return fail(TENO_EARG, "null argument");
  for (int m = 0; m < b->n; ++m)
    if (!U[m]) return fail(TENO_EARG, "null state pointer");
  DeviceScope ds(b->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = batch_descriptors(b, U, dt_dev, st);
  if (rc) return rc;
  if (b->tune.use_graph && !b->exec) {
    if (st == nullptr) return fail(TENO_EARG, "graph capture needs a non-default stream");
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    batch_launch_step(b, st);
    e = hipStreamEndCapture(st, &b->graph);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      b->drop_graph();
      return hip_fail(e, "hipGraphInstantiate");
    }
    b->stats.captures++;
  }
  if (b->tune.use_graph) {
    hipError_t e = hipGraphLaunch(b->exec, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    b->stats.replays++;
  } else {
    batch_launch_step(b, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch launch");
  }
  return TENO_OK;
}

int teno_batch_set_flags(teno_batch* b, uint16_t* const* flags3) {
  if (!b) return fail(TENO_EARG, "null argument");
  if (flags3)
    for (int m = 0; m < b->n; ++m)
      if (!flags3[m]) return fail(TENO_EARG, "null flag pointer");
  if (flags3)
    b->flags3.assign(flags3, flags3 + b->n);
  else
    b->flags3.clear();
  b->desc_valid = false;  // the next call writes them into the descriptors
  return TENO_OK;
}

int teno_batch_get_stats(const teno_batch* b, teno_batch_stats* out) {
  if (!b || !out) return fail(TENO_EARG, "null argument");
  *out = b->stats;
  return TENO_OK;
}

void teno_batch_destroy(teno_batch* b) {
  if (!b) return;
  DeviceScope ds(b->device);
  delete b;
}

}  // extern "C"

// allocation-free entry point (its own static device scratch)
#include "noalloc.inc"
