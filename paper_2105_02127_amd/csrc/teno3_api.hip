// C ABI of the tetrahedral path (include/teno3.h): argument checks, device
// buffers and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/teno3.h"
#include "internal3.h"
#include "kernels3.hpp"

using namespace teno;
using namespace teno::t3;

namespace {

struct DevScope3 {
  int prev = -1;
  bool ok = true;
  explicit DevScope3(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DevScope3() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int hip_fail3(hipError_t e, const char* what) {
  return fail(TENO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

const double kA3[3] = {1.0, 0.75, 1.0 / 3.0};
const double kB3[3] = {0.0, 0.25, 2.0 / 3.0};
const double kC3[3] = {1.0, 0.25, 2.0 / 3.0};

}  // namespace

struct teno3_solver {
  int device = 0;
  Dims3 d;
  teno_params prm{};
  int n_cell = 0, n_pad = 0, n_tiles = 0, n_face = 0, n_bface = 0, n_dtblk = 0;
  double w[7] = {0, 0, 0, 0, 0, 0, 0};
  int32_t* idx = nullptr;
  double2* M = nullptr;
  double* tab = nullptr;  // psi, packed large form, packed small form
  int4* fcell = nullptr;
  double4* fgeo = nullptr;
  int* bkind = nullptr;
  int4* cfaces = nullptr;
  int* cside = nullptr;
  double* geo = nullptr;
  double* vol = nullptr;
  int32_t* user_of = nullptr;
  double* fp = nullptr;
  double* phi = nullptr;
  double* W1 = nullptr;
  double* W2 = nullptr;
  double* dtpart = nullptr;
  Diag3* diag = nullptr;
  std::vector<void*> allocs;
  unsigned prof = 0;
  struct Ev {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Ev> evs;
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_n[3] = {0, 0, 0};

  template <class T>
  int alloc(T*& p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 256));
    if (e != hipSuccess) return fail(TENO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(q);
    p = (T*)q;
    return TENO_OK;
  }
  ~teno3_solver() {
    for (auto& e : evs) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (void* q : allocs) (void)hipFree(q);
  }
};

namespace {

template <class F>
int timed3(teno3_solver* s, int kind, hipStream_t st, F&& launch) {
  const bool on = (s->prof >> kind) & 1;
  hipEvent_t a = nullptr, b = nullptr;
  if (on) {
    if (hipEventCreate(&a) != hipSuccess) return fail(TENO_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return fail(TENO_EHIP, "hipEventCreate failed");
    }
    (void)hipEventRecord(a, st);
  }
  launch();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (on) {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
    return hip_fail3(e, "kernel launch");
  }
  if (on) {
    (void)hipEventRecord(b, st);
    s->evs.push_back({kind, a, b});
  }
  return TENO_OK;
}

int launch_recon3(teno3_solver* s, const double* U, uint32_t* flags, hipStream_t st) {
  Recon3Args a;
  a.U = U;
  a.idx = s->idx;
  a.M = s->M;
  a.tab = s->tab;
  a.fp = s->fp;
  a.flags = flags;
  a.user_of = s->user_of;
  a.diag = s->diag;
  a.n_cell = s->n_cell;
  a.n_tiles = s->n_tiles;
  a.n_pad = s->n_pad;
  a.variant = s->prm.variant;
  a.fallback = s->prm.fallback;
  a.power = s->prm.power;
  a.ct = s->prm.ct;
  a.eps = s->prm.eps;
  a.gamma = s->prm.gamma;
  if (s->prm.ct > 0.0) {
    a.tie_lo = s->prm.ct * (1.0 - s->prm.tie_rel);
    a.tie_hi = s->prm.ct * (1.0 + s->prm.tie_rel);
  } else {
    a.tie_lo = 1.0;
    a.tie_hi = 0.0;
  }
  const int blocks = (s->n_tiles + 3) / 4;
  return timed3(s, 0, st, [&]() {
    switch (s->d.order) {
      case 3: hipLaunchKernelGGL(k_reconstruct3<3>, dim3(blocks), dim3(256), 0, st, a); break;
      case 4: hipLaunchKernelGGL(k_reconstruct3<4>, dim3(blocks), dim3(256), 0, st, a); break;
      case 5: hipLaunchKernelGGL(k_reconstruct3<5>, dim3(blocks), dim3(256), 0, st, a); break;
      default: hipLaunchKernelGGL(k_reconstruct3<6>, dim3(blocks), dim3(256), 0, st, a); break;
    }
  });
}

int launch_flux3(teno3_solver* s, const double* Un, const double* Uk, double* out, const double* dt,
                 int k, bool rk, hipStream_t st) {
  Flux3Args f;
  f.fp = s->fp;
  f.fcell = s->fcell;
  f.fgeo = s->fgeo;
  f.bkind = s->bkind;
  f.phi = s->phi;
  std::memcpy(f.w, s->w, sizeof(f.w));
  f.gamma = s->prm.gamma;
  f.n_face = s->n_face;
  f.n_pad = s->n_pad;
  Update3Args c;
  c.cfaces = s->cfaces;
  c.cside = s->cside;
  c.vol = s->vol;
  c.phi = s->phi;
  c.Un = Un;
  c.Uk = Uk;
  c.out = out;
  c.dt = dt;
  c.ca = rk ? kA3[k] : 0.0;
  c.cb = rk ? kB3[k] : 0.0;
  c.cc = rk ? kC3[k] : 0.0;
  c.n_cell = s->n_cell;
  c.rk = rk ? 1 : 0;
  const int fb = (s->n_face + 255) / 256, cb = (s->n_cell + 255) / 256;
  return timed3(s, 1, st, [&]() {
    if (s->d.npt == 6)
      hipLaunchKernelGGL(k_face_flux3<6>, dim3(fb), dim3(256), 0, st, f);
    else
      hipLaunchKernelGGL(k_face_flux3<7>, dim3(fb), dim3(256), 0, st, f);
    hipLaunchKernelGGL(k_cell_update3, dim3(cb), dim3(256), 0, st, c);
  });
}

int check3(teno3_solver* s) {
  if (!s) return fail(TENO_EARG, "null solver");
  return TENO_OK;
}

}  // namespace

extern "C" {

int teno3_mesh_create(int32_t n_vert, const double* xyz, int32_t n_cell, const int32_t* tet,
                      const double* period, teno3_mesh** out) {
  if (!out) return fail(TENO_EARG, "null output");
  *out = nullptr;
  teno3_mesh* m = new (std::nothrow) teno3_mesh();
  if (!m) return fail(TENO_ENOMEM, "host allocation failed");
  int rc;
  try {
    rc = mesh3_create(n_vert, xyz, n_cell, tet, period, m->m);
  } catch (const std::bad_alloc&) {
    rc = fail(TENO_ENOMEM, "host allocation failed");
  }
  if (rc) {
    delete m;
    return rc;
  }
  *out = m;
  return TENO_OK;
}

int teno3_mesh_boundary_count(const teno3_mesh* m, int32_t* n_bface) {
  if (!m || !n_bface) return fail(TENO_EARG, "null argument");
  *n_bface = (int32_t)m->m.bface.size();
  return TENO_OK;
}

int teno3_mesh_boundary_faces(const teno3_mesh* m, int32_t* verts, int32_t* cell) {
  if (!m || !verts) return fail(TENO_EARG, "null argument");
  const Mesh3& x = m->m;
  for (size_t b = 0; b < x.bface.size(); ++b) {
    const int f = x.bface[b], i = x.fL[f], e = x.fLe[f];
    for (int j = 0; j < 3; ++j) verts[3 * b + j] = x.tet[4 * (size_t)i + kFaceVerts3[e][j]];
    if (cell) cell[b] = i;
  }
  return TENO_OK;
}

int teno3_mesh_set_boundary(teno3_mesh* m, const int32_t* kind) {
  if (!m) return fail(TENO_EARG, "null argument");
  Mesh3& x = m->m;
  if (x.bface.empty()) return TENO_OK;
  if (!kind) return fail(TENO_EARG, "null argument");
  for (size_t b = 0; b < x.bface.size(); ++b)
    if (kind[b] != TENO_BC_TRANSMISSIVE && kind[b] != TENO_BC_REFLECTIVE)
      return fail(TENO_EARG, "tetrahedra: boundary kind must be transmissive or reflective");
  x.bkind.assign(kind, kind + x.bface.size());
  x.bkind_sorted = x.bkind;
  return TENO_OK;
}

int teno3_mesh_setup(teno3_mesh* m, const teno_params* p) {
  if (!m || !p) return fail(TENO_EARG, "null argument");
  try {
    return mesh3_setup(m->m, *p);
  } catch (const std::bad_alloc&) {
    return fail(TENO_ENOMEM, "host allocation failed during set-up");
  }
}

int teno3_mesh_info(const teno3_mesh* m, teno_info* out) {
  if (!m || !out) return fail(TENO_EARG, "null argument");
  const Mesh3& x = m->m;
  std::memset(out, 0, sizeof(*out));
  out->n_cell = x.nc;
  out->n_face = x.nf;
  out->n_bface = (int64_t)x.bface.size();
  if (x.ready) {
    out->order = x.d.order;
    out->n_quad = x.d.npt;
    out->n_coef_large = x.d.nu;
    out->rows_large = x.d.nl;
    out->n_coef_small = kSmall3Coef;
    out->rows_small = kSmall3Rows;
    out->matrix_doubles_per_cell = 4 * kSmall3Coef * kSmall3Rows + (int64_t)x.d.nu * x.d.nl;
    out->min_rcond = x.min_rcond;
    out->face_state_doubles = (int64_t)4 * x.d.npt * x.n_pad * 5;
  }
  return TENO_OK;
}

int teno3_mesh_permutation(const teno3_mesh* m, int32_t* perm) {
  if (!m || !perm) return fail(TENO_EARG, "null argument");
  if (!m->m.ready) return fail(TENO_EARG, "teno3_mesh_setup not called");
  std::memcpy(perm, m->m.perm.data(), sizeof(int32_t) * m->m.nc);
  return TENO_OK;
}

int teno3_mesh_stencil(const teno3_mesh* m, int32_t cell, int32_t k, int32_t* members) {
  if (!m || !members) return fail(TENO_EARG, "null argument");
  const Mesh3& x = m->m;
  if (!x.ready) return fail(TENO_EARG, "teno3_mesh_setup not called");
  if (cell < 0 || cell >= x.nc || k < 0 || k > 4) return fail(TENO_EARG, "cell or stencil out of range");
  const int t = x.inv[cell], tile = t / kTile3, c = t % kTile3;
  const int nrow = k == 4 ? x.d.nl : kSmall3Rows, row0 = k == 4 ? 4 * kSmall3Rows : k * kSmall3Rows;
  for (int s = 0; s < nrow; ++s)
    members[s] = x.perm[x.idx[((size_t)tile * x.d.rows + row0 + s) * kTile3 + c]];
  return nrow;
}

int teno3_mesh_lsq_operator(const teno3_mesh* m, int32_t cell, int32_t k, double* M) {
  if (!m || !M) return fail(TENO_EARG, "null argument");
  const Mesh3& x = m->m;
  if (!x.ready) return fail(TENO_EARG, "teno3_mesh_setup not called");
  if (cell < 0 || cell >= x.nc || k < 0 || k > 4) return fail(TENO_EARG, "cell or stencil out of range");
  const int t = x.inv[cell], tile = t / kTile3, c = t % kTile3;
  const bool big = k == 4;
  const int nrow = big ? x.d.nl : kSmall3Rows, nco = big ? x.d.nu : kSmall3Coef;
  const int rs = big ? x.d.rsl : kSmall3Stored, j0 = big ? 4 * kSmall3Blk : k * kSmall3Blk;
  for (int l = 0; l < nco; ++l)
    for (int s = 0; s < nrow; ++s) {
      const int j = j0 + s * rs + l;
      M[(size_t)l * nrow + s] = x.M[(((size_t)tile * (x.d.jp / 2) + j / 2) * kTile3 + c) * 2 + (j & 1)];
    }
  return nrow;
}

void teno3_mesh_destroy(teno3_mesh* m) { delete m; }

int teno3_solver_create(const teno3_mesh* mesh, int32_t device, teno3_solver** out) {
  if (!mesh || !out) return fail(TENO_EARG, "null argument");
  *out = nullptr;
  const Mesh3& m = mesh->m;
  if (!m.ready) return fail(TENO_EARG, "teno3_mesh_setup not called");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(TENO_EHIP, "no HIP device");
  if (device < 0 || device >= ndev) return fail(TENO_EARG, "device out of range");
  DevScope3 ds(device);
  if (!ds.ok) return fail(TENO_EHIP, "hipSetDevice failed");
  teno3_solver* s = new (std::nothrow) teno3_solver();
  if (!s) return fail(TENO_ENOMEM, "host allocation failed");
  s->device = device;
  s->d = m.d;
  s->prm = m.prm;
  s->n_cell = m.nc;
  s->n_pad = m.n_pad;
  s->n_tiles = m.n_tiles;
  s->n_face = m.nf;
  s->n_bface = (int)m.bface.size();
  s->n_dtblk = (m.nc + 255) / 256;
  double bary[7][3];
  face_rule3(m.d.order, bary, s->w);
  const size_t np = m.n_pad;
  int rc = TENO_OK;
  auto A = [&](auto& p, size_t n) {
    if (rc == TENO_OK) rc = s->alloc(p, n);
  };
  A(s->idx, m.idx.size());
  A(s->M, m.M.size() / 2);
  // psi, then the two smoothness forms packed by rows of their upper
  // triangles with doubled off-diagonal entries (the kernels' layout)
  std::vector<double> tab(m.psi);
  auto pack = [&](const std::vector<double>& B, int n) {
    for (int l = 0; l < n; ++l)
      for (int c = l; c < n; ++c) tab.push_back(c == l ? B[(size_t)l * n + c] : 2.0 * B[(size_t)l * n + c]);
  };
  pack(m.Blarge, m.d.nu);
  pack(m.Bsmall, kSmall3Coef);
  A(s->tab, tab.size());
  A(s->fcell, (size_t)m.nf);
  A(s->fgeo, (size_t)m.nf);
  A(s->bkind, std::max<size_t>(1, m.bkind_sorted.size()));
  A(s->cfaces, np);
  A(s->cside, np);
  A(s->geo, np * 17);
  A(s->vol, np);
  A(s->user_of, np);
  A(s->fp, (size_t)4 * m.d.npt * np * 5);
  A(s->phi, (size_t)m.nf * 5);
  A(s->W1, (size_t)m.nc * 5);
  A(s->W2, (size_t)m.nc * 5);
  A(s->dtpart, (size_t)s->n_dtblk);
  A(s->diag, 1);
  if (rc) {
    delete s;
    return rc;
  }
  std::vector<double> vol(np);
  for (size_t t = 0; t < np; ++t) vol[t] = m.geo[t * 17 + 16];
  struct Up {
    void* dst;
    const void* src;
    size_t n;
  } ups[] = {{s->idx, m.idx.data(), m.idx.size() * sizeof(int32_t)},
             {s->M, m.M.data(), m.M.size() * sizeof(double)},
             {s->tab, tab.data(), tab.size() * sizeof(double)},
             {s->fcell, m.face_cells.data(), m.face_cells.size() * sizeof(int32_t)},
             {s->fgeo, m.face_geo.data(), m.face_geo.size() * sizeof(double)},
             {s->bkind, m.bkind_sorted.data(), m.bkind_sorted.size() * sizeof(int32_t)},
             {s->cfaces, m.cell_faces.data(), m.cell_faces.size() * sizeof(int32_t)},
             {s->cside, m.cell_side.data(), m.cell_side.size() * sizeof(int32_t)},
             {s->geo, m.geo.data(), m.geo.size() * sizeof(double)},
             {s->vol, vol.data(), vol.size() * sizeof(double)},
             {s->user_of, m.user_of.data(), m.user_of.size() * sizeof(int32_t)}};
  for (auto& u : ups) {
    if (u.n == 0) continue;
    hipError_t e = hipMemcpy(u.dst, u.src, u.n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      delete s;
      return hip_fail3(e, "hipMemcpy upload");
    }
  }
  hipLaunchKernelGGL(k_diag3_reset, dim3(1), dim3(64), 0, 0, s->diag);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete s;
    return hip_fail3(e, "solver initialisation");
  }
  *out = s;
  return TENO_OK;
}

void teno3_solver_destroy(teno3_solver* s) {
  if (!s) return;
  DevScope3 ds(s->device);
  delete s;
}

int teno3_reconstruct(teno3_solver* s, const double* U, double* face_states, uint32_t* flags,
                      void* stream) {
  if (int rc = check3(s)) return rc;
  if (!U) return fail(TENO_EARG, "null state");
  DevScope3 ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = launch_recon3(s, U, flags, st);
  if (rc) return rc;
  if (face_states) {
    hipError_t e = hipMemcpy2DAsync(face_states, (size_t)s->n_cell * 40, s->fp, (size_t)s->n_pad * 40,
                                    (size_t)s->n_cell * 40, (size_t)4 * s->d.npt,
                                    hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail3(e, "hipMemcpy2DAsync");
  }
  return TENO_OK;
}

int teno3_residual(teno3_solver* s, const double* U, double* R, uint32_t* flags, void* stream) {
  if (int rc = check3(s)) return rc;
  if (!U || !R) return fail(TENO_EARG, "null state");
  DevScope3 ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = launch_recon3(s, U, flags, st);
  if (rc) return rc;
  return launch_flux3(s, U, U, R, nullptr, 0, false, st);
}

int teno3_max_dt(teno3_solver* s, const double* U, double cfl, double* dt_dev, void* stream) {
  if (int rc = check3(s)) return rc;
  if (!U || !dt_dev) return fail(TENO_EARG, "null argument");
  if (!(cfl > 0.0)) return fail(TENO_EARG, "cfl must be positive");
  DevScope3 ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  return timed3(s, 2, st, [&]() {
    hipLaunchKernelGGL(k_dt3_partial, dim3(s->n_dtblk), dim3(256), 0, st, U, (const double*)s->geo,
                       s->n_cell, s->prm.gamma, s->dtpart);
    hipLaunchKernelGGL(k_dt3_final, dim3(1), dim3(256), 0, st, (const double*)s->dtpart, s->n_dtblk,
                       cfl, dt_dev);
  });
}

int teno3_rk_stage(teno3_solver* s, int32_t k, const double* Un, const double* Uk, double* Uk1,
                   const double* dt_dev, uint32_t* flags, void* stream) {
  if (int rc = check3(s)) return rc;
  if (k < 0 || k > 2) return fail(TENO_EARG, "stage must be 0, 1 or 2");
  if (!Un || !Uk || !Uk1 || !dt_dev) return fail(TENO_EARG, "null argument");
  if (k == 0 && Uk != Un) return fail(TENO_EARG, "stage 0 needs Uk == Un");
  if (Uk1 == Uk && Uk != Un) return fail(TENO_EARG, "Uk1 must not alias Uk");
  DevScope3 ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = launch_recon3(s, Uk, flags, st);
  if (rc) return rc;
  return launch_flux3(s, Un, Uk, Uk1, dt_dev, k, true, st);
}

int teno3_rk_step(teno3_solver* s, double* U, const double* dt_dev, uint32_t* flags3,
                  void* stream) {
  if (int rc = check3(s)) return rc;
  if (!U || !dt_dev) return fail(TENO_EARG, "null argument");
  DevScope3 ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)s->n_cell;
  auto fl = [&](int k) { return flags3 ? flags3 + (size_t)k * n : nullptr; };
  const double* in[3] = {U, s->W1, s->W2};
  double* out[3] = {s->W1, s->W2, U};
  for (int k = 0; k < 3; ++k) {
    int rc = launch_recon3(s, in[k], fl(k), st);
    if (rc) return rc;
    rc = launch_flux3(s, U, in[k], out[k], dt_dev, k, true, st);
    if (rc) return rc;
  }
  return TENO_OK;
}

int teno3_diagnostics(teno3_solver* s, teno_diag* out, int32_t reset, void* stream) {
  if (int rc = check3(s)) return rc;
  if (!out) return fail(TENO_EARG, "null argument");
  DevScope3 ds(s->device);
  hipStream_t st = (hipStream_t)stream;
  Diag3 h;
  hipError_t e = hipMemcpyAsync(&h, s->diag, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail3(e, "diagnostics read");
  out->nonphysical = (int64_t)h.nonphysical;
  out->near_ties = (int64_t)h.near_ties;
  out->fallbacks = (int64_t)h.fallbacks;
  out->first_bad_cell = h.first_bad == LLONG_MAX ? -1 : (int64_t)h.first_bad;
  if (reset) {
    hipLaunchKernelGGL(k_diag3_reset, dim3(1), dim3(64), 0, st, s->diag);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail3(e, "diagnostics reset");
  }
  return TENO_OK;
}

int teno3_profile_enable(teno3_solver* s, int32_t kinds) {
  if (int rc = check3(s)) return rc;
  s->prof = (unsigned)kinds & 7u;
  return TENO_OK;
}

int teno3_profile_read(teno3_solver* s, double* ms, int64_t* launches, int32_t reset) {
  if (int rc = check3(s)) return rc;
  DevScope3 ds(s->device);
  for (auto& e : s->evs) {
    hipError_t r = hipEventSynchronize(e.b);
    if (r != hipSuccess) return hip_fail3(r, "hipEventSynchronize");
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e.a, e.b);
    s->prof_ms[e.kind] += t;
    s->prof_n[e.kind] += 1;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  s->evs.clear();
  for (int k = 0; k < 3; ++k) {
    if (ms) ms[k] = s->prof_ms[k];
    if (launches) launches[k] = s->prof_n[k];
    if (reset) {
      s->prof_ms[k] = 0;
      s->prof_n[k] = 0;
    }
  }
  return TENO_OK;
}

}  // extern "C"
