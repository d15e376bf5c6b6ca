// HIP kernels of the TENO residual for gfx950 (MI355X), FP64.
//
//   k_reconstruct  one 64-lane wavefront per tile of 16 cells, one lane per
//                  (cell, conservative variable).  Streams the cell's
//                  least-squares operators (tile-major, double2 loads, fully
//                  coalesced), gathers stencil differences, forms the
//                  coefficients of the three small and the large stencil
//                  (Sec. 2.2 eqs. 08-10), smoothness indicators (Sec. 2.3),
//                  strong scale separation and the two-step ENO-like selection
//                  (Sec. 3.2-3.3), and writes the face Gauss-point states once.
//  k_flux_update   one lane per cell: rotated HLL flux with Einfeldt/Roe wave
//                  speeds (Sec. 4) on the cell's three faces from its own and
//                  its neighbours' face states, face quadrature, gather into
//                  the residual (Sec. 2.1), optional SSP-RK3 stage combine.
//                  Each face flux is evaluated by both of its cells from
//                  identical inputs in identical order, so the two
//                  contributions cancel exactly (no atomics, deterministic).
//  k_dt_*          constant-CFL step: per-block minima, then one block.
//  k_adj_*         adjoint of the residual with the selection frozen.
//
// Lane-to-work mapping and tile layout are described in internal.h.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.h"
#include "tables.h"

namespace teno {

struct DevDiag {
  unsigned long long nonphysical;
  unsigned long long near_ties;
  unsigned long long fallbacks;
  long long first_bad;  // LLONG_MAX when none
};

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that its L2 holds the neighbourhood it gathers.
__device__ __forceinline__ int xcd_remap(int b, int nblk) {
  const int X = 8;
  const int q = nblk / X, r = nblk % X;
  const int x = b % X, local = b / X;
  return x * q + (x < r ? x : r) + local;
}

// ---------------------------------------------------------------------------
// Euler helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool physical(double r, double mx, double my, double e, double g) {
  if (isnan(r) || isnan(mx) || isnan(my) || isnan(e)) return false;
  if (!(r > 0.0)) return false;
  const double p = (g - 1.0) * (e - 0.5 * (mx * mx + my * my) / r);
  return p > 0.0;
}

// Forward-mode dual number with NDIR directional derivatives (adjoint only).
template <int NDIR>
struct Dual {
  double v;
  double d[NDIR];
};

template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(double s, const Dual<N>& a) {
  Dual<N> r;
  r.v = s * a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(double s, const Dual<N>& a) {
  Dual<N> r = a;
  r.v = s + a.v;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> dsqrt(const Dual<N>& a) {
  Dual<N> r;
  r.v = sqrt(a.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
  return r;
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
template <int N>
__device__ __forceinline__ double vof(const Dual<N>& a) { return a.v; }
__device__ __forceinline__ double vof(double a) { return a; }

// HLL flux through unit normal (nx, ny): rotate into the face frame, HLL with
// S_L = min(u_L - c_L, u~ - c~), S_R = max(u_R + c_R, u~ + c~) from Roe
// averages (both velocity components in c~), rotate back.
template <class T>
__device__ __forceinline__ void hll(const T uL[4], const T uR[4], double nx, double ny, double g,
                                    T out[4]) {
  const T L0 = uL[0], L1 = nx * uL[1] + ny * uL[2], L2 = nx * uL[2] + (-ny) * uL[1], L3 = uL[3];
  const T R0 = uR[0], R1 = nx * uR[1] + ny * uR[2], R2 = nx * uR[2] + (-ny) * uR[1], R3 = uR[3];
  const T unL = L1 / L0, utL = L2 / L0, unR = R1 / R0, utR = R2 / R0;
  const T pL = (g - 1.0) * (L3 - (0.5 * L0) * (unL * unL + utL * utL));
  const T pR = (g - 1.0) * (R3 - (0.5 * R0) * (unR * unR + utR * utR));
  const T cL = dsqrt(g * pL / L0), cR = dsqrt(g * pR / R0);
  const T HL = (L3 + pL) / L0, HR = (R3 + pR) / R0;
  const T D = dsqrt(R0 / L0);
  const T den = 1.0 + D;
  const T ut = (unL + D * unR) / den, vt = (utL + D * utR) / den, Ht = (HL + D * HR) / den;
  const T ct = dsqrt((g - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt)));
  const T a1 = unL - cL, a2 = ut - ct;
  const T SL = vof(a2) < vof(a1) ? a2 : a1;
  const T b1 = unR + cR, b2 = ut + ct;
  const T SR = vof(b2) > vof(b1) ? b2 : b1;
  const T FL[4] = {L1, L1 * unL + pL, L1 * utL, unL * (L3 + pL)};
  const T FR[4] = {R1, R1 * unR + pR, R1 * utR, unR * (R3 + pR)};
  const T UL[4] = {L0, L1, L2, L3};
  const T UR[4] = {R0, R1, R2, R3};
  T F[4];
  if (vof(SL) >= 0.0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = FL[c];
  } else if (vof(SR) <= 0.0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = FR[c];
  } else {
    const T inv = SR - SL;
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (UR[c] - UL[c])) / inv;
  }
  out[0] = F[0];
  out[1] = nx * F[1] - ny * F[2];
  out[2] = ny * F[1] + nx * F[2];
  out[3] = F[3];
}

// ---------------------------------------------------------------------------
// reconstruction
// ---------------------------------------------------------------------------
struct ReconArgs {
  const double* __restrict__ U;        // [n_cell][4]
  const int4* __restrict__ idx;        // [n_tiles][rows4][16] int4
  const double2* __restrict__ M;       // [n_tiles][J2][16] double2
  double* __restrict__ fp;             // [3 nq][n_pad][4]
  uint16_t* flags;                     // out, or in when frozen
  const int32_t* __restrict__ user_of; // [n_pad]
  DevDiag* diag;
  int n_cell, n_tiles, n_pad;
  int frozen, variant, fallback, power;
  double ct, eps, gamma, tie_rel;
};

__device__ __forceinline__ double gamma_k(double beta, double eps, int power) {
  const double x = beta + eps;
  double xp = 1.0;
  for (int t = 0; t < power; ++t) xp *= x;
  return 1.0 / xp;
}

template <int N>
__device__ __forceinline__ double quad_form(const double (&B)[N][N], const double* a) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) t = fma(B[l][m], a[m], t);
    s = fma(a[l], t, s);
  }
  return s;
}

// Accumulate rows [R0, R1) of the operator stream: row r gathers
// d = U[member r] - U_0 and adds M[j] d to acc[l] for entry
// j = J0 + (r - R0) * NC + l (all indices compile-time constants).
template <int R0, int R1, int J0, int NC>
struct Rows {
  template <int G = R0>
  static __device__ __forceinline__ void run(const double* __restrict__ U,
                                             const int4* __restrict__ ip,
                                             const double2* __restrict__ mp, int v, double u0,
                                             double* acc) {
    if constexpr (G < R1) {
      const int4 q = ip[(G >> 2) * kTile];
      const int id = (G & 3) == 0 ? q.x : ((G & 3) == 1 ? q.y : ((G & 3) == 2 ? q.z : q.w));
      const double d = U[(size_t)id * 4 + v] - u0;
#pragma unroll
      for (int l = 0; l < NC; ++l) {
        const int j = J0 + (G - R0) * NC + l;
        const double2 m2 = mp[(j >> 1) * kTile];
        acc[l] = fma((j & 1) ? m2.y : m2.x, d, acc[l]);
      }
      run<G + 1>(U, ip, mp, v, u0, acc);
    }
  }
};

// Occupancy target of the reconstruction kernel (waves per SIMD); 0 leaves
// the register budget to the compiler.
#ifndef TENO_RECON_WAVES_PER_EU
#define TENO_RECON_WAVES_PER_EU 0
#endif
#if TENO_RECON_WAVES_PER_EU > 0
#define TENO_RECON_ATTR __attribute__((amdgpu_waves_per_eu(TENO_RECON_WAVES_PER_EU)))
#else
#define TENO_RECON_ATTR
#endif

template <int P, int NQ>
__global__ __launch_bounds__(256) TENO_RECON_ATTR void k_reconstruct(ReconArgs a) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  constexpr int NP = 3 * NQ;
  const int lane = threadIdx.x & 63;
  const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (tile >= a.n_tiles) return;  // whole wavefront leaves together
  const int c = lane >> 2, v = lane & 3;
  const int cell = tile * kTile + c;
  const bool live = cell < a.n_cell;
  const double u0 = a.U[(size_t)(live ? cell : 0) * 4 + v];
  const int4* __restrict__ ip = a.idx + (size_t)tile * O::ROWS4 * kTile + c;
  const double2* __restrict__ mp = a.M + (size_t)tile * O::J2 * kTile + c;

  // ---- small stencils: rows 0..32, entries 0..164 ----
  double as0[5] = {0, 0, 0, 0, 0}, as1[5] = {0, 0, 0, 0, 0}, as2[5] = {0, 0, 0, 0, 0};
  Rows<0, 11, 0, 5>::run(a.U, ip, mp, v, u0, as0);
  Rows<11, 22, 55, 5>::run(a.U, ip, mp, v, u0, as1);
  Rows<22, 33, 110, 5>::run(a.U, ip, mp, v, u0, as2);

  const bool frozen = a.frozen != 0;
  unsigned nib = 0;
  int ties = 0;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  if (!frozen && a.variant == 0) {
    g0 = gamma_k(quad_form(SmoothForm<2>::B.v, as0), a.eps, a.power);
    g1 = gamma_k(quad_form(SmoothForm<2>::B.v, as1), a.eps, a.power);
    g2 = gamma_k(quad_form(SmoothForm<2>::B.v, as2), a.eps, a.power);
  }
  // ---- large stencil: rows 33..33+NL-1 ----
  double aK[NU];
#pragma unroll
  for (int l = 0; l < NU; ++l) aK[l] = 0.0;
  Rows<33, O::ROWS, 165, NU>::run(a.U, ip, mp, v, u0, aK);

  if (frozen) {
    nib = live ? ((a.flags[cell] >> (4 * v)) & 0xFu) : 8u;
  } else if (a.variant == 1) {
    nib = 8u;
  } else {
    const double gK = gamma_k(quad_form(SmoothForm<O::R>::B.v, aK), a.eps, a.power);
    const double ssum = (g0 + g1) + g2;
    const double chiK = gK / (ssum + gK);
    const bool tie_on = a.ct > 0.0;
    if (tie_on && fabs(chiK / a.ct - 1.0) <= a.tie_rel) ++ties;
    if (chiK >= a.ct) {
      nib = 8u;
    } else {
      const double x0 = g0 / ssum, x1 = g1 / ssum, x2 = g2 / ssum;
      if (tie_on) {
        ties += fabs(x0 / a.ct - 1.0) <= a.tie_rel;
        ties += fabs(x1 / a.ct - 1.0) <= a.tie_rel;
        ties += fabs(x2 / a.ct - 1.0) <= a.tie_rel;
      }
      nib = (x0 >= a.ct ? 1u : 0u) | (x1 >= a.ct ? 2u : 0u) | (x2 >= a.ct ? 4u : 0u);
    }
  }
  // ---- combined coefficients ----
  const bool keepK = (nib & 8u) != 0;
  const int cnt = (int)(nib & 1u) + (int)((nib >> 1) & 1u) + (int)((nib >> 2) & 1u);
  double ab[NU];
#pragma unroll
  for (int l = 0; l < NU; ++l) {
    double sm = 0.0;
    if (l < 5) {
      double acc = 0.0;
      if (nib & 1u) acc += as0[l];
      if (nib & 2u) acc += as1[l];
      if (nib & 4u) acc += as2[l];
      sm = cnt > 0 ? acc / (double)cnt : 0.0;
    }
    ab[l] = keepK ? aK[l] : sm;
  }
  // ---- face Gauss points ----
  double val[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    double s = u0;
#pragma unroll
    for (int l = 0; l < NU; ++l) s = fma(ab[l], FaceBasis<O::R, NQ>::P.v[q][l], s);
    val[q] = s;
  }
  // ---- non-physical states (all four lanes of a cell agree) ----
  if (!frozen) {
    const int base = lane & ~3;
    const double r0 = __shfl(u0, base + 0), r1 = __shfl(u0, base + 1);
    const double r2 = __shfl(u0, base + 2), r3 = __shfl(u0, base + 3);
    const bool avg_ok = physical(r0, r1, r2, r3, a.gamma);
    bool fp_ok = true;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const double s0 = __shfl(val[q], base + 0), s1 = __shfl(val[q], base + 1);
      const double s2 = __shfl(val[q], base + 2), s3 = __shfl(val[q], base + 3);
      fp_ok = fp_ok && physical(s0, s1, s2, s3, a.gamma);
    }
    if (live && v == 0 && !(avg_ok && fp_ok)) {
      atomicAdd(&a.diag->nonphysical, 1ull);
      atomicMin(&a.diag->first_bad, (long long)a.user_of[cell]);
    }
    if (!fp_ok && avg_ok && a.fallback) {
#pragma unroll
      for (int q = 0; q < NP; ++q) val[q] = u0;
      nib = 0u;
      if (live && v == 0) atomicAdd(&a.diag->fallbacks, 1ull);
    }
    if (live && ties) atomicAdd(&a.diag->near_ties, (unsigned long long)ties);
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < NP; ++q) a.fp[((size_t)q * a.n_pad + cell) * 4 + v] = val[q];
  }
  if (!frozen && a.flags) {
    unsigned f = nib << (4 * v);
    f |= __shfl_xor(f, 1);
    f |= __shfl_xor(f, 2);
    if (live && v == 0) a.flags[cell] = (uint16_t)f;
  }
}

// ---------------------------------------------------------------------------
// flux, residual, Runge-Kutta stage
// ---------------------------------------------------------------------------
struct FluxArgs {
  const double* __restrict__ fp;       // [3 nq][n_pad][4]
  const int4* __restrict__ nbinfo;     // [n_pad]
  const double* __restrict__ geo;      // [n_pad][10]
  const double* Un;                    // [n][4]
  const double* Uk;                    // [n][4]
  double* out;                         // R or U^(k+1)
  const double* dt;                    // device scalar
  double ca, cb, cc;                   // out = ca Un + cb Uk + cc (dt R)
  double gamma;
  int n_cell, n_pad;
};

template <int NQ, bool RK>
__global__ __launch_bounds__(256) void k_flux_update(FluxArgs a) {
  const int t = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (t >= a.n_cell) return;
  const int4 nb = a.nbinfo[t];
  const double* g = a.geo + (size_t)t * 10;
  const double2* fp2 = reinterpret_cast<const double2*>(a.fp);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int j = e == 0 ? nb.x : (e == 1 ? nb.y : nb.z);
    const int ej = (nb.w >> (2 * e)) & 3;
    const bool isL = (nb.w >> (6 + e)) & 1;
    const double nx = g[3 * e], ny = g[3 * e + 1], len = g[3 * e + 2];
    double phi[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int qi = e * NQ + (isL ? k : NQ - 1 - k);
      const int qj = ej * NQ + (isL ? NQ - 1 - k : k);
      const size_t oi = ((size_t)qi * a.n_pad + t) * 2;
      const size_t oj = ((size_t)qj * a.n_pad + j) * 2;
      const double2 i0 = fp2[oi], i1 = fp2[oi + 1];
      const double2 j0 = fp2[oj], j1 = fp2[oj + 1];
      const double own[4] = {i0.x, i0.y, i1.x, i1.y};
      const double oth[4] = {j0.x, j0.y, j1.x, j1.y};
      double F[4];
      if (isL) hll<double>(own, oth, nx, ny, a.gamma, F);
      else hll<double>(oth, own, nx, ny, a.gamma, F);
#pragma unroll
      for (int c = 0; c < 4; ++c) phi[c] = phi[c] + FaceRule<NQ>::w[k] * F[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double p = phi[c] * len;
      acc[c] = isL ? acc[c] + p : acc[c] - p;
    }
  }
  const double area = g[9];
  double R[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) R[c] = -acc[c] / area;
  double* o = a.out + (size_t)t * 4;
  if (RK) {
    const double dt = *a.dt;
    const double* un = a.Un + (size_t)t * 4;
    const double* uk = a.Uk + (size_t)t * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) o[c] = a.ca * un[c] + a.cb * uk[c] + a.cc * (dt * R[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) o[c] = R[c];
  }
}

// ---------------------------------------------------------------------------
// time step
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_min(double x, double* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmin(x, __shfl_xor(x, o));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) x = fmin(x, sh[k]);
    sh[0] = x;
  }
  __syncthreads();
  return sh[0];
}

__global__ __launch_bounds__(256) void k_dt_partial(const double* __restrict__ U,
                                                    const double* __restrict__ geo, int n,
                                                    double g, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int t = blockIdx.x * 256 + threadIdx.x;
  double lim = INFINITY;
  if (t < n) {
    const double* u = U + (size_t)t * 4;
    const double* gg = geo + (size_t)t * 10;
    const double vx = u[1] / u[0], vy = u[2] / u[0];
    const double p = (g - 1.0) * (u[3] - 0.5 * u[0] * (vx * vx + vy * vy));
    const double c = sqrt(g * p / u[0]);
    double den = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const double un = vx * gg[3 * e] + vy * gg[3 * e + 1];
      den = den + gg[3 * e + 2] * (fabs(un) + c);
    }
    lim = gg[9] / den;
  }
  const double m = block_min(lim, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_dt_final(const double* __restrict__ partial, int n,
                                                  double cfl, double* __restrict__ dt) {
  __shared__ double sh[4];
  double x = INFINITY;
  for (int i = threadIdx.x; i < n; i += 256) x = fmin(x, partial[i]);
  const double m = block_min(x, sh);
  if (threadIdx.x == 0) *dt = cfl * m;
}

// ---------------------------------------------------------------------------
// adjoint of the residual (selection frozen)
// ---------------------------------------------------------------------------
// Phase 1 (one lane per cell): adjoint of the cell's own face-point states.
// Face f gets Phi_bar = lam_R/|V_R| - lam_L/|V_L| (scaled by `scale`); each
// side differentiates the flux with respect to its own state only.
struct AdjArgs {
  const double* __restrict__ fp;
  const int4* __restrict__ nbinfo;
  const double* __restrict__ geo;
  const double* __restrict__ lam;
  const double* scale_dev;  // device scalar multiplying lam (nullable = 1)
  double scale;
  double* __restrict__ fpbar;  // [3 nq][n_pad][4]
  double gamma;
  int n_cell, n_pad;
};

template <int NQ>
__global__ __launch_bounds__(256) void k_adj_face(AdjArgs a) {
  const int t = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (t >= a.n_cell) return;
  const int4 nb = a.nbinfo[t];
  const double* g = a.geo + (size_t)t * 10;
  const double sc = a.scale * (a.scale_dev ? *a.scale_dev : 1.0);
  const double2* fp2 = reinterpret_cast<const double2*>(a.fp);
  const double ai = g[9];
  double li[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) li[c] = a.lam[(size_t)t * 4 + c];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int j = e == 0 ? nb.x : (e == 1 ? nb.y : nb.z);
    const int ej = (nb.w >> (2 * e)) & 3;
    const bool isL = (nb.w >> (6 + e)) & 1;
    const double nx = g[3 * e], ny = g[3 * e + 1], len = g[3 * e + 2];
    const double aj = a.geo[(size_t)j * 10 + 9];
    double pb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double lj = a.lam[(size_t)j * 4 + c];
      const double lL = isL ? li[c] : lj, lR = isL ? lj : li[c];
      const double aL = isL ? ai : aj, aR = isL ? aj : ai;
      pb[c] = sc * (lR / aR - lL / aL);
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int qi = e * NQ + (isL ? k : NQ - 1 - k);
      const int qj = ej * NQ + (isL ? NQ - 1 - k : k);
      const size_t oi = ((size_t)qi * a.n_pad + t) * 2;
      const size_t oj = ((size_t)qj * a.n_pad + j) * 2;
      const double2 i0 = fp2[oi], i1 = fp2[oi + 1];
      const double2 j0 = fp2[oj], j1 = fp2[oj + 1];
      const double own[4] = {i0.x, i0.y, i1.x, i1.y};
      const double oth[4] = {j0.x, j0.y, j1.x, j1.y};
      Dual<4> o[4], p[4], F[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        o[c].v = own[c];
        p[c].v = oth[c];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          o[c].d[d] = (c == d) ? 1.0 : 0.0;
          p[c].d[d] = 0.0;
        }
      }
      if (isL) hll<Dual<4>>(o, p, nx, ny, a.gamma, F);
      else hll<Dual<4>>(p, o, nx, ny, a.gamma, F);
      const double w = len * FaceRule<NQ>::w[k];
      double* out = a.fpbar + ((size_t)qi * a.n_pad + t) * 4;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) s = fma(pb[c], F[c].d[d], s);
        out[d] = w * s;
      }
    }
  }
}

// Phase 2 (one lane per (cell, variable)): transpose of the reconstruction.
// Writes the adjoint of every stencil difference d_s = U_s - U_0 to
// dbar[row][n_pad][4] and the cell's own direct part to own[n][4].
struct AdjReconArgs {
  const double* __restrict__ fpbar;
  const uint16_t* __restrict__ flags;
  const double2* __restrict__ M;
  double* __restrict__ dbar;   // [rows4*4][n_pad][4]
  double* __restrict__ own;    // [n_pad][4]
  int n_cell, n_tiles, n_pad;
};

template <int P, int NQ>
__global__ __launch_bounds__(256) void k_adj_recon(AdjReconArgs a) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  constexpr int NP = 3 * NQ;
  const int lane = threadIdx.x & 63;
  const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (tile >= a.n_tiles) return;
  const int c = lane >> 2, v = lane & 3;
  const int cell = tile * kTile + c;
  if (cell >= a.n_cell) return;
  const unsigned nib = (a.flags[cell] >> (4 * v)) & 0xFu;
  double gsum = 0.0;
  double ab[NU];
#pragma unroll
  for (int l = 0; l < NU; ++l) ab[l] = 0.0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const double gq = a.fpbar[((size_t)q * a.n_pad + cell) * 4 + v];
    gsum += gq;
#pragma unroll
    for (int l = 0; l < NU; ++l) ab[l] = fma(FaceBasis<O::R, NQ>::P.v[q][l], gq, ab[l]);
  }
  const double2* __restrict__ mp = a.M + (size_t)tile * O::J2 * kTile + c;
  const bool keepK = nib & 8u;
  const int cnt = (int)(nib & 1u) + (int)((nib >> 1) & 1u) + (int)((nib >> 2) & 1u);
  double dsum = 0.0;
  // small stencils: coefficient adjoint ab[l]/cnt when kept in step two
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double wk = (!keepK && (nib & (1u << k)) && cnt > 0) ? 1.0 / (double)cnt : 0.0;
#pragma unroll
    for (int s = 0; s < 11; ++s) {
      double d = 0.0;
#pragma unroll
      for (int l = 0; l < 5; ++l) {
        const int j = k * 55 + s * 5 + l;
        const double2 q = mp[(j >> 1) * kTile];
        d = fma((j & 1) ? q.y : q.x, ab[l], d);
      }
      d *= wk;
      dsum += d;
      a.dbar[((size_t)(k * 11 + s) * a.n_pad + cell) * 4 + v] = d;
    }
  }
  const double wK = keepK ? 1.0 : 0.0;
#pragma unroll 1
  for (int s = 0; s < O::NL; ++s) {
    double d = 0.0;
#pragma unroll
    for (int l = 0; l < NU; ++l) {
      const int j = 165 + s * NU + l;
      const double2 q = mp[(j >> 1) * kTile];
      d = fma((j & 1) ? q.y : q.x, ab[l], d);
    }
    d *= wK;
    dsum += d;
    a.dbar[((size_t)(33 + s) * a.n_pad + cell) * 4 + v] = d;
  }
  a.own[(size_t)cell * 4 + v] = gsum - dsum;
}

// Phase 3 (one lane per cell): U_bar[j] = own[j] + sum over every stencil
// row naming j of that row's adjoint, in a fixed order (no atomics); then
// out = U_bar + beta * extra (extra nullable).
__global__ __launch_bounds__(256) void k_adj_gather(const double* __restrict__ own,
                                                    const double* __restrict__ dbar,
                                                    const int32_t* __restrict__ rev_ptr,
                                                    const int32_t* __restrict__ rev_ent, int rows4x4,
                                                    int n_cell, int n_pad, const double* extra,
                                                    double beta, double* out) {
  const int j = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (j >= n_cell) return;
  double s[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) s[c] = own[(size_t)j * 4 + c];
  const int b = rev_ptr[j], e = rev_ptr[j + 1];
  for (int t = b; t < e; ++t) {
    const int ent = rev_ent[t];
    const int i = ent / rows4x4, r = ent - i * rows4x4;
    const double2* d2 = reinterpret_cast<const double2*>(dbar + ((size_t)r * n_pad + i) * 4);
    const double2 x = d2[0], y = d2[1];
    s[0] += x.x;
    s[1] += x.y;
    s[2] += y.x;
    s[3] += y.y;
  }
  if (extra) {
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] = s[c] + beta * extra[(size_t)j * 4 + c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) out[(size_t)j * 4 + c] = s[c];
}

// out = a1 x1 + a2 x2 (+ a3 x3), elementwise over n doubles.
__global__ __launch_bounds__(256) void k_lincomb(double* out, double a1, const double* x1,
                                                 double a2, const double* x2, double a3,
                                                 const double* x3, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = a1 * x1[i];
  if (x2) s = s + a2 * x2[i];
  if (x3) s = s + a3 * x3[i];
  out[i] = s;
}

__global__ void k_diag_reset(DevDiag* d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    d->nonphysical = 0;
    d->near_ties = 0;
    d->fallbacks = 0;
    d->first_bad = LLONG_MAX;
  }
}

}  // namespace teno
