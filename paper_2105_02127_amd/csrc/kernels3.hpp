// HIP kernels of the tetrahedral path (gfx950): per-stage reconstruction
// with TENO selection, HLL face fluxes, residual gather and SSP-RK3 update,
// CFL time step.  Conservative variables (rho, rho u, rho v, rho w, E).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal3.h"

namespace teno {
namespace t3 {

template <int P>
struct O3 {
  static constexpr int R = P - 1;
  static constexpr int NU = (R + 1) * (R + 2) * (R + 3) / 6 - 1;  // large-stencil unknowns
  static constexpr int NL = 2 * NU + 1;                           // its rows
  static constexpr int NPT = P <= 4 ? 6 : 7;                      // points per face
  static constexpr int RSL = NU + (NU & 1);                       // stored large row
  static constexpr int ROWS = 4 * kSmall3Rows + NL;
  static constexpr int JP = 4 * kSmall3Blk + NL * RSL;
};

struct Diag3 {
  unsigned long long nonphysical;
  unsigned long long near_ties;
  unsigned long long fallbacks;
  long long first_bad;  // LLONG_MAX when none
};

struct Recon3Args {
  const double* __restrict__ U;        // [n][5]
  const int32_t* __restrict__ idx;     // [n_tiles][rows][12] stencil members
  const double2* __restrict__ M;       // [n_tiles][jp/2][12] operator entry pairs
  // universal tables, staged in LDS by every block: psi [4 npt][nu] (basis at
  // the face points), then the large and the small smoothness forms packed by
  // rows of their upper triangles (diagonal, then doubled off-diagonals)
  const double* __restrict__ tab;
  double* __restrict__ fp;             // [4 npt][n_pad][5] face-point states
  uint32_t* flags;                     // [n] 5 bits per variable (nullable)
  const int32_t* __restrict__ user_of; // [n_pad]
  Diag3* diag;
  int n_cell, n_tiles, n_pad;
  int variant, fallback, power;
  double ct, eps, gamma, tie_lo, tie_hi;
};

template <int N>
constexpr int packed3() {
  return N * (N + 1) / 2;
}

__device__ __forceinline__ int xcd_remap3(int b, int nblk) {
  const int X = 8;
  const int q = nblk / X, r = nblk % X;
  const int x = b % X, local = b / X;
  return x * q + (x < r ? x : r) + local;
}

__device__ __forceinline__ double gamma3(double beta, double eps, int power) {
  const double x = beta + eps;
  double v = 1.0;
  for (int t = 0; t < power; ++t) v *= x;
  return 1.0 / v;
}

__device__ __forceinline__ int tie3(const Recon3Args& a, double chi) {
  return (chi >= a.tie_lo && chi <= a.tie_hi) ? 1 : 0;
}

// Makes the table offset o depend on the running sum t: the table reads of
// the next chunk cannot be issued before the arithmetic of this one, so the
// compiler does not hoist every read of a fully unrolled loop (one register
// pair per table entry) ahead of its use.
__device__ __forceinline__ void chain3(int& o, double& t) {
  asm volatile("" : "+v"(o), "+v"(t));
}

// a^T B a with B packed by rows of its upper triangle (diagonal first, the
// off-diagonal entries doubled); T is an LDS table, read in chunks of eight
template <int N>
__device__ __forceinline__ double qform3(const double* T, const double (&x)[N]) {
  double s = 0.0;
  int o = 0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    double t = T[o] * x[l];
#pragma unroll
    for (int m = l + 1; m < N; ++m) {
      t = fma(T[o + m - l], x[m], t);
      if ((m - l) % 8 == 0) chain3(o, t);
    }
    s = fma(x[l], t, s);
    o += N - l;
    chain3(o, s);
  }
  return s;
}

// Least squares of one stencil (Sec. 2.2 eqs. 08-10), a = M d with
// d_s = U_member(s) - U_0, for all five variables at once.  The five lanes
// of a cell split the row's entry pairs (lane g takes pairs g, g + 5, ...)
// so every operator byte is loaded by one lane only.  Lane g gathers
// variable g of the row's member (its id read from the tile's rows staged
// in LDS, so the gather never waits behind the operator loads) and the five
// lanes share the five values by lane shuffles; each lane accumulates
// acc[t][k][v] for its pairs.  Lanes past the row's last pair re-read that
// pair (the loads stay unconditional) and their sums are never read.  NB
// rows live in fixed buffers and the loop is unrolled by NB: while one row
// is accumulated the next NB - 1 are in flight.
// hold small stencils' coefficients for the selection (1) or stream them
// again where the large stencil is rejected (0); at order 6, how many
#ifndef TENO3_HOLD_SMALL
#define TENO3_HOLD_SMALL 1
#endif
#ifndef TENO3_HOLD_P6
#define TENO3_HOLD_P6 2
#endif
// the cell's five member values are shared through LDS (1) or by lane
// shuffles (0)
#ifndef TENO3_LDS_SHARE
#define TENO3_LDS_SHARE 1
#endif
template <int NR, int RS, int NB>
struct Stream3 {
  static constexpr int NPAIR = RS / 2;
  static constexpr int NT = (NPAIR + kVars3 - 1) / kVars3;
  using Acc = double[NT][2][kVars3];
  typedef double v2d __attribute__((ext_vector_type(2)));

  const int32_t* sid;              // LDS: member ids of this stencil's rows, [row][kTile3]
  const double2* __restrict__ mp;  // this cell's pairs of row 0 (stride kTile3)
  const double* __restrict__ U;
  double* xs;                      // LDS: the wavefront's 64-double exchange slot (the
                                   // transposes' scratch, idle while a stream runs)
  int c, g;
  double u0[kVars3];
  double xq[NB];
  v2d mq[NB][NT];

  __device__ __forceinline__ int pair_of(int t) const {
    const int p = g + kVars3 * t;
    return p < NPAIR ? p : NPAIR - 1;
  }
  __device__ __forceinline__ void issue(int s, double& x, v2d (&m)[NT]) const {
    s = s < NR ? s : NR - 1;  // loads past the last row re-read it (never used)
    const int id = sid[s * kTile3 + c];
    x = U[(size_t)id * kVars3 + g];
    const double2* __restrict__ mr = mp + (size_t)s * NPAIR * kTile3;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      m[t] = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(&mr[(size_t)pair_of(t) * kTile3]));
  }
  __device__ __forceinline__ void accumulate(double x, const v2d (&m)[NT], Acc& acc) const {
    const int b = kVars3 * c;
    double d[kVars3];
#if TENO3_LDS_SHARE
    // one LDS write and three reads (the cell's five values are adjacent)
    // instead of five two-word lane shuffles; a wavefront's LDS operations
    // complete in order, so the next row's write cannot overtake these reads
    xs[threadIdx.x & 63] = x;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int v = 0; v < kVars3; ++v) d[v] = xs[b + v] - u0[v];
#else
#pragma unroll
    for (int v = 0; v < kVars3; ++v) d[v] = __shfl(x, b + v) - u0[v];
#endif
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < kVars3; ++v) {
        acc[t][0][v] = fma(m[t].x, d[v], acc[t][0][v]);
        acc[t][1][v] = fma(m[t].y, d[v], acc[t][1][v]);
      }
  }
  __device__ __forceinline__ void run(Acc& acc) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < kVars3; ++v) acc[t][0][v] = acc[t][1][v] = 0.0;
#pragma unroll
    for (int k = 0; k < NB - 1; ++k) issue(k, xq[k], mq[k]);
    int s = 0;
#pragma unroll 1
    for (; s + NB - 1 < NR; s += NB) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int nb = (k + NB - 1) % NB;
        issue(s + k + NB - 1, xq[nb], mq[nb]);
        accumulate(xq[k], mq[k], acc);
      }
    }
#pragma unroll
    for (int k = 0; k < NB - 1; ++k)
      if (s + k < NR) accumulate(xq[k], mq[k], acc);
  }
};

// rows in flight: the small streams have one pair per lane and row, so more
// of their rows fit in registers than of the large ones
#ifndef TENO3_SMALL_BUFFERS
#define TENO3_SMALL_BUFFERS 4
#endif
#ifndef TENO3_LARGE_BUFFERS
#define TENO3_LARGE_BUFFERS 3
#endif

// Hands lane (c, v) variable v's coefficients from the split sums: every
// lane writes its pairs' sums for all variables to the wave's scratch, one
// pair slot t at a time, and reads back the variable it owns.  Lanes 60-63
// (no cell) write nothing.
template <int NT, int NC>
__device__ __forceinline__ void transpose3(const double (&acc)[NT][2][kVars3], double* sc, int lane,
                                           int c, int g, double (&co)[NC]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (lane < 60) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int v = 0; v < kVars3; ++v) sc[((c * kVars3 + g) * 2 + k) * kVars3 + v] = acc[t][k][v];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int h = 0; h < kVars3; ++h)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int l = 2 * (h + kVars3 * t) + k;
        if (l < NC) co[l] = sc[((c * kVars3 + h) * 2 + k) * kVars3 + g];
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__device__ __forceinline__ bool physical3(double r, double mx, double my, double mz, double e,
                                          double g) {
  if (!(r > 0.0)) return false;
  const double p = (g - 1.0) * (e - 0.5 * (mx * mx + my * my + mz * mz) / r);
  return p > 0.0;  // false for NaN
}

// waves per SIMD for the order-P kernel (1: left to the compiler).  Holding
// the small stencils' coefficients takes the order-4 kernel to 178 VGPRs (2
// waves); capped at 3 waves it spills 16 and measured 4% faster.
#ifndef TENO3_WAVES_P4
#define TENO3_WAVES_P4 3
#endif
template <int P>
struct Recon3Waves {
  static constexpr int value = P == 4 ? TENO3_WAVES_P4 : 1;
};

// Reconstruction of one tile (12 cells; lane 5c + g): the least-squares
// streams split each row's pairs over the cell's five lanes (all variables
// per lane), and a transpose through LDS gives lane g the coefficients of
// variable g for the selection of Sec. 3.3 with K = 4.  The large stencil's
// coefficients come first, then the small stencils' coefficients and
// indicators, the selection, and where a variable rejects the large stencil
// the mean of the kept small stencils: held in registers at orders 3-4,
// streamed again at orders 5-6 (only the stencils some lane keeps, and only
// in wavefronts where a variable rejects).  Face values of the selected
// polynomial are written as they are formed.
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Recon3Waves<P>::value)))
void k_reconstruct3(Recon3Args a) {
  using O = O3<P>;
  constexpr int NU = O::NU, NPT = O::NPT, NP = 4 * NPT;
  constexpr int NPSI = NP * NU, NBL = packed3<NU>(), NBS = packed3<kSmall3Coef>();
  constexpr int NSC = kTile3 * kVars3 * 2 * kVars3;  // one pair slot of every lane
  constexpr int NID = O::ROWS * kTile3;                // the tile's member ids
  __shared__ double tab[NPSI + NBL + NBS];
  __shared__ double scratch[4][NSC];
  __shared__ int32_t ids[4][NID];
  for (int i = threadIdx.x; i < NPSI + NBL + NBS; i += 256) tab[i] = a.tab[i];
  {
    const int w = threadIdx.x >> 6;
    const int t = xcd_remap3(blockIdx.x, gridDim.x) * 4 + w;
    if (t < a.n_tiles) {
      const int32_t* __restrict__ src = a.idx + (size_t)t * NID;
      for (int i = threadIdx.x & 63; i < NID; i += 64) ids[w][i] = src[i];
    }
  }
  __syncthreads();
  const double* psi = tab;
  const double* Bl = tab + NPSI;
  const double* Bs = tab + NPSI + NBL;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile = __builtin_amdgcn_readfirstlane(xcd_remap3(blockIdx.x, gridDim.x) * 4 + wave);
  if (tile >= a.n_tiles) return;  // whole wavefront leaves together; only wave barriers follow
  double* sc = scratch[wave];
  const int c = lane < 60 ? lane / kVars3 : kTile3 - 1;
  const int g = lane < 60 ? lane - kVars3 * c : 0;
  const int v = g;
  const int cell = tile * kTile3 + c;
  const bool live = lane < 60 && cell < a.n_cell;
  const int cl = cell < a.n_cell ? cell : tile * kTile3;
  double u0[kVars3];
#pragma unroll
  for (int q = 0; q < kVars3; ++q) u0[q] = a.U[(size_t)cl * kVars3 + q];
  const double u0v = u0[v];

  using SmallS = Stream3<kSmall3Rows, kSmall3Stored, TENO3_SMALL_BUFFERS>;
  using LargeS = Stream3<O::NL, O::RSL, TENO3_LARGE_BUFFERS>;
  const int32_t* tid = ids[wave];
  auto small_stream = [&](int k) {
    SmallS st{tid + k * kSmall3Rows * kTile3,
              a.M + ((size_t)tile * (O::JP / 2) + k * kSmall3Blk / 2) * kTile3 + c, a.U, sc, c,
              g};
#pragma unroll
    for (int q = 0; q < kVars3; ++q) st.u0[q] = u0[q];
    return st;
  };

  // ---- large stencil ----
  double co[NU];
  {
    LargeS st{tid + 4 * kSmall3Rows * kTile3,
              a.M + ((size_t)tile * (O::JP / 2) + 4 * kSmall3Blk / 2) * kTile3 + c, a.U, sc, c,
              g};
#pragma unroll
    for (int q = 0; q < kVars3; ++q) st.u0[q] = u0[q];
    typename LargeS::Acc acc;
    st.run(acc);
    transpose3<LargeS::NT, NU>(acc, sc, lane, c, g, co);
  }
  // ---- selection (Sec. 3.2-3.3, K = 4); the linear scheme keeps the large
  // stencil and never reads the small ones.  Each indicator is formed in the
  // block that uses it, so that its table reads are not hoisted apart from
  // its arithmetic.
  // The small stencils' coefficients held for the selection: all four at
  // orders 3-5 (36 values per lane), the first two at order 6, whose kernel
  // already uses every register of two waves per SIMD (all four would cost a
  // wave).  Where a variable rejects the large stencil, the wavefront streams
  // again the stencils it does not hold and some lane keeps.
  constexpr int NH = !TENO3_HOLD_SMALL ? 0 : (P <= 5 ? 4 : TENO3_HOLD_P6);
  double held[NH > 0 ? NH : 1][kSmall3Coef];
  unsigned nib = 0x10u;
  int ties = 0;
  if (a.variant == 0) {
    double gk[4], gs = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      SmallS st = small_stream(k);
      typename SmallS::Acc acc;
      st.run(acc);
      double as[kSmall3Coef];
      transpose3<SmallS::NT, kSmall3Coef>(acc, sc, lane, c, g, as);
      gk[k] = gamma3(qform3<kSmall3Coef>(Bs, as), a.eps, a.power);
      if (k < NH) {
#pragma unroll
        for (int l = 0; l < kSmall3Coef; ++l) held[k < NH ? k : 0][l] = as[l];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) gs += gk[k];
    const double gK = gamma3(qform3<NU>(Bl, co), a.eps, a.power);
    const double chiK = gK / (gs + gK);
    ties += tie3(a, chiK);
    if (chiK < a.ct) {
      nib = 0u;
      const double is = 1.0 / gs;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double x = gk[k] * is;
        ties += tie3(a, x);
        if (x >= a.ct) nib |= 1u << k;
      }
    }
  }
  // ---- large stencil rejected: the mean of the kept small stencils, in
  // stencil order (streams run for the whole wavefront; each lane takes
  // what it keeps) ----
  if (__any(!(nib & 0x10u))) {
    const bool rej = !(nib & 0x10u);
    double ab[kSmall3Coef];
#pragma unroll
    for (int l = 0; l < kSmall3Coef; ++l) ab[l] = 0.0;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < NH; ++k)
      if (rej && ((nib >> k) & 1u)) {
#pragma unroll
        for (int l = 0; l < kSmall3Coef; ++l) ab[l] += held[k][l];
        ++cnt;
      }
#pragma unroll 1
    for (int k = NH; k < 4; ++k) {
      if (!__any(rej && ((nib >> k) & 1u))) continue;
      SmallS st = small_stream(k);
      typename SmallS::Acc acc;
      st.run(acc);
      double as[kSmall3Coef];
      transpose3<SmallS::NT, kSmall3Coef>(acc, sc, lane, c, g, as);
      if (rej && ((nib >> k) & 1u)) {
#pragma unroll
        for (int l = 0; l < kSmall3Coef; ++l) ab[l] += as[l];
        ++cnt;
      }
    }
    // the small stencils' basis is the first nine functions of the large one
    if (rej) {
#pragma unroll
      for (int l = 0; l < NU; ++l) co[l] = (l < kSmall3Coef && cnt > 0) ? ab[l] / (double)cnt : 0.0;
    }
  }
  // ---- face values, written as formed; the five lanes of a cell share
  // their values for the physical-state test ----
  const int b0 = kVars3 * c;
  bool fp_ok = true;
  double* out = a.fp + (size_t)cell * kVars3 + v;
  const size_t qstride = (size_t)a.n_pad * kVars3;
#pragma unroll 1
  for (int q = 0; q < NP; ++q) {
    double s = u0v;
    int o = q * NU;
#pragma unroll
    for (int l = 0; l < NU; ++l) {
      s = fma(co[l], psi[o + l], s);
      if (l % 8 == 7) chain3(o, s);
    }
    fp_ok = physical3(__shfl(s, b0), __shfl(s, b0 + 1), __shfl(s, b0 + 2), __shfl(s, b0 + 3),
                      __shfl(s, b0 + 4), a.gamma) && fp_ok;
    if (live) out[q * qstride] = s;
  }
  const bool avg_ok = physical3(u0[0], u0[1], u0[2], u0[3], u0[4], a.gamma);
  if (live && v == 0 && !(avg_ok && fp_ok)) {
    atomicAdd(&a.diag->nonphysical, 1ull);
    atomicMin(&a.diag->first_bad, (long long)a.user_of[cell]);
  }
  if (!fp_ok && avg_ok && a.fallback) {
    if (live) {
      for (int q = 0; q < NP; ++q) out[q * qstride] = u0v;
      if (v == 0) atomicAdd(&a.diag->fallbacks, 1ull);
    }
    nib = 0u;
  }
  if (live && ties) atomicAdd(&a.diag->near_ties, (unsigned long long)ties);
  if (a.flags) {
    const unsigned f = nib << (5 * v);
    const unsigned all = __shfl(f, b0) | __shfl(f, b0 + 1) | __shfl(f, b0 + 2) | __shfl(f, b0 + 3) |
                         __shfl(f, b0 + 4);
    if (live && v == 0) a.flags[cell] = all;
  }
}

// ---------------------------------------------------------------------------
// HLL flux (Sec. 4) in the face normal: the rotated form of Sec. 4.1 written
// without the rotation (the HLL flux with Einfeldt/Roe speeds commutes with
// rotations), F = F(U_L) if S_L >= 0, F(U_R) if S_R <= 0, else the HLL mean.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void hll3(const double uL[5], const double uR[5], const double n[3],
                                     double g, double F[5]) {
  const double irL = 1.0 / uL[0], irR = 1.0 / uR[0];
  const double vL[3] = {uL[1] * irL, uL[2] * irL, uL[3] * irL};
  const double vR[3] = {uR[1] * irR, uR[2] * irR, uR[3] * irR};
  const double pL = (g - 1.0) * (uL[4] - 0.5 * uL[0] * (vL[0] * vL[0] + vL[1] * vL[1] + vL[2] * vL[2]));
  const double pR = (g - 1.0) * (uR[4] - 0.5 * uR[0] * (vR[0] * vR[0] + vR[1] * vR[1] + vR[2] * vR[2]));
  const double unL = vL[0] * n[0] + vL[1] * n[1] + vL[2] * n[2];
  const double unR = vR[0] * n[0] + vR[1] * n[1] + vR[2] * n[2];
  const double cL = sqrt(g * pL * irL), cR = sqrt(g * pR * irR);
  const double HL = (uL[4] + pL) * irL, HR = (uR[4] + pR) * irR;
  const double D = sqrt(uR[0] * irL), iD = 1.0 / (1.0 + D);
  double vt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) vt[a] = (vL[a] + D * vR[a]) * iD;
  const double Ht = (HL + D * HR) * iD;
  const double ct = sqrt((g - 1.0) * (Ht - 0.5 * (vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2])));
  const double unt = vt[0] * n[0] + vt[1] * n[1] + vt[2] * n[2];
  const double SL = fmin(unL - cL, unt - ct), SR = fmax(unR + cR, unt + ct);
  const double FL[5] = {uL[0] * unL, uL[1] * unL + pL * n[0], uL[2] * unL + pL * n[1],
                        uL[3] * unL + pL * n[2], (uL[4] + pL) * unL};
  const double FR[5] = {uR[0] * unR, uR[1] * unR + pR * n[0], uR[2] * unR + pR * n[1],
                        uR[3] * unR + pR * n[2], (uR[4] + pR) * unR};
  if (SL >= 0.0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) F[c] = FL[c];
  } else if (SR <= 0.0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) F[c] = FR[c];
  } else {
    const double is = 1.0 / (SR - SL);
#pragma unroll
    for (int c = 0; c < 5; ++c) F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (uR[c] - uL[c])) * is;
  }
}

struct Flux3Args {
  const double* __restrict__ fp;      // [4 npt][n_pad][5]
  const int4* __restrict__ fcell;     // [n_face]: L, R (-1-b: boundary b), eL | eR << 2, pairing
  const double4* __restrict__ fgeo;   // [n_face]: nx, ny, nz, |A|
  const int* __restrict__ bkind;      // [n_bface]
  double* __restrict__ phi;           // [n_face][5]
  double w[7];                        // face rule weights
  double gamma;
  int n_face, n_pad;
};

template <int NPT>
__global__ __launch_bounds__(256) void k_face_flux3(Flux3Args a) {
  const int f = xcd_remap3(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (f >= a.n_face) return;
  const int4 fc = a.fcell[f];
  const double4 gg = a.fgeo[f];
  const double n[3] = {gg.x, gg.y, gg.z};
  const int eL = fc.z & 3, eR = fc.z >> 2;
  double phi[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    double uL[5], uR[5];
    const double* pl = a.fp + ((size_t)(eL * NPT + k) * a.n_pad + fc.x) * kVars3;
#pragma unroll
    for (int c = 0; c < 5; ++c) uL[c] = pl[c];
    if (fc.y >= 0) {
      const int kr = (fc.w >> (3 * k)) & 7;
      const double* pr = a.fp + ((size_t)(eR * NPT + kr) * a.n_pad + fc.y) * kVars3;
#pragma unroll
      for (int c = 0; c < 5; ++c) uR[c] = pr[c];
    } else {
      // outer state of the boundary face: transmissive copies the inner
      // state, reflective reverses its normal momentum
#pragma unroll
      for (int c = 0; c < 5; ++c) uR[c] = uL[c];
      if (a.bkind[-1 - fc.y] == TENO_BC_REFLECTIVE) {
        const double mn = uL[1] * n[0] + uL[2] * n[1] + uL[3] * n[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) uR[1 + d] = uL[1 + d] - 2.0 * mn * n[d];
      }
    }
    double F[5];
    hll3(uL, uR, n, a.gamma, F);
#pragma unroll
    for (int c = 0; c < 5; ++c) phi[c] = fma(a.w[k], F[c], phi[c]);
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) a.phi[(size_t)f * 5 + c] = gg.w * phi[c];
}

struct Update3Args {
  const int4* __restrict__ cfaces;    // [n_pad]: faces of local faces 0..3
  const int* __restrict__ cside;      // [n_pad]: bit e when the cell is face e's L
  const double* __restrict__ vol;     // [n_pad]: |V|
  const double* __restrict__ phi;     // [n_face][5]
  const double* Un;
  const double* Uk;
  double* out;                        // R or U^(k+1)
  const double* dt;
  double ca, cb, cc;
  int n_cell, rk;
};

__global__ __launch_bounds__(256) void k_cell_update3(Update3Args a) {
  const int t = xcd_remap3(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (t >= a.n_cell) return;
  const int4 cf = a.cfaces[t];
  const int side = a.cside[t];
  const int fs[4] = {cf.x, cf.y, cf.z, cf.w};
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double* p = a.phi + (size_t)fs[e] * 5;
    const bool isL = (side >> e) & 1;
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] = isL ? acc[c] + p[c] : acc[c] - p[c];
  }
  const double ia = -1.0 / a.vol[t];
  double* o = a.out + (size_t)t * 5;
  if (a.rk) {
    const double dt = *a.dt;
    const double* un = a.Un + (size_t)t * 5;
    const double* uk = a.Uk + (size_t)t * 5;
#pragma unroll
    for (int c = 0; c < 5; ++c) o[c] = a.ca * un[c] + a.cb * uk[c] + a.cc * (dt * (acc[c] * ia));
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) o[c] = acc[c] * ia;
  }
}

__device__ __forceinline__ double block_min3(double x, double* sh) {
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

// |V_i| / sum_f |A_if| (|u_i . n_if| + c_i) per block, then cfl * min
__global__ __launch_bounds__(256) void k_dt3_partial(const double* __restrict__ U,
                                                     const double* __restrict__ geo, int n,
                                                     double g, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int t = blockIdx.x * 256 + threadIdx.x;
  double lim = INFINITY;
  if (t < n) {
    const double* u = U + (size_t)t * 5;
    const double* gg = geo + (size_t)t * 17;
    const double ir = 1.0 / u[0];
    const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    const double p = (g - 1.0) * (u[4] - 0.5 * u[0] * (vx * vx + vy * vy + vz * vz));
    const double c = sqrt(g * p * ir);
    double den = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      den += gg[4 * e + 3] * (fabs(vx * gg[4 * e] + vy * gg[4 * e + 1] + vz * gg[4 * e + 2]) + c);
    lim = gg[16] / den;
  }
  const double m = block_min3(lim, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_dt3_final(const double* __restrict__ partial, int n,
                                                   double cfl, double* __restrict__ dt) {
  __shared__ double sh[4];
  double x = INFINITY;
  for (int i = threadIdx.x; i < n; i += 256) x = fmin(x, partial[i]);
  const double m = block_min3(x, sh);
  if (threadIdx.x == 0) *dt = cfl * m;
}

__global__ void k_diag3_reset(Diag3* d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    d->nonphysical = 0;
    d->near_ties = 0;
    d->fallbacks = 0;
    d->first_bad = LLONG_MAX;
  }
}

}  // namespace t3
}  // namespace teno
