// HIP kernels of the TENO residual for gfx950 (MI355X), FP64.
//
//   k_reconstruct  one 64-lane wavefront per tile of 16 cells, four lanes per
//                  cell.  Least-squares phase (Sec. 2.2 eqs. 08-10): the four
//                  lanes split the coefficient index (lane g owns l = g,
//                  g+4, ...) and carry all four conservative variables, so
//                  every operator entry is loaded by exactly one lane and a
//                  wavefront load moves 512 contiguous bytes; stencil
//                  differences are gathered one variable per lane and shared
//                  by DPP quad broadcasts.  Selection phase: DPP quad
//                  transposes give lane g the full coefficient vector of
//                  variable g, which then forms the smoothness indicators
//                  (Sec. 2.3), the strong scale separation and the two-step
//                  ENO-like selection (Sec. 3.2-3.3), and the face
//                  Gauss-point states, written once.
//  k_face_flux     one lane per face: rotated HLL flux with Einfeldt/Roe wave
//                  speeds (Sec. 4) at the face's Gauss point pairs and the
//                  face quadrature, written once per face.
//  k_cell_update   one lane per cell: gather of its three face fluxes into
//                  the residual (Sec. 2.1), optional SSP-RK3 stage combine
//                  (a gather in a fixed order: no atomics, deterministic).
//  k_dt_*          constant-CFL step: per-block minima, then one block.
//  k_adj_*         adjoint of the residual with the selection frozen.
//
// Lane-to-work mapping and tile layout are described in internal.h.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

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

// HLL flux through unit normal (nx, ny): rotate into the face frame, HLL with
// S_L = min(u_L - c_L, u~ - c~), S_R = max(u_R + c_R, u~ + c~) from Roe
// averages (both velocity components in c~), rotate back.  The quotients
// share four reciprocals (1/rho_L, 1/rho_R, 1/(1 + sqrt(rho_R/rho_L)),
// 1/(S_R - S_L)): FP64 division is a long instruction sequence and this
// function is most of the flux kernel's work.
__device__ __forceinline__ void hll(const double uL[4], const double uR[4], double nx, double ny,
                                    double g, double out[4]) {
  const double L0 = uL[0], L1 = nx * uL[1] + ny * uL[2], L2 = nx * uL[2] + (-ny) * uL[1], L3 = uL[3];
  const double R0 = uR[0], R1 = nx * uR[1] + ny * uR[2], R2 = nx * uR[2] + (-ny) * uR[1], R3 = uR[3];
  const double iL = 1.0 / L0, iR = 1.0 / R0;
  const double unL = L1 * iL, utL = L2 * iL, unR = R1 * iR, utR = R2 * iR;
  const double pL = (g - 1.0) * (L3 - (0.5 * L0) * (unL * unL + utL * utL));
  const double pR = (g - 1.0) * (R3 - (0.5 * R0) * (unR * unR + utR * utR));
  const double cL = sqrt(g * pL * iL), cR = sqrt(g * pR * iR);
  const double HL = (L3 + pL) * iL, HR = (R3 + pR) * iR;
  const double D = sqrt(R0 * iL);
  const double iden = 1.0 / (1.0 + D);
  const double ut = (unL + D * unR) * iden, vt = (utL + D * utR) * iden, Ht = (HL + D * HR) * iden;
  const double ct = sqrt((g - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt)));
  const double a1 = unL - cL, a2 = ut - ct;
  const double SL = a2 < a1 ? a2 : a1;
  const double b1 = unR + cR, b2 = ut + ct;
  const double SR = b2 > b1 ? b2 : b1;
  const double FL[4] = {L1, L1 * unL + pL, L1 * utL, unL * (L3 + pL)};
  const double FR[4] = {R1, R1 * unR + pR, R1 * utR, unR * (R3 + pR)};
  const double UL[4] = {L0, L1, L2, L3};
  const double UR[4] = {R0, R1, R2, R3};
  double F[4];
  if (SL >= 0.0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = FL[c];
  } else if (SR <= 0.0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = FR[c];
  } else {
    const double iS = 1.0 / (SR - SL);
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (UR[c] - UL[c])) * iS;
  }
  out[0] = F[0];
  out[1] = nx * F[1] - ny * F[2];
  out[2] = ny * F[1] + nx * F[2];
  out[3] = F[3];
}

// Reverse mode of hll (the same flux, the same branches): adds
// ob^T d(out)/d(uL) to gL and ob^T d(out)/d(uR) to gR.  The speed selections
// and the flux case follow the primal values, as the flux does.  One pass
// forward, one back: both sides' adjoints for about three times the flux's
// arithmetic.
__device__ __forceinline__ void hll_vjp(const double uL[4], const double uR[4], double nx,
                                        double ny, double g, const double ob[4], double gL[4],
                                        double gR[4]) {
  const double gm = g - 1.0;
  // ---- primal, keeping what the reverse pass needs ----
  const double L0 = uL[0], L1 = nx * uL[1] + ny * uL[2], L2 = nx * uL[2] + (-ny) * uL[1], L3 = uL[3];
  const double R0 = uR[0], R1 = nx * uR[1] + ny * uR[2], R2 = nx * uR[2] + (-ny) * uR[1], R3 = uR[3];
  const double iL = 1.0 / L0, iR = 1.0 / R0;
  const double unL = L1 * iL, utL = L2 * iL, unR = R1 * iR, utR = R2 * iR;
  const double qL = unL * unL + utL * utL, qR = unR * unR + utR * utR;
  const double pL = gm * (L3 - (0.5 * L0) * qL), pR = gm * (R3 - (0.5 * R0) * qR);
  const double cL = sqrt(g * pL * iL), cR = sqrt(g * pR * iR);
  const double EL = L3 + pL, ER = R3 + pR;  // rho H
  const double HL = EL * iL, HR = ER * iR;
  const double D = sqrt(R0 * iL);
  const double iden = 1.0 / (1.0 + D);
  const double nu = unL + D * unR, nv = utL + D * utR, nH = HL + D * HR;
  const double ut = nu * iden, vt = nv * iden, Ht = nH * iden;
  const double ct = sqrt(gm * (Ht - 0.5 * (ut * ut + vt * vt)));
  const double a1 = unL - cL, a2 = ut - ct;
  const bool l2 = a2 < a1;
  const double SL = l2 ? a2 : a1;
  const double b1 = unR + cR, b2 = ut + ct;
  const bool r2 = b2 > b1;
  const double SR = r2 ? b2 : b1;
  const double FL[4] = {L1, L1 * unL + pL, L1 * utL, unL * EL};
  const double FR[4] = {R1, R1 * unR + pR, R1 * utR, unR * ER};
  const double UL[4] = {L0, L1, L2, L3}, UR[4] = {R0, R1, R2, R3};
  // ---- reverse ----
  // out = (F0, nx F1 - ny F2, ny F1 + nx F2, F3)
  const double Fb[4] = {ob[0], nx * ob[1] + ny * ob[2], nx * ob[2] - ny * ob[1], ob[3]};
  double FLb[4] = {0.0, 0.0, 0.0, 0.0}, FRb[4] = {0.0, 0.0, 0.0, 0.0};
  double Lb[4] = {0.0, 0.0, 0.0, 0.0}, Rb[4] = {0.0, 0.0, 0.0, 0.0};
  double SLb = 0.0, SRb = 0.0;
  if (SL >= 0.0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) FLb[c] = Fb[c];
  } else if (SR <= 0.0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) FRb[c] = Fb[c];
  } else {
    // F_c = N_c iS, N_c = SR FL_c - SL FR_c + SL SR (UR_c - UL_c), iS = 1 / (SR - SL)
    const double iS = 1.0 / (SR - SL);
    double iSb = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double dU = UR[c] - UL[c];
      const double N = SR * FL[c] - SL * FR[c] + SL * SR * dU;
      const double Nb = Fb[c] * iS;
      iSb += Fb[c] * N;
      FLb[c] = SR * Nb;
      FRb[c] = -SL * Nb;
      SRb += Nb * (FL[c] + SL * dU);
      SLb += Nb * (SR * dU - FR[c]);
      Rb[c] += SL * SR * Nb;
      Lb[c] -= SL * SR * Nb;
    }
    const double t = -iS * iS * iSb;  // d(iS) = -iS^2 d(SR - SL)
    SRb += t;
    SLb -= t;
  }
  // the physical fluxes
  Lb[1] += FLb[0] + FLb[1] * unL + FLb[2] * utL;
  Rb[1] += FRb[0] + FRb[1] * unR + FRb[2] * utR;
  double unLb = FLb[1] * L1 + FLb[3] * EL, unRb = FRb[1] * R1 + FRb[3] * ER;
  double utLb = FLb[2] * L1, utRb = FRb[2] * R1;
  double pLb = FLb[1], pRb = FRb[1];
  double ELb = FLb[3] * unL, ERb = FRb[3] * unR;
  // the wave-speed estimates
  const double a1b = l2 ? 0.0 : SLb, a2b = l2 ? SLb : 0.0;
  const double b1b = r2 ? 0.0 : SRb, b2b = r2 ? SRb : 0.0;
  unLb += a1b;
  const double cLb = -a1b;
  unRb += b1b;
  const double cRb = b1b;
  double utb = a2b + b2b;
  const double ctb = b2b - a2b;
  // ct = sqrt(X), X = (g - 1) (Ht - (ut^2 + vt^2) / 2)
  const double Xb = ctb * 0.5 / ct;
  const double Htb = gm * Xb;
  utb -= gm * ut * Xb;
  const double vtb = -gm * vt * Xb;
  // Roe averages: ut = nu iden, vt = nv iden, Ht = nH iden
  const double nub = utb * iden, nvb = vtb * iden, nHb = Htb * iden;
  const double idenb = utb * nu + vtb * nv + Htb * nH;
  unLb += nub;
  unRb += D * nub;
  utLb += nvb;
  utRb += D * nvb;
  const double HLb = nHb, HRb = D * nHb;
  double Db = unR * nub + utR * nvb + HR * nHb - iden * iden * idenb;
  // D = sqrt(R0 iL)
  const double Yb = Db * 0.5 / D;
  Rb[0] += Yb * iL;
  double iLb = Yb * R0, iRb = 0.0;
  // H = (E + p) / rho
  ELb += HLb * iL;
  iLb += HLb * EL;
  ERb += HRb * iR;
  iRb += HRb * ER;
  // c = sqrt(g p / rho)
  const double ZLb = cLb * 0.5 / cL, ZRb = cRb * 0.5 / cR;
  pLb += g * iL * ZLb + ELb;
  iLb += g * pL * ZLb;
  pRb += g * iR * ZRb + ERb;
  iRb += g * pR * ZRb;
  Lb[3] += ELb;
  Rb[3] += ERb;
  // p = (g - 1) (E - rho q / 2)
  Lb[3] += gm * pLb;
  Rb[3] += gm * pRb;
  Lb[0] -= 0.5 * gm * qL * pLb;
  Rb[0] -= 0.5 * gm * qR * pRb;
  const double qLb = -0.5 * gm * L0 * pLb, qRb = -0.5 * gm * R0 * pRb;
  unLb += 2.0 * unL * qLb;
  utLb += 2.0 * utL * qLb;
  unRb += 2.0 * unR * qRb;
  utRb += 2.0 * utR * qRb;
  // un = m_n / rho, ut = m_t / rho
  Lb[1] += unLb * iL;
  Lb[2] += utLb * iL;
  iLb += unLb * L1 + utLb * L2;
  Rb[1] += unRb * iR;
  Rb[2] += utRb * iR;
  iRb += unRb * R1 + utRb * R2;
  Lb[0] -= iL * iL * iLb;
  Rb[0] -= iR * iR * iRb;
  // the rotation into the face frame
  gL[0] += Lb[0];
  gL[1] += nx * Lb[1] - ny * Lb[2];
  gL[2] += ny * Lb[1] + nx * Lb[2];
  gL[3] += Lb[3];
  gR[0] += Rb[0];
  gR[1] += nx * Rb[1] - ny * Rb[2];
  gR[2] += ny * Rb[1] + nx * Rb[2];
  gR[3] += Rb[3];
}

// ---------------------------------------------------------------------------
// reconstruction
// ---------------------------------------------------------------------------
struct ReconArgs {
  const double* __restrict__ U;        // [n_cell][4]
  const int4* __restrict__ slot;       // [n_tiles][rows4][16][4] uint16, 8 per int4
  const int* __restrict__ tmem;        // [n_tiles][ustride] distinct members of a tile
  int ustride;                         // members per tile list
  int lds_stride;                      // LDS per wavefront in int4 (stage_int4)
  const double2* __restrict__ M;       // [n_tiles][JP * kTile] doubles: the tile's blocks
  double* __restrict__ fp;             // [3 nq][n_pad][4]
  uint16_t* flags;                     // out, or in when frozen
  const int32_t* __restrict__ user_of; // [n_pad]
  const double* __restrict__ geo;      // [n_pad][10]: (nx, ny, len) x 3 edges, area
  const int4* __restrict__ nbinfo;     // [n_pad]: .w bit 6+e set when the cell is edge e's L side
  DevDiag* diag;
  int n_cell, n_tiles, n_pad;
  int frozen, variant, fallback, power;
  double ct, eps, gamma, tie_rel;
  double tie_lo, tie_hi;               // near-tie window ct (1 -+ tie_rel); empty when ct = 0
  double cw_dK, cw_ds;                 // CWENO linear weights: large, each small
};

// chi within the near-tie window around C_T (counted, never decided on).
__device__ __forceinline__ int near_tie(const ReconArgs& a, double chi) {
  return (chi >= a.tie_lo && chi <= a.tie_hi) ? 1 : 0;
}

__device__ __forceinline__ double gamma_k(double beta, double eps, int power) {
  const double x = beta + eps;
  double xp;
  if (power == 6) {  // the paper's q: the same products, in the same order, unrolled
    xp = x * x;
    xp *= x;
    xp *= x;
    xp *= x;
    xp *= x;
  } else {
    xp = 1.0;
    for (int t = 0; t < power; ++t) xp *= x;
  }
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

// The same form from U, the upper triangle of B with its off-diagonal
// entries doubled: about half the multiply-adds, but with fewer
// instructions between them the compiler keeps more values live.
template <int N>
__device__ __forceinline__ double quad_form_upper(const double (&U)[N][N], const double* a) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    double t = U[l][l] * a[l];
#pragma unroll
    for (int m = l + 1; m < N; ++m) t = fma(U[l][m], a[m], t);
    s = fma(a[l], t, s);
  }
  return s;
}

// beta = a^T B a of degree R from the full table, or from its doubled upper
// triangle (UP).
template <int R, bool UP>
__device__ __forceinline__ double smoothness(const double* a) {
  if constexpr (UP)
    return quad_form_upper(SmoothForm<R>::U.v, a);
  else
    return quad_form(SmoothForm<R>::B.v, a);
}

// Broadcast lane K of every group of four lanes (DPP quad permutation).
template <int K>
__device__ __forceinline__ double quad_bcast(double x) {
  constexpr int ctrl = K * 0x55;  // quad_perm(K, K, K, K)
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double pick4(double t0, double t1, double t2, double t3, int g) {
  return g == 0 ? t0 : (g == 1 ? t1 : (g == 2 ? t2 : t3));
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Least-squares phase (Sec. 2.2 eqs. 08-10) of one stencil as a stream of
// its NR rows: a = M d with d_s = U_member(s) - U_0, row s of M^T stored at
// entries J0 + s*RS .. (RS even; entries past the coefficient count are
// zero).  Each cell has LPC = 64 / kTile lanes (g = 0..LPC-1); lane g gathers
// variable g % 4 of the row's member, the four lanes share d for all four
// variables by quad broadcast, and lane g adds the entry pairs p = g + LPC t
// it owns (coefficients 2p and 2p+1, one 16-byte load each) into
// acc[t][k][v].  Every entry is loaded by exactly one lane, and every
// coefficient adds the rows one at a time in row order, as a plain GEMV does.
//
// The states of the tile's distinct stencil members and each row's slot among
// them are staged in LDS once per tile, so the row loop's only memory loads
// are the operator entries.  NB row buffers live in fixed registers and the row
// loop is unrolled by NB: while one row is accumulated the next NB-1 are in
// flight, and no register changes role between iterations (a rotating
// buffer would force a full wait every row).  prime() issues the first
// NB-1 rows, so a caller can start the stream before it finishes other work.
#ifndef TENO_ROW_BUFFERS
#define TENO_ROW_BUFFERS 3
#endif
#ifndef TENO_M_NONTEMPORAL
#define TENO_M_NONTEMPORAL 1
#endif

template <int R0, int NR, int RS>
struct RowStream {
  static constexpr int NB = TENO_ROW_BUFFERS;
  static constexpr int LPC = kLanesPerCell;
  static constexpr int NPAIR = RS / 2;                // pairs per row
  static constexpr int NT = (NPAIR + LPC - 1) / LPC;  // pair slots per lane
  static_assert(RS % 2 == 0, "rows are whole pairs");
  using Acc = double[NT][2][4];

  const double* us;                    // LDS: states of the tile's distinct members
  const uint16_t* sidx;                // LDS: each stencil row's member slot
  const double2* __restrict__ mp;      // this cell's pairs of the block
  int c, g;
  double u0g;
  double xq[NB];
  double2 mq[NB][NT];

  __device__ __forceinline__ void issue(int s, double& x, double2 (&m)[NT]) const {
    s = s < NR ? s : NR - 1;  // loads past the last row re-read it (never used)
    const int r = R0 + s;
    const int id = sidx[(r >> 2) * (kTile * 4) + c * 4 + (r & 3)];
    x = us[id * 4 + (g & 3)];
    const double2* __restrict__ mr = mp + (size_t)(s * RS / 2) * kTile;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // Lanes past the row's last pair re-read that pair: the load stays
      // unconditional (a predicated load merged with a zero would make the
      // compiler copy the buffers and wait for every load at the back edge),
      // and the accumulators it feeds are never read.
      const int pr = (LPC * t + LPC - 1 < NPAIR) ? g + LPC * t : min(g + LPC * t, NPAIR - 1);
#if TENO_M_NONTEMPORAL
      // operator entries are read once per stage: keep them out of the way
      // of the gathered states in the caches
      typedef double v2d __attribute__((ext_vector_type(2)));
      const v2d w = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(&mr[(size_t)pr * kTile]));
      m[t] = make_double2(w.x, w.y);
#else
      m[t] = mr[(size_t)pr * kTile];
#endif
    }
  }

  __device__ __forceinline__ void accumulate(double xv, const double2 (&m)[NT], Acc& acc) const {
    const double x = xv - u0g;
    const double d[4] = {quad_bcast<0>(x), quad_bcast<1>(x), quad_bcast<2>(x), quad_bcast<3>(x)};
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[t][0][q] = fma(m[t].x, d[q], acc[t][0][q]);
        acc[t][1][q] = fma(m[t].y, d[q], acc[t][1][q]);
      }
  }

  __device__ __forceinline__ void prime() {
    static_for<0, NB - 1>([&](auto k) { issue(k, xq[k], mq[k]); });
  }

  // All rows into acc; prime() must have been called.
  __device__ __forceinline__ void run(Acc& acc) {
    int s = 0;
#pragma unroll 1
    for (; s + NB - 1 < NR; s += NB) {
      static_for<0, NB>([&](auto k) {
        constexpr int nb = (k + NB - 1) % NB;
        issue(s + k + NB - 1, xq[nb], mq[nb]);
        accumulate(xq[k], mq[k], acc);
      });
    }
    static_for<0, NB - 1>([&](auto k) {
      if (s + k < NR) accumulate(xq[k], mq[k], acc);
    });
  }

  // Coefficient l (variable v): pair l/2 is held by lane (l/2) % LPC of the
  // cell's lane group in slot (l/2) / LPC, component l % 2.
  template <int l>
  __device__ __forceinline__ static double coef(const Acc& acc, int v, int lane) {
    constexpr int src = (l / 2) % LPC, t = (l / 2) / LPC, k = l % 2;
    if constexpr (LPC == 4) {
      return pick4(quad_bcast<src>(acc[t][k][0]), quad_bcast<src>(acc[t][k][1]),
                   quad_bcast<src>(acc[t][k][2]), quad_bcast<src>(acc[t][k][3]), v);
    } else {
      const int sl = (lane & ~(LPC - 1)) | src;
      return pick4(__shfl(acc[t][k][0], sl), __shfl(acc[t][k][1], sl), __shfl(acc[t][k][2], sl),
                   __shfl(acc[t][k][3], sl), v);
    }
  }
};

// The same least-squares phase for a block stored rows by lane (odd L, see
// block_offset): the NR rows come in groups of four, lane g of a cell owns
// row 4j + g of group j and adds all L entries of it into all four
// variables, acc[l][v] += M_l d_v, with d read from the staged member states
// (all four variables of the member).  Every lane's loads are distinct and
// contiguous across the wavefront, and no difference is broadcast.  Lanes
// past the last group's rows re-read its last row with d = 0.  The groups
// are few (3 for a small stencil, 5 for the large one at order 4) and fully
// unrolled; NB of them are in flight.  coef<l>() sums the four lanes'
// partial sums of coefficient l in a fixed order (lanes {0,1} and {2,3}
// first) and hands lane g variable g.
#ifndef TENO_LANE_BUFFERS
#define TENO_LANE_BUFFERS 2
#endif

template <class T>
struct TypeTag {
  using type = T;
};

template <int K>
__device__ __forceinline__ double quad_perm_dpp(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), K, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), K, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int R0, int NR, int L>
struct RowLanes {
  static constexpr int NG = (NR + 3) / 4;
  static constexpr int NB = TENO_LANE_BUFFERS < NG ? TENO_LANE_BUFFERS : NG;
  static_assert(kTile == 16, "rows by lane need four lanes per cell");
  using Acc = double[L][4];

  const double* us;                    // LDS: states of the tile's distinct members
  const uint16_t* sidx;                // LDS: each stencil row's member slot
  const double* __restrict__ mb;       // the tile's block
  int c, g;
  double u0[4];                        // the cell's means, all four variables
  double xq[NB][4];
  double mq[NB][L];

  template <int J>
  __device__ __forceinline__ void issue(double (&x)[4], double (&m)[L]) const {
    constexpr int rg = group_rows(NR, J);
    const int gg = g < rg ? g : rg - 1;
    const int r = R0 + 4 * J + gg;
    const int id = sidx[(r >> 2) * (kTile * 4) + c * 4 + (r & 3)];
    const double2* u = reinterpret_cast<const double2*>(us + id * 4);
    const double2 a0 = u[0], a1 = u[1];
    x[0] = a0.x;
    x[1] = a0.y;
    x[2] = a1.x;
    x[3] = a1.y;
    const double* __restrict__ p = mb + 4 * kTile * L * J + c * rg + gg;
#pragma unroll
    for (int l = 0; l < L; ++l) m[l] = __builtin_nontemporal_load(p + l * kTile * rg);
  }

  template <int J>
  __device__ __forceinline__ void accumulate(const double (&x)[4], const double (&m)[L],
                                             Acc& acc) const {
    constexpr int rg = group_rows(NR, J);
    const bool on = rg == 4 || g < rg;
    double d[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = on ? x[v] - u0[v] : 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[l][v] = fma(m[l], d[v], acc[l][v]);
  }

  __device__ __forceinline__ void prime() {
    static_for<0, NB - 1>([&](auto k) { issue<k>(xq[k], mq[k]); });
  }

  __device__ __forceinline__ void run(Acc& acc) {
    static_for<0, NG>([&](auto j) {
      constexpr int nj = j + NB - 1;
      if constexpr (nj < NG) issue<nj>(xq[nj % NB], mq[nj % NB]);
      accumulate<j>(xq[j % NB], mq[j % NB], acc);
    });
  }

  // Coefficient l of variable v = g: reduce-scatter over the cell's four
  // lanes.  Lane g keeps the variables of its parity and takes its
  // neighbour's (g ^ 1) sums of them, then keeps variable g and takes
  // lane g ^ 2's pair sum of it.  Called with all four lanes active.
  template <int l>
  __device__ __forceinline__ static double coef(const Acc& acc, int v, int lane) {
    const bool odd = lane & 1, hi = lane & 2;
    const double k0 = odd ? acc[l][1] : acc[l][0];
    const double k1 = odd ? acc[l][3] : acc[l][2];
    const double s0 = odd ? acc[l][0] : acc[l][1];
    const double s1 = odd ? acc[l][2] : acc[l][3];
    const double p0 = k0 + quad_perm_dpp<0xB1>(s0);  // quad_perm(1, 0, 3, 2)
    const double p1 = k1 + quad_perm_dpp<0xB1>(s1);
    const double keep = hi ? p1 : p0, send = hi ? p0 : p1;
    return keep + quad_perm_dpp<0x4E>(send);  // quad_perm(2, 3, 0, 1)
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

// LDS ordering between the lanes of one wavefront (staged indices).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of one wavefront, in int4: the tile's member slots (uint16, 8 per
// int4), then the states of its distinct members (two int4 each).
__host__ __device__ constexpr int slot_int4(int rows4) { return rows4 * kTile / 2; }
__host__ __device__ constexpr int stage_int4(int rows4, int ustride) {
  return slot_int4(rows4) + 2 * ustride;
}

// Selection of one variable from its stencils' coefficients, in two parts so
// that the small stencils' part can run while the large stencil's rows
// stream in.  Small part: TENO step two over the small stencils (Sec. 3.3)
// and their mean, or the CWENO sums of alpha_k a^k and d_k a^k (Sec. 2.4).
template <bool CW>
struct SmallPart {
  unsigned nsm = 0;  // kept small stencils (bit k)
  int ties = 0;      // near ties among the small stencils' chi
  double ssum = 0.0; // sum of their gammas (TENO) or alphas (CWENO)
  double asm_[5];    // mean of the kept ones (TENO) or sum alpha_k a^k (CWENO)
  double dsm[CW ? 5 : 1];  // CWENO: sum d_k a^k
};

// bcoef(k, l) and coef(k, l): coefficient l of small stencil k, read for
// the indicators and for the combination (a caller may recompute it rather
// than hold all fifteen values).  Both are called by all lanes of a cell
// together, never under a lane-dependent condition.
template <bool CW, bool UP = false, class BCoef, class CCoef>
__device__ __forceinline__ void small_part(const ReconArgs& a, bool frozen, unsigned nib_in,
                                           BCoef&& bcoef, CCoef&& coef, SmallPart<CW>& sp) {
  auto beta = [&](int k) {
    double w[5];
#pragma unroll
    for (int l = 0; l < 5; ++l) w[l] = bcoef(k, l);
    return smoothness<2, UP>(w);
  };
  sp.nsm = nib_in & 7u;
  if (!CW && !frozen && a.variant == 0) {
    const double g0 = gamma_k(beta(0), a.eps, a.power);
    const double g1 = gamma_k(beta(1), a.eps, a.power);
    const double g2 = gamma_k(beta(2), a.eps, a.power);
    sp.ssum = (g0 + g1) + g2;
    const double is = 1.0 / sp.ssum;
    const double x0 = g0 * is, x1 = g1 * is, x2 = g2 * is;
    sp.ties += near_tie(a, x0) + near_tie(a, x1) + near_tie(a, x2);
    sp.nsm = (x0 >= a.ct ? 1u : 0u) | (x1 >= a.ct ? 2u : 0u) | (x2 >= a.ct ? 4u : 0u);
  }
  if constexpr (!CW) {
    const unsigned nsm = sp.nsm;
    const int cnt = (int)(nsm & 1u) + (int)((nsm >> 1) & 1u) + (int)((nsm >> 2) & 1u);
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      // read outside the lane-dependent conditions: a coefficient formed by
      // quad broadcasts needs all four lanes of the cell active
      const double c0 = coef(0, l), c1 = coef(1, l), c2 = coef(2, l);
      double acc = 0.0;
      if (nsm & 1u) acc += c0;
      if (nsm & 2u) acc += c1;
      if (nsm & 4u) acc += c2;
      sp.asm_[l] = cnt > 0 ? acc / (double)cnt : 0.0;
    }
  } else {
    // alpha_k = d_k / (beta_k + eps)^power of the small stencils; their
    // shares of the combination are finished once the large stencil's
    // weight is known
    const double w0 = a.cw_ds * gamma_k(beta(0), a.eps, a.power);
    const double w1 = a.cw_ds * gamma_k(beta(1), a.eps, a.power);
    const double w2 = a.cw_ds * gamma_k(beta(2), a.eps, a.power);
    sp.ssum = (w0 + w1) + w2;
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      const double c0 = coef(0, l), c1 = coef(1, l), c2 = coef(2, l);
      sp.asm_[l] = (w0 * c0 + w1 * c1) + w2 * c2;
      sp.dsm[l] = a.cw_ds * ((c0 + c1) + c2);
    }
  }
}

// Large part: TENO step one (Sec. 3.2) and the selected coefficients, or
// the CWENO combination P = (w_K/d_K)(P_K - sum_k d_k P_k) + sum_k w_k P_k.
// ab gets the combined coefficients, nib the variable's 4-bit flag.
template <int P, bool CW, bool UP = false>
__device__ __forceinline__ void large_part(const ReconArgs& a, bool frozen, unsigned nib_in,
                                           const SmallPart<CW>& sp,
                                           const double (&aK)[OrderT<P>::NU],
                                           double (&ab)[OrderT<P>::NU], unsigned& nib, int& ties) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  if constexpr (CW) {
    const double wK = a.cw_dK * gamma_k(smoothness<O::R, UP>(aK), a.eps, a.power);
    const double iS = 1.0 / (sp.ssum + wK);
    const double cK = wK / a.cw_dK;
#pragma unroll
    for (int l = 0; l < NU; ++l)
      ab[l] = l < 5 ? (cK * (aK[l] - sp.dsm[l]) + sp.asm_[l]) * iS : (cK * aK[l]) * iS;
    nib = 0u;
  } else {
    bool keepK = true;
    if (frozen) {
      keepK = (nib_in & 8u) != 0;
    } else if (a.variant == 0) {
      const double gK = gamma_k(smoothness<O::R, UP>(aK), a.eps, a.power);
      const double chiK = gK / (sp.ssum + gK);
      ties += near_tie(a, chiK);
      keepK = chiK >= a.ct;
      if (!keepK) ties += sp.ties;
    }
    nib = keepK ? 8u : sp.nsm;
#pragma unroll
    for (int l = 0; l < NU; ++l) ab[l] = keepK ? aK[l] : (l < 5 ? sp.asm_[l] : 0.0);
  }
}

// Characteristic projection of lane variable v (Sec. 2.3): row v of L
// (char_lrow) and row v of R (char_rrow), where R's columns are the right
// eigenvectors of the Euler flux Jacobian in direction (nx, ny) at the cell
// mean u (quad lanes 0..3), for the speeds u.n - c, u.n (entropy), u.n
// (shear), u.n + c, and L = R^-1 in closed form (b1 = (gamma-1)/c^2,
// b2 = b1 |u|^2 / 2).  A mean that is not physical keeps the conservative
// variables (identity rows).  The two are formed apart, each when needed,
// to keep fewer registers live.
// The normal-independent part of the projection state, formed once per cell.
struct CharState {
  double ux, uy, q2, c, ic, H, b1, b2;
};
__device__ __forceinline__ CharState char_state(double u0, double g) {
  const double rho = quad_bcast<0>(u0), mx = quad_bcast<1>(u0), my = quad_bcast<2>(u0),
               en = quad_bcast<3>(u0);
  CharState S;
  const double ir = 1.0 / rho;
  S.ux = mx * ir;
  S.uy = my * ir;
  S.q2 = S.ux * S.ux + S.uy * S.uy;
  const double p = (g - 1.0) * (en - 0.5 * rho * S.q2);
  S.c = sqrt(g * p * ir);
  S.ic = 1.0 / S.c;
  S.H = (en + p) * ir;
  S.b1 = (g - 1.0) * S.ic * S.ic;
  S.b2 = 0.5 * S.q2 * S.b1;
  return S;
}

// The part of the state that costs a division or a square root (u = m / rho,
// c, 1 / c), kept across a cell's edges where registers allow; the rest is
// formed again from it on each edge, with H = c^2 / (gamma - 1) + |u|^2 / 2.
struct CharCore {
  double ux, uy, c, ic;
};
__device__ __forceinline__ CharCore char_core(const CharState& S) { return {S.ux, S.uy, S.c, S.ic}; }
__device__ __forceinline__ CharState char_expand(CharCore K, double g) {
  // opaque copies: left visible, the expansion is the same on every edge
  // and the compiler forms it once and holds all of it
  asm volatile("" : "+v"(K.ux), "+v"(K.uy), "+v"(K.c), "+v"(K.ic));
  CharState S;
  S.ux = K.ux;
  S.uy = K.uy;
  S.q2 = K.ux * K.ux + K.uy * K.uy;
  S.c = K.c;
  S.ic = K.ic;
  S.H = K.c * K.c / (g - 1.0) + 0.5 * S.q2;
  S.b1 = (g - 1.0) * K.ic * K.ic;
  S.b2 = 0.5 * S.q2 * S.b1;
  return S;
}

__device__ __forceinline__ void char_lrow(const CharState& S, double nx, double ny, bool ok, int v,
                                          double (&lrow)[4]) {
  if (!ok) {
#pragma unroll
    for (int j = 0; j < 4; ++j) lrow[j] = (j == v) ? 1.0 : 0.0;
    return;
  }
  const double un = S.ux * nx + S.uy * ny, ut = S.uy * nx - S.ux * ny;
  const double b1 = S.b1, b2 = S.b2, ic = S.ic;
  const double L[4][4] = {
      {0.5 * (b2 + un * ic), -0.5 * (b1 * S.ux + nx * ic), -0.5 * (b1 * S.uy + ny * ic), 0.5 * b1},
      {1.0 - b2, b1 * S.ux, b1 * S.uy, -b1},
      {-ut, -ny, nx, 0.0},
      {0.5 * (b2 - un * ic), -0.5 * (b1 * S.ux - nx * ic), -0.5 * (b1 * S.uy - ny * ic), 0.5 * b1}};
#pragma unroll
  for (int j = 0; j < 4; ++j) lrow[j] = pick4(L[0][j], L[1][j], L[2][j], L[3][j], v);
}

__device__ __forceinline__ void char_rrow(const CharState& S, double nx, double ny, bool ok, int v,
                                          double (&rrow)[4]) {
  if (!ok) {
#pragma unroll
    for (int j = 0; j < 4; ++j) rrow[j] = (j == v) ? 1.0 : 0.0;
    return;
  }
  const double un = S.ux * nx + S.uy * ny, ut = S.uy * nx - S.ux * ny;
  const double R[4][4] = {{1.0, 1.0, 0.0, 1.0},
                          {S.ux - S.c * nx, S.ux, -ny, S.ux + S.c * nx},
                          {S.uy - S.c * ny, S.uy, nx, S.uy + S.c * ny},
                          {S.H - S.c * un, 0.5 * S.q2, ut, S.H + S.c * un}};
#pragma unroll
  for (int j = 0; j < 4; ++j) rrow[j] = pick4(R[0][j], R[1][j], R[2][j], R[3][j], v);
}

// sum_j row[j] x_j, x_j = lane j's x of this cell's quad.  Operand and
// result pass through opaque copies, which keep each product whole and in
// order: the broadcasts of a coefficient are the same on every edge, and
// left visible the compiler forms them all ahead of their use and holds
// four copies of every coefficient across the edges.
__device__ __forceinline__ double quad_dot(const double (&row)[4], double x) {
  asm volatile("" : "+v"(x));
  double s = row[0] * quad_bcast<0>(x);
  s = fma(row[1], quad_bcast<1>(x), s);
  s = fma(row[2], quad_bcast<2>(x), s);
  s = fma(row[3], quad_bcast<3>(x), s);
  asm volatile("" : "+v"(s));
  return s;
}

// Characteristic-variable phase of one cell (Sec. 2.3), after the
// least-squares phase: for each local edge, project the coefficients of
// all four stencils onto the edge's characteristic variables (lane v:
// variable v), select (or weight) per variable, evaluate at the edge's
// Gauss points and map back.  Edges run one after another (a loop, not
// unrolled) so that only one edge's projected coefficients are live; each
// edge's states and flags are written as soon as they are known and
// overwritten if the cell falls back to first order.
template <int P, int NQ, bool CW>
__device__ __forceinline__ void char_edges(const ReconArgs& a, const double (&as)[3][5],
                                           const double (&aK)[OrderT<P>::NU], double u0, int cell,
                                           bool live, bool writer, int g, int v) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  const bool avg_ok = physical(quad_bcast<0>(u0), quad_bcast<1>(u0), quad_bcast<2>(u0),
                               quad_bcast<3>(u0), a.gamma);
  const double* __restrict__ gc = a.geo + (size_t)(live ? cell : 0) * 10;
  const int side = a.nbinfo[live ? cell : 0].w;  // face normals point out of the L side
  int ties = 0;
  bool fp_ok = true;
  // TENO keeps the costly part of the projection state across the edges;
  // CWENO, with more registers live, forms it again on each edge
  constexpr bool keep_core = !CW;
  // the indicators from the doubled upper triangles (half the multiply-adds)
  // where that keeps the kernel's waves per SIMD: TENO up to order 5; at
  // order 6 and for CWENO it costs a wave and measured 6-9% slower
  constexpr bool kUpper = !CW && P <= 5;
  const CharCore core = keep_core ? char_core(char_state(u0, a.gamma)) : CharCore{};
  auto state = [&]() { return keep_core ? char_expand(core, a.gamma) : char_state(u0, a.gamma); };
  static_for<0, 3>([&](auto E) {
    constexpr int e = E;
    // one edge at a time: keeps the scheduler from overlapping the edges
    __builtin_amdgcn_sched_barrier(0);
    // outward unit normal of edge e
    const double sg = ((side >> (6 + e)) & 1) ? 1.0 : -1.0;
    const double nx = sg * gc[3 * e], ny = sg * gc[3 * e + 1];
    double wK[NU], ab[NU];
    SmallPart<CW> sp;
    {
      double lrow[4];
      char_lrow(state(), nx, ny, avg_ok, v, lrow);
#pragma unroll
      for (int l = 0; l < NU; ++l) wK[l] = quad_dot(lrow, aK[l]);
      // The small stencils' projected coefficients are held for the
      // indicators and the combination where that keeps the kernel's waves
      // per SIMD (CWENO, orders 3 and 5); for TENO at orders 4 and 6 holding
      // them costs a wave per SIMD (120 -> 134, 164 -> 178 VGPRs) and
      // projecting them twice measured faster.
      constexpr bool hold = CW || P == 3 || P == 5;
      if constexpr (!hold) {
        auto proj = [&](int k, int l) { return quad_dot(lrow, as[k][l]); };
        small_part<CW, kUpper>(a, false, 8u, proj, proj, sp);
      } else {
        double ws[3][5];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 5; ++l) ws[k][l] = quad_dot(lrow, as[k][l]);
        auto held = [&](int k, int l) { return ws[k][l]; };
        small_part<CW, kUpper>(a, false, 8u, held, held, sp);
      }
    }
    unsigned nib = 0u;
    large_part<P, CW, kUpper>(a, false, 8u, sp, wK, ab, nib, ties);
    double rrow[4];
    char_rrow(state(), nx, ny, avg_ok, v, rrow);
    const double* __restrict__ fb = &FaceBasis<O::R, NQ>::P.v[e * NQ][0];
#pragma unroll
    for (int kq = 0; kq < NQ; ++kq) {
      double dw = 0.0;
#pragma unroll
      for (int l = 0; l < NU; ++l) dw = fma(ab[l], fb[kq * NU + l], dw);
      const double val = u0 + quad_dot(rrow, dw);
      fp_ok = fp_ok && physical(quad_bcast<0>(val), quad_bcast<1>(val), quad_bcast<2>(val),
                                quad_bcast<3>(val), a.gamma);
      if (live && writer) a.fp[((size_t)(e * NQ + kq) * a.n_pad + cell) * 4 + v] = val;
    }
    if (a.flags) {  // one word per local edge: flags[e][n_cell]
      unsigned f = nib << (4 * v);
      f |= __shfl_xor(f, 1);
      f |= __shfl_xor(f, 2);
      if (live && g == 0) a.flags[(size_t)e * a.n_cell + cell] = (uint16_t)f;
    }
  });
  __builtin_amdgcn_sched_barrier(0);
  // ---- non-physical states (all four lanes of a cell agree) ----
  if (live && g == 0 && !(avg_ok && fp_ok)) {
    atomicAdd(&a.diag->nonphysical, 1ull);
    atomicMin(&a.diag->first_bad, (long long)a.user_of[cell]);
  }
  if (!fp_ok && avg_ok && a.fallback) {
    if (live && writer)
      for (int q = 0; q < 3 * NQ; ++q) a.fp[((size_t)q * a.n_pad + cell) * 4 + v] = u0;
    if (a.flags && live && g == 0)
      for (int e = 0; e < 3; ++e) a.flags[(size_t)e * a.n_cell + cell] = 0;
    if (live && g == 0) atomicAdd(&a.diag->fallbacks, 1ull);
  }
  if (live && writer && ties) atomicAdd(&a.diag->near_ties, (unsigned long long)ties);
}

// Reconstruction of one tile of kTile cells by one wavefront; `stage` is
// this wavefront's LDS area (stage_int4(ROWS4, a.ustride) int4).  CW selects the
// CWENO weighting (Sec. 2.4) instead of the TENO selection (Sec. 3); CH
// selects in characteristic variables, edge by edge (Sec. 2.3).
#ifndef TENO_CHAR_GRAM
#define TENO_CHAR_GRAM 1
#endif
// Characteristic TENO (and Linear) without projecting the coefficients for
// the indicators.  For each stencil the Gram matrix G = sum_lm B_lm a_l a_m^T
// of the four variables' coefficient vectors (4 x 4, symmetric) is formed
// once per cell; the indicator of characteristic variable v on an edge is
// then L_v^T G L_v, which equals beta of the projected coefficients L_v a.
// The selection follows per variable.  Where the four variables of a cell
// select alike on an edge (every smooth cell, and any jump that all fields
// see), the projection cancels (R L = I) and the face states are the
// conservative combination of the same stencils; only cells whose fields
// select differently project the coefficients and map back, as in
// char_edges.  The Gram matrices live in the wave's staging LDS (16 cells x
// 4 stencils x 10 entries), which the least-squares phase no longer needs.
constexpr int kCharGramDoubles = kTile * 4 * 10;
__host__ __device__ constexpr int char_gram_int4() { return kCharGramDoubles * 8 / 16; }

__device__ __forceinline__ int gram_off(int i, int j) {  // i <= j
  return i * 4 - (i * (i - 1)) / 2 + (j - i);
}

// Row v of the Gram matrix of one stencil, G_vj = (a^j)^T B a^v, from the
// factor B = L D L^T: with z = L^T a, G_vj = sum_l d_l z^v_l z^j_l.  One
// component of z at a time; the empty asm ties each step to the previous
// step's sums so that the compiler does not form all of z up front.
template <int R>
__device__ __forceinline__ void gram_rows(const double* a, int v, double* G) {
  using S = SmoothForm<R>;
  constexpr int N = S::N;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    double z = a[l];
    asm volatile("" : "+v"(z), "+v"(r0), "+v"(r1), "+v"(r2), "+v"(r3));
#pragma unroll
    for (int m = l + 1; m < N; ++m) z = fma(S::LDL.Lt[l][m], a[m], z);
    const double w = S::LDL.d[l] * z;
    r0 = fma(quad_bcast<0>(z), w, r0);
    r1 = fma(quad_bcast<1>(z), w, r1);
    r2 = fma(quad_bcast<2>(z), w, r2);
    r3 = fma(quad_bcast<3>(z), w, r3);
  }
  const double r[4] = {r0, r1, r2, r3};
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (j >= v) G[gram_off(v, j)] = r[j];
}

// Row v of the left eigenvector matrix for edge normal (nx, ny), formed
// directly for the lane's own variable: with
//   A = (b2, -b1 ux, -b1 uy, b1), B = (un, -nx, -ny, 0) / c, C = (-ut, -ny, nx, 0)
// the rows are A/2 + B/2 (v = 0), (1, 0, 0, 0) - A (v = 1), C (v = 2) and
// A/2 - B/2 (v = 3), the same matrix as char_lrow.
__device__ __forceinline__ void char_lrow_lane(const CharState& S, double nx, double ny, bool ok,
                                               int v, double (&lrow)[4]) {
  const double un = S.ux * nx + S.uy * ny, ut = S.uy * nx - S.ux * ny;
  const double ca = v == 1 ? -1.0 : (v == 2 ? 0.0 : 0.5);
  const double cb = v == 0 ? 0.5 : (v == 3 ? -0.5 : 0.0);
  const double cc = v == 2 ? 1.0 : 0.0;
  const double cd = v == 1 ? 1.0 : 0.0;
  const double A[4] = {S.b2, -S.b1 * S.ux, -S.b1 * S.uy, S.b1};
  const double B[4] = {un * S.ic, -nx * S.ic, -ny * S.ic, 0.0};
  const double Cv[4] = {-ut, -ny, nx, 0.0};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double r = fma(ca, A[j], fma(cb, B[j], cc * Cv[j])) + (j == 0 ? cd : 0.0);
    lrow[j] = ok ? r : (j == v ? 1.0 : 0.0);
  }
}

// The ten products of a row L that pair with the stored entries of G
// (diagonal once, off-diagonal doubled), in gram_off order.
__device__ __forceinline__ void gram_weights(const double (&L)[4], double (&q)[10]) {
  const double t0 = L[0] + L[0], t1 = L[1] + L[1], t2 = L[2] + L[2];
  q[0] = L[0] * L[0];
  q[1] = t0 * L[1];
  q[2] = t0 * L[2];
  q[3] = t0 * L[3];
  q[4] = L[1] * L[1];
  q[5] = t1 * L[2];
  q[6] = t1 * L[3];
  q[7] = L[2] * L[2];
  q[8] = t2 * L[3];
  q[9] = L[3] * L[3];
}

__device__ __forceinline__ double gram_dot(const double* G, const double (&q)[10]) {
  double s = q[0] * G[0];
#pragma unroll
  for (int k = 1; k < 10; ++k) s = fma(q[k], G[k], s);
  return s;
}

template <int P, int NQ>
__device__ __forceinline__ void char_edges_gram(const ReconArgs& a, const double (&as)[3][5],
                                                const double (&aK)[OrderT<P>::NU], double u0,
                                                int cell, bool live, bool writer, int g, int v,
                                                int c, int4* stage) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  const bool avg_ok = physical(quad_bcast<0>(u0), quad_bcast<1>(u0), quad_bcast<2>(u0),
                               quad_bcast<3>(u0), a.gamma);
  const double* __restrict__ gc = a.geo + (size_t)(live ? cell : 0) * 10;
  const int side = a.nbinfo[live ? cell : 0].w;  // face normals point out of the L side
  // ---- Gram matrices of the four stencils (the staging LDS is free now) ----
  double* gram = reinterpret_cast<double*>(stage) + c * 40;
  wave_lds_sync();
  if (a.variant == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) gram_rows<2>(as[k], v, gram + 10 * k);
  }
  gram_rows<O::R>(aK, v, gram + 30);
  wave_lds_sync();
  int ties = 0;
  bool fp_ok = true;
  const CharCore core = char_core(char_state(u0, a.gamma));
  auto state = [&]() { return char_expand(core, a.gamma); };
  static_for<0, 3>([&](auto E) {
    constexpr int e = E;
    __builtin_amdgcn_sched_barrier(0);
    const double sg = ((side >> (6 + e)) & 1) ? 1.0 : -1.0;
    const double nx = sg * gc[3 * e], ny = sg * gc[3 * e + 1];
    double lrow[4];
    char_lrow_lane(state(), nx, ny, avg_ok, v, lrow);
    // ---- selection of characteristic variable v (Sec. 3.2-3.3) ----
    unsigned nib = 8u;
    if (a.variant == 0) {
      // an opaque offset per edge keeps the 40 Gram entries from being read
      // once and held in registers across the three edges
      int goff = c * 40;
      asm volatile("" : "+v"(goff));
      const double* gram = reinterpret_cast<const double*>(stage) + goff;
      double q[10];
      gram_weights(lrow, q);
      const double g0 = gamma_k(gram_dot(gram, q), a.eps, a.power);
      const double g1 = gamma_k(gram_dot(gram + 10, q), a.eps, a.power);
      const double g2 = gamma_k(gram_dot(gram + 20, q), a.eps, a.power);
      const double ssum = (g0 + g1) + g2;
      const double is = 1.0 / ssum;
      const double x0 = g0 * is, x1 = g1 * is, x2 = g2 * is;
      const int st = near_tie(a, x0) + near_tie(a, x1) + near_tie(a, x2);
      const unsigned nsm = (x0 >= a.ct ? 1u : 0u) | (x1 >= a.ct ? 2u : 0u) | (x2 >= a.ct ? 4u : 0u);
      const double gK = gamma_k(gram_dot(gram + 30, q), a.eps, a.power);
      const double chiK = gK / (ssum + gK);
      ties += near_tie(a, chiK);
      const bool keepK = chiK >= a.ct;
      if (!keepK) ties += st;
      nib = keepK ? 8u : nsm;
    }
    // ---- do the cell's four variables select alike? ----
    const unsigned n0 = (unsigned)__builtin_amdgcn_mov_dpp((int)nib, 0x00, 0xF, 0xF, false);
    const unsigned n1 = (unsigned)__builtin_amdgcn_mov_dpp((int)nib, 0x55, 0xF, 0xF, false);
    const unsigned n2 = (unsigned)__builtin_amdgcn_mov_dpp((int)nib, 0xAA, 0xF, 0xF, false);
    const unsigned n3 = (unsigned)__builtin_amdgcn_mov_dpp((int)nib, 0xFF, 0xF, 0xF, false);
    const bool alike = n0 == n1 && n1 == n2 && n2 == n3;
    const double* __restrict__ fb = &FaceBasis<O::R, NQ>::P.v[e * NQ][0];
    // the combined coefficients one at a time, straight into the face sums
    const int cnt = (int)(nib & 1u) + (int)((nib >> 1) & 1u) + (int)((nib >> 2) & 1u);
    const double inv = cnt == 3 ? 1.0 / 3.0 : (cnt == 2 ? 0.5 : (cnt == 1 ? 1.0 : 0.0));
    double val[NQ];
    if (alike) {
      // the conservative combination of the stencils every field selected
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) val[kq] = u0;
#pragma unroll
      for (int l = 0; l < NU; ++l) {
        double ab = aK[l];
        if (l < 5 && !(nib & 8u)) {
          double sm = 0.0;
          if (nib & 1u) sm += as[0][l];
          if (nib & 2u) sm += as[1][l];
          if (nib & 4u) sm += as[2][l];
          ab = sm * inv;
        } else if (!(nib & 8u)) {
          ab = 0.0;
        }
#pragma unroll
        for (int kq = 0; kq < NQ; ++kq) val[kq] = fma(ab, fb[kq * NU + l], val[kq]);
      }
    } else {
      // fields select differently: project, combine per variable, map back
      double dw[NQ];
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) dw[kq] = 0.0;
#pragma unroll
      for (int l = 0; l < NU; ++l) {
        // every lane of the quad takes part in each projection (the four
        // variables of a cell may select differently here)
        double xk = aK[l];
        asm volatile("" : "+v"(xk), "+v"(dw[0]), "+v"(dw[NQ - 1]));
        const double wk = quad_dot(lrow, xk);
        double ab = (nib & 8u) ? wk : 0.0;
        if (l < 5) {
          double x0 = as[0][l], x1 = as[1][l], x2 = as[2][l];
          asm volatile("" : "+v"(x0), "+v"(x1), "+v"(x2) : "v"(wk));
          const double w0 = quad_dot(lrow, x0), w1 = quad_dot(lrow, x1), w2 = quad_dot(lrow, x2);
          double sm = 0.0;
          if (nib & 1u) sm += w0;
          if (nib & 2u) sm += w1;
          if (nib & 4u) sm += w2;
          if (!(nib & 8u)) ab = sm * inv;
        }
#pragma unroll
        for (int kq = 0; kq < NQ; ++kq) dw[kq] = fma(ab, fb[kq * NU + l], dw[kq]);
      }
      double rrow[4];
      char_rrow(state(), nx, ny, avg_ok, v, rrow);
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) val[kq] = u0 + quad_dot(rrow, dw[kq]);
    }
#pragma unroll
    for (int kq = 0; kq < NQ; ++kq) {
      fp_ok = fp_ok && physical(quad_bcast<0>(val[kq]), quad_bcast<1>(val[kq]),
                                quad_bcast<2>(val[kq]), quad_bcast<3>(val[kq]), a.gamma);
      if (live && writer) a.fp[((size_t)(e * NQ + kq) * a.n_pad + cell) * 4 + v] = val[kq];
    }
    if (a.flags) {  // one word per local edge: flags[e][n_cell]
      unsigned f = nib << (4 * v);
      f |= __shfl_xor(f, 1);
      f |= __shfl_xor(f, 2);
      if (live && g == 0) a.flags[(size_t)e * a.n_cell + cell] = (uint16_t)f;
    }
  });
  __builtin_amdgcn_sched_barrier(0);
  // ---- non-physical states (all four lanes of a cell agree) ----
  if (live && g == 0 && !(avg_ok && fp_ok)) {
    atomicAdd(&a.diag->nonphysical, 1ull);
    atomicMin(&a.diag->first_bad, (long long)a.user_of[cell]);
  }
  if (!fp_ok && avg_ok && a.fallback) {
    if (live && writer)
      for (int q = 0; q < 3 * NQ; ++q) a.fp[((size_t)q * a.n_pad + cell) * 4 + v] = u0;
    if (a.flags && live && g == 0)
      for (int e = 0; e < 3; ++e) a.flags[(size_t)e * a.n_cell + cell] = 0;
    if (live && g == 0) atomicAdd(&a.diag->fallbacks, 1ull);
  }
  if (live && writer && ties) atomicAdd(&a.diag->near_ties, (unsigned long long)ties);
}

// Characteristic CWENO (Sec. 2.4 in the variables of Sec. 2.3) with the
// indicators of char_edges_gram: the weights of variable v on an edge come
// from L_v^T G_k L_v.  The CWENO polynomial is a linear combination of the
// stencils' polynomials, P = lK P_K + sum_k l_k p_k with lK = (w_K/d_K)/S and
// l_k = (alpha_k - d_k w_K/d_K)/S, so each stencil is evaluated at the edge's
// Gauss points in conservative variables and only those point values are
// projected (four stencils x NQ points instead of every coefficient).
template <int P, int NQ>
__device__ __forceinline__ void char_edges_cweno_gram(const ReconArgs& a,
                                                      const double (&as)[3][5],
                                                      const double (&aK)[OrderT<P>::NU],
                                                      double u0, int cell, bool live,
                                                      bool writer, int g, int v, int c,
                                                      int4* stage) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  const bool avg_ok = physical(quad_bcast<0>(u0), quad_bcast<1>(u0), quad_bcast<2>(u0),
                               quad_bcast<3>(u0), a.gamma);
  const double* __restrict__ gc = a.geo + (size_t)(live ? cell : 0) * 10;
  const int side = a.nbinfo[live ? cell : 0].w;  // face normals point out of the L side
  double* gram = reinterpret_cast<double*>(stage) + c * 40;
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 3; ++k) gram_rows<2>(as[k], v, gram + 10 * k);
  gram_rows<O::R>(aK, v, gram + 30);
  wave_lds_sync();
  bool fp_ok = true;
  const CharCore core = char_core(char_state(u0, a.gamma));
  auto state = [&]() { return char_expand(core, a.gamma); };
  static_for<0, 3>([&](auto E) {
    constexpr int e = E;
    __builtin_amdgcn_sched_barrier(0);
    const double sg = ((side >> (6 + e)) & 1) ? 1.0 : -1.0;
    const double nx = sg * gc[3 * e], ny = sg * gc[3 * e + 1];
    double lrow[4];
    char_lrow_lane(state(), nx, ny, avg_ok, v, lrow);
    int goff = c * 40;
    asm volatile("" : "+v"(goff));
    const double* gm = reinterpret_cast<const double*>(stage) + goff;
    double q[10];
    gram_weights(lrow, q);
    const double w0 = a.cw_ds * gamma_k(gram_dot(gm, q), a.eps, a.power);
    const double w1 = a.cw_ds * gamma_k(gram_dot(gm + 10, q), a.eps, a.power);
    const double w2 = a.cw_ds * gamma_k(gram_dot(gm + 20, q), a.eps, a.power);
    const double wK = a.cw_dK * gamma_k(gram_dot(gm + 30, q), a.eps, a.power);
    const double iS = 1.0 / (((w0 + w1) + w2) + wK);
    const double cK = wK / a.cw_dK;
    const double lK = cK * iS;
    const double l0 = (w0 - cK * a.cw_ds) * iS, l1 = (w1 - cK * a.cw_ds) * iS,
                 l2 = (w2 - cK * a.cw_ds) * iS;
    double rrow[4];
    char_rrow(state(), nx, ny, avg_ok, v, rrow);
    const double* __restrict__ fb = &FaceBasis<O::R, NQ>::P.v[e * NQ][0];
#pragma unroll
    for (int kq = 0; kq < NQ; ++kq) {
      // the four stencils' values of the lane's conservative variable
      double pK = 0.0, p0 = 0.0, p1 = 0.0, p2 = 0.0;
#pragma unroll
      for (int l = 0; l < NU; ++l) pK = fma(aK[l], fb[kq * NU + l], pK);
#pragma unroll
      for (int l = 0; l < 5; ++l) {
        p0 = fma(as[0][l], fb[kq * NU + l], p0);
        p1 = fma(as[1][l], fb[kq * NU + l], p1);
        p2 = fma(as[2][l], fb[kq * NU + l], p2);
      }
      const double dw = lK * quad_dot(lrow, pK) +
                        ((l0 * quad_dot(lrow, p0) + l1 * quad_dot(lrow, p1)) +
                         l2 * quad_dot(lrow, p2));
      const double val = u0 + quad_dot(rrow, dw);
      fp_ok = fp_ok && physical(quad_bcast<0>(val), quad_bcast<1>(val), quad_bcast<2>(val),
                                quad_bcast<3>(val), a.gamma);
      if (live && writer) a.fp[((size_t)(e * NQ + kq) * a.n_pad + cell) * 4 + v] = val;
    }
    if (a.flags && live && g == 0) a.flags[(size_t)e * a.n_cell + cell] = 0;
  });
  __builtin_amdgcn_sched_barrier(0);
  // ---- non-physical states (all four lanes of a cell agree) ----
  if (live && g == 0 && !(avg_ok && fp_ok)) {
    atomicAdd(&a.diag->nonphysical, 1ull);
    atomicMin(&a.diag->first_bad, (long long)a.user_of[cell]);
  }
  if (!fp_ok && avg_ok && a.fallback) {
    if (live && writer)
      for (int q = 0; q < 3 * NQ; ++q) a.fp[((size_t)q * a.n_pad + cell) * 4 + v] = u0;
    if (live && g == 0) atomicAdd(&a.diag->fallbacks, 1ull);
  }
}

#ifndef TENO_CHAR_CWENO_GRAM
#define TENO_CHAR_CWENO_GRAM 1
#endif
template <int P, int NQ, bool CW = false, bool CH = false>
__device__ __forceinline__ void reconstruct_tile(const ReconArgs& a, int tile, int lane,
                                                 int4* stage) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  constexpr int NP = 3 * NQ;
  static_assert(!CH || kLanesPerCell == 4, "the projection shares values within a quad");
  // stage this tile's member slots ([row4][cell][4] uint16) and the states
  // of its distinct stencil members in LDS
  wave_lds_sync();  // earlier readers of `stage` are done
  {
    constexpr int NS = slot_int4(O::ROWS4);
    const int4* __restrict__ src = a.slot + (size_t)tile * NS;
    for (int i = lane; i < NS; i += 64) stage[i] = src[i];
    double2* ust = reinterpret_cast<double2*>(stage + NS);
    const int* __restrict__ mem = a.tmem + (size_t)tile * a.ustride;
    for (int i = lane; i < a.ustride; i += 64) {
      const double2* u = reinterpret_cast<const double2*>(a.U + (size_t)mem[i] * 4);
      ust[2 * i] = u[0];
      ust[2 * i + 1] = u[1];
    }
  }
  wave_lds_sync();
  const uint16_t* sidx = reinterpret_cast<const uint16_t*>(stage);
  const double* us = reinterpret_cast<const double*>(stage + slot_int4(O::ROWS4));
  // g: coefficient group of the lane within its cell; v = g % 4: the
  // variable it gathers and, in the selection phase, the variable it owns
  // (with 8 lanes per cell, lanes 4..7 repeat 0..3 and do not write).
  const int c = lane / kLanesPerCell, g = lane % kLanesPerCell, v = g & 3;
  const bool writer = g < 4;
  const int cell = tile * kTile + c;
  const bool live = cell < a.n_cell;
  const double u0 = a.U[(size_t)(live ? cell : 0) * 4 + v];
  // the tile's operator stream (JP doubles per cell) and its blocks; meshes
  // in conservative variables are dense
  constexpr bool D = !CH;
  constexpr int JP = O::template JPD<D>;
  const double* __restrict__ mt = reinterpret_cast<const double*>(a.M) + (size_t)tile * JP * kTile;
  auto pairs = [&](int k) {
    return reinterpret_cast<const double2*>(mt + (size_t)block_start(k, D) * kTile) + c;
  };
  auto lanes = [&](int k) { return mt + (size_t)block_start(k, D) * kTile; };
  const bool frozen = a.frozen != 0;
  const unsigned nib_in = (frozen && live) ? ((a.flags[cell] >> (4 * v)) & 0xFu) : 8u;

  // ---- small stencils (rows 0..32), then step two of the selection, which
  //      needs only their indicators.  Each stream is started before the
  //      previous stencil's coefficients are gathered, and the large
  //      stencil's first rows load during that last step ----
  constexpr bool LL = large_lane_rows(O::NU, D), SL = lane_rows(kSmallCoef, D);
  using LargeS = std::conditional_t<LL, RowLanes<33, O::NL, O::NU>,
                                    RowStream<33, O::NL, stored_row(O::NU)>>;
  double u0q[4] = {u0, u0, u0, u0};
  if constexpr (LL || SL) {
    u0q[0] = quad_bcast<0>(u0);
    u0q[1] = quad_bcast<1>(u0);
    u0q[2] = quad_bcast<2>(u0);
    u0q[3] = quad_bcast<3>(u0);
  }
  auto make_large = [&]() {
    if constexpr (LL)
      return LargeS{us, sidx, lanes(3), c, g, {u0q[0], u0q[1], u0q[2], u0q[3]}};
    else
      return LargeS{us, sidx, pairs(3), c, g, u0};
  };
  LargeS ls = make_large();
  double as[3][5];
  {
    using S0 = std::conditional_t<SL, RowLanes<0, 11, 5>, RowStream<0, 11, stored_row(5)>>;
    using S1 = std::conditional_t<SL, RowLanes<11, 11, 5>, RowStream<11, 11, stored_row(5)>>;
    using S2 = std::conditional_t<SL, RowLanes<22, 11, 5>, RowStream<22, 11, stored_row(5)>>;
    auto make = [&](auto tag, int k) {
      using S = typename decltype(tag)::type;
      if constexpr (SL)
        return S{us, sidx, lanes(k), c, g, {u0q[0], u0q[1], u0q[2], u0q[3]}};
      else
        return S{us, sidx, pairs(k), c, g, u0};
    };
    S0 s0 = make(TypeTag<S0>{}, 0);
    S1 s1 = make(TypeTag<S1>{}, 1);
    S2 s2 = make(TypeTag<S2>{}, 2);
    typename S0::Acc sk0 = {}, sk1 = {}, sk2 = {};
    s0.prime();
    s0.run(sk0);
    s1.prime();
    static_for<0, 5>([&](auto L) { as[0][L] = S0::template coef<L>(sk0, v, lane); });
    s1.run(sk1);
    s2.prime();
    static_for<0, 5>([&](auto L) { as[1][L] = S1::template coef<L>(sk1, v, lane); });
    s2.run(sk2);
    ls.prime();
    static_for<0, 5>([&](auto L) { as[2][L] = S2::template coef<L>(sk2, v, lane); });
  }
  SmallPart<CW> sp;
  if constexpr (!CH) {
    auto c = [&](int k, int l) { return as[k][l]; };
    small_part<CW>(a, frozen, nib_in, c, c, sp);
  }

  // ---- large stencil (rows 33.., entries 165..) ----
  double aK[NU];
  {
    typename LargeS::Acc sk = {};
    ls.run(sk);
    static_for<0, NU>([&](auto L) { aK[L] = LargeS::template coef<L>(sk, v, lane); });
  }
  if constexpr (CH) {
#if TENO_CHAR_GRAM
    if constexpr (!CW)
      char_edges_gram<P, NQ>(a, as, aK, u0, cell, live, writer, g, v, c, stage);
    else if constexpr (TENO_CHAR_CWENO_GRAM)
      char_edges_cweno_gram<P, NQ>(a, as, aK, u0, cell, live, writer, g, v, c, stage);
    else
#endif
      char_edges<P, NQ, CW>(a, as, aK, u0, cell, live, writer, g, v);
    return;
  }
  int ties = 0;
  unsigned nib = 0u;
  double val[NP];
  {
    double ab[NU];
    large_part<P, CW>(a, frozen, nib_in, sp, aK, ab, nib, ties);
    // ---- face Gauss points (variable v of this cell) ----
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      double s = u0;
#pragma unroll
      for (int l = 0; l < NU; ++l) s = fma(ab[l], FaceBasis<O::R, NQ>::P.v[q][l], s);
      val[q] = s;
    }
  }
  // ---- non-physical states (all four lanes of a cell agree) ----
  if (!frozen) {
    const bool avg_ok = physical(quad_bcast<0>(u0), quad_bcast<1>(u0), quad_bcast<2>(u0),
                                 quad_bcast<3>(u0), a.gamma);
    bool fp_ok = true;
#pragma unroll
    for (int q = 0; q < NP; ++q)
      fp_ok = fp_ok && physical(quad_bcast<0>(val[q]), quad_bcast<1>(val[q]),
                                quad_bcast<2>(val[q]), quad_bcast<3>(val[q]), a.gamma);
    if (live && g == 0 && !(avg_ok && fp_ok)) {  // one lane per cell
      atomicAdd(&a.diag->nonphysical, 1ull);
      atomicMin(&a.diag->first_bad, (long long)a.user_of[cell]);
    }
    if (!fp_ok && avg_ok && a.fallback) {
#pragma unroll
      for (int q = 0; q < NP; ++q) val[q] = u0;
      nib = 0u;
      if (live && g == 0) atomicAdd(&a.diag->fallbacks, 1ull);
    }
    if (live && writer && ties) atomicAdd(&a.diag->near_ties, (unsigned long long)ties);
  }
  if (live && writer) {
#pragma unroll
    for (int q = 0; q < NP; ++q) a.fp[((size_t)q * a.n_pad + cell) * 4 + v] = val[q];
  }
  if (!frozen && a.flags) {
    unsigned f = nib << (4 * v);
    f |= __shfl_xor(f, 1);
    f |= __shfl_xor(f, 2);
    if (live && g == 0) a.flags[cell] = (uint16_t)f;
  }
}

// Per-order occupancy targets (waves per SIMD; 1 leaves the budget to the
// compiler): TENO at order 3 in rows-by-lane blocks needs 132 registers left
// alone and runs faster held to 128 (four waves); TENO at order 5 (130
// registers, 2 spilled when held to 128) measured 1% faster at four waves
// with one wavefront per block.  The other kernels measured best
// unconstrained (order 4 and CWENO 6 lose 10-14% at four waves).
template <int P, bool CW>
struct ReconWaves {
  static constexpr int value = TENO_RECON_WAVES_PER_EU > 0 ? TENO_RECON_WAVES_PER_EU
                               : ((P == 3 || P == 5) && !CW && lane_rows(kSmallCoef, true)) ? 4
                                                                                        : 1;
};

// Wavefronts per block of the reconstruction kernels (one tile each).  One
// wavefront per block lets the dispatcher start each tile on its own, so
// the streaming and selection phases of the wavefronts on a SIMD drift
// apart; it measured 1.5-3% faster than four per block.
#ifndef TENO_RECON_BLOCK_WAVES
#define TENO_RECON_BLOCK_WAVES 1
#endif
constexpr int kReconBlockWaves = TENO_RECON_BLOCK_WAVES;

template <int P, int NQ, bool CW>
__global__ __launch_bounds__(64 * kReconBlockWaves)
__attribute__((amdgpu_waves_per_eu(ReconWaves<P, CW>::value)))
void k_reconstruct(ReconArgs a) {
  extern __shared__ int4 lds[];  // kReconBlockWaves wavefronts x a.lds_stride
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = xcd_remap(blockIdx.x, gridDim.x) * kReconBlockWaves + wave;
  if (tile >= a.n_tiles) return;  // whole wavefront leaves together
  reconstruct_tile<P, NQ, CW, false>(a, tile, lane, lds + wave * a.lds_stride);
}

// The same in characteristic variables.  The TENO kernel's register budget
// is capped at TENO_CHAR_WAVES_PER_EU wavefronts per SIMD (left alone, the
// order-6 kernel takes 175 VGPRs and two waves); the CWENO kernel, which
// holds the projected coefficients of every stencil across its weights, is
// left to the compiler.
#ifndef TENO_CHAR_WAVES_PER_EU
#define TENO_CHAR_WAVES_PER_EU 3
#endif
template <bool CW>
struct CharWaves {
  static constexpr int value = (!CW && TENO_CHAR_WAVES_PER_EU > 0) ? TENO_CHAR_WAVES_PER_EU : 1;
};
template <int P, int NQ, bool CW>
__global__ __launch_bounds__(64 * kReconBlockWaves)
__attribute__((amdgpu_waves_per_eu(CharWaves<CW>::value)))
void k_reconstruct_char(ReconArgs a) {
  extern __shared__ int4 lds[];  // kReconBlockWaves wavefronts x a.lds_stride
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = xcd_remap(blockIdx.x, gridDim.x) * kReconBlockWaves + wave;
  if (tile >= a.n_tiles) return;  // whole wavefront leaves together
  reconstruct_tile<P, NQ, CW, true>(a, tile, lane, lds + wave * a.lds_stride);
}

// ---------------------------------------------------------------------------
// flux, residual, Runge-Kutta stage
// ---------------------------------------------------------------------------
// Flux and residual (Sec. 2.1, Sec. 4), in two launches.
//  face_flux    one lane per face (faces sorted by their L cell): rotated HLL
//               at the N_q point pairs (L point k with R point N_q-1-k),
//               Gauss quadrature, Phi_f = |A| sum_k w_k F_k, written once.
//  cell_update  one lane per cell: R = -(1/|V|) sum_e s_e Phi_f(e) over its
//               three faces in local-edge order (s = +1 on the L side), then
//               the optional SSP-RK3 stage combine.  A gather: no atomics.
struct FaceFluxArgs {
  const double* __restrict__ fp;       // [3 nq][n_pad][4]
  const int4* __restrict__ fcell;      // [n_face]: L, R, eL | eR << 2, boundary index or -1
  const double2* __restrict__ fgeo;    // [n_face][2]: (nx, ny), (|A|, 0)
  double* __restrict__ phi;            // [n_face][4]
  const int* __restrict__ bkind;       // [n_bface] TENO_BC_*
  const double* __restrict__ bstate;   // [n_bface][4] prescribed states
  double gamma;
  int n_face, n_pad;
};

// Outer state of boundary face b at one Gauss point (normal (nx, ny) out of
// the domain): transmissive copies the inner state, reflective reverses its
// normal momentum, prescribed takes the given state.
__device__ __forceinline__ void boundary_state(int kind, const double* __restrict__ bstate, int b,
                                               const double uL[4], double nx, double ny,
                                               double uR[4]) {
  if (kind == TENO_BC_PRESCRIBED) {
#pragma unroll
    for (int c = 0; c < 4; ++c) uR[c] = bstate[4 * (size_t)b + c];
  } else if (kind == TENO_BC_REFLECTIVE) {
    const double mn = uL[1] * nx + uL[2] * ny;
    uR[0] = uL[0];
    uR[1] = uL[1] - 2.0 * mn * nx;
    uR[2] = uL[2] - 2.0 * mn * ny;
    uR[3] = uL[3];
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) uR[c] = uL[c];
  }
}

template <int NQ, bool BND = false>
__device__ __forceinline__ void face_flux(const FaceFluxArgs& a, int f, int b = -1) {
  const int4 fc = a.fcell[f];
  const double2 nrm = a.fgeo[2 * (size_t)f], len = a.fgeo[2 * (size_t)f + 1];
  const int eL = fc.z & 3, eR = (fc.z >> 2) & 3;
  const double2* fp2 = reinterpret_cast<const double2*>(a.fp);
  double phi[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const size_t oL = ((size_t)(eL * NQ + k) * a.n_pad + fc.x) * 2;
    const double2 l0 = fp2[oL], l1 = fp2[oL + 1];
    const double uL[4] = {l0.x, l0.y, l1.x, l1.y};
    double uR[4];
    if constexpr (BND) {
      boundary_state(a.bkind[b], a.bstate, b, uL, nrm.x, nrm.y, uR);
    } else {
      const size_t oR = ((size_t)(eR * NQ + NQ - 1 - k) * a.n_pad + fc.y) * 2;
      const double2 r0 = fp2[oR], r1 = fp2[oR + 1];
      uR[0] = r0.x;
      uR[1] = r0.y;
      uR[2] = r1.x;
      uR[3] = r1.y;
    }
    double F[4];
    hll(uL, uR, nrm.x, nrm.y, a.gamma, F);
#pragma unroll
    for (int c = 0; c < 4; ++c) phi[c] = phi[c] + FaceRule<NQ>::w[k] * F[c];
  }
  double2* out = reinterpret_cast<double2*>(a.phi) + 2 * (size_t)f;
  out[0] = make_double2(phi[0] * len.x, phi[1] * len.x);
  out[1] = make_double2(phi[2] * len.x, phi[3] * len.x);
}

// Every face, boundary faces included as if their outer side were the cell
// itself; k_boundary_flux then rewrites the boundary faces.
template <int NQ>
__global__ __launch_bounds__(256) void k_face_flux(FaceFluxArgs a) {
  const int f = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (f < a.n_face) face_flux<NQ>(a, f);
}

// Boundary faces only (after k_face_flux, same stream): bf[b] is the face
// index of boundary face b, whose outer state comes from its condition.
template <int NQ>
__global__ __launch_bounds__(256) void k_boundary_flux(FaceFluxArgs a, const int* __restrict__ bf,
                                                       int n_bface) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b < n_bface) face_flux<NQ, true>(a, bf[b], b);
}

struct CellUpdateArgs {
  const int4* __restrict__ cfaces;     // [n_pad]: faces of local edges 0..2, L bits
  const double* __restrict__ vol;      // [n_pad]
  const double* __restrict__ phi;      // [n_face][4]
  const double* Un;                    // [n][4]
  const double* Uk;                    // [n][4]
  double* out;                         // R or U^(k+1)
  const double* dt;                    // device scalar
  double ca, cb, cc;                   // out = ca Un + cb Uk + cc (dt R)
  int n_cell;
};

template <bool RK>
__device__ __forceinline__ void cell_update(const CellUpdateArgs& a, int t, double* kept = nullptr) {
  const int4 cf = a.cfaces[t];
  const double2* ph = reinterpret_cast<const double2*>(a.phi);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const size_t f = (size_t)(e == 0 ? cf.x : (e == 1 ? cf.y : cf.z));
    const bool isL = (cf.w >> e) & 1;
    const double2 x = ph[2 * f], y = ph[2 * f + 1];
    const double p[4] = {x.x, x.y, y.x, y.y};
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = isL ? acc[c] + p[c] : acc[c] - p[c];
  }
  const double ia = -1.0 / a.vol[t];
  double R[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) R[c] = acc[c] * ia;
  double* o = a.out + (size_t)t * 4;
  if (RK) {
    const double dt = *a.dt;
    const double* un = a.Un + (size_t)t * 4;
    const double* uk = a.Uk + (size_t)t * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double x = a.ca * un[c] + a.cb * uk[c] + a.cc * (dt * R[c]);
      o[c] = x;
      if (kept) kept[c] = x;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) o[c] = R[c];
  }
}

template <bool RK>
__global__ __launch_bounds__(256) void k_cell_update(CellUpdateArgs a) {
  const int t = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (t < a.n_cell) cell_update<RK>(a, t);
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

// |V_i| / sum_j |A_ij| (|u_i . n_ij| + c_i) from the cell average u of cell t.
__device__ __forceinline__ double dt_limit_of(const double* u, const double* __restrict__ geo,
                                              int t, double g) {
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
  return gg[9] / den;
}

__device__ __forceinline__ double cell_dt_limit(const double* __restrict__ U,
                                                const double* __restrict__ geo, int t, double g) {
  return dt_limit_of(U + (size_t)t * 4, geo, t, g);
}

// The last stage's gather and update, fused with the first half of the
// constant-CFL step of the state it writes: each block's minimum of
// |V_i| / sum_j |A_ij| (|u_i . n_ij| + c_i) over its new cell averages, from
// the values in registers and with k_dt_partial's arithmetic, so that
// k_dt_final over these minima gives teno_max_dt of the new state bit for
// bit.  (The minima are reduced by a second launch, not by the last block
// to finish: on this multi-die GPU the device-scope fence that would order
// each block's minimum before its count writes back the block's whole L2.)
__global__ __launch_bounds__(256) void k_cell_update_dt(CellUpdateArgs a,
                                                        const double* __restrict__ geo, double g,
                                                        double* __restrict__ partial) {
  __shared__ double sh[4];
  const int t = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  double lim = INFINITY;
  if (t < a.n_cell) {
    double u[4];
    cell_update<true>(a, t, u);
    lim = dt_limit_of(u, geo, t, g);
  }
  const double m = block_min(lim, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_dt_partial(const double* __restrict__ U,
                                                    const double* __restrict__ geo, int n,
                                                    double g, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int t = blockIdx.x * 256 + threadIdx.x;
  const double lim = t < n ? cell_dt_limit(U, geo, t, g) : INFINITY;
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
// Phase 1 (one lane per face): adjoint of the face-point states.  Face f
// gets Phi_bar = lam_R/|V_R| - lam_L/|V_L| (scaled by `scale`); at each of
// its Gauss points the lane runs the reverse mode of the HLL flux (hll_vjp)
// and writes both sides' face-point adjoints.
struct AdjFaceArgs {
  const double* __restrict__ fp;      // [3 nq][n_pad][4]
  const int4* __restrict__ fcell;     // [n_face]: L, R, eL | eR << 2
  const double2* __restrict__ fgeo;   // [n_face][2]: (nx, ny), (|A|, 0)
  const double* __restrict__ vol;     // [n_pad]
  const double* __restrict__ lam;
  const double* scale_dev;            // device scalar multiplying lam (nullable = 1)
  double scale;
  double* __restrict__ fpbar;         // [3 nq][n_pad][4]
  const int* __restrict__ bkind;      // [n_bface] boundary conditions (meshes with open axes)
  const double* __restrict__ bstate;  // [n_bface][4] prescribed states
  double gamma;
  int n_face, n_pad;
};

template <int NQ>
__device__ __forceinline__ void adj_face(const AdjFaceArgs& a, int f) {
  const int4 fc = a.fcell[f];
  const double2 nrm = a.fgeo[2 * (size_t)f], len = a.fgeo[2 * (size_t)f + 1];
  const int L = fc.x, R = fc.y, eL = fc.z & 3, eR = (fc.z >> 2) & 3;
  const double sc = a.scale * (a.scale_dev ? *a.scale_dev : 1.0);
  const double aL = a.vol[L], aR = a.vol[R];
  double pb[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
    pb[c] = sc * (a.lam[(size_t)R * 4 + c] / aR - a.lam[(size_t)L * 4 + c] / aL);
  const double2* fp2 = reinterpret_cast<const double2*>(a.fp);
  double2* out2 = reinterpret_cast<double2*>(a.fpbar);
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int qL = eL * NQ + k, qR = eR * NQ + NQ - 1 - k;
    const size_t oL = ((size_t)qL * a.n_pad + L) * 2, oR = ((size_t)qR * a.n_pad + R) * 2;
    const double2 l0 = fp2[oL], l1 = fp2[oL + 1], r0 = fp2[oR], r1 = fp2[oR + 1];
    const double vl[4] = {l0.x, l0.y, l1.x, l1.y}, vr[4] = {r0.x, r0.y, r1.x, r1.y};
    double gL[4] = {0.0, 0.0, 0.0, 0.0}, gR[4] = {0.0, 0.0, 0.0, 0.0};
    hll_vjp(vl, vr, nrm.x, nrm.y, a.gamma, pb, gL, gR);
    const double w = len.x * FaceRule<NQ>::w[k];
    out2[oL] = make_double2(w * gL[0], w * gL[1]);
    out2[oL + 1] = make_double2(w * gL[2], w * gL[3]);
    out2[oR] = make_double2(w * gR[0], w * gR[1]);
    out2[oR + 1] = make_double2(w * gR[2], w * gR[3]);
  }
}

template <int NQ>
__global__ __launch_bounds__(256) void k_adj_faces(AdjFaceArgs a) {
  const int f = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (f >= a.n_face) return;
  adj_face<NQ>(a, f);
}

// Boundary faces only (after k_adj_faces, same stream; bf[b] is the face of
// boundary face b).  Only the inner cell's term enters the face's adjoint,
// and the outer state follows the inner one through the face's condition,
// so the inner side also takes the outer side's adjoint through that map,
// transposed: the identity (transmissive), the mirror I - 2 n n^T of the
// momentum (reflective, symmetric), nothing (prescribed).  Rewrites every
// face point of the edge, which k_adj_faces filled as if the cell were on
// both sides.
template <int NQ>
__global__ __launch_bounds__(256) void k_adj_boundary(AdjFaceArgs a, const int* __restrict__ bf,
                                                      int n_bface) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n_bface) return;
  const int f = bf[b];
  const int4 fc = a.fcell[f];
  const double2 nrm = a.fgeo[2 * (size_t)f], len = a.fgeo[2 * (size_t)f + 1];
  const int L = fc.x, eL = fc.z & 3, kind = a.bkind[b];
  const double sc = a.scale * (a.scale_dev ? *a.scale_dev : 1.0);
  const double aL = a.vol[L];
  double pb[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) pb[c] = -sc * (a.lam[(size_t)L * 4 + c] / aL);
  const double2* fp2 = reinterpret_cast<const double2*>(a.fp);
  double2* out2 = reinterpret_cast<double2*>(a.fpbar);
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const size_t oL = ((size_t)(eL * NQ + k) * a.n_pad + L) * 2;
    const double2 l0 = fp2[oL], l1 = fp2[oL + 1];
    const double uL[4] = {l0.x, l0.y, l1.x, l1.y};
    double uR[4];
    boundary_state(kind, a.bstate, b, uL, nrm.x, nrm.y, uR);
    double gL[4] = {0.0, 0.0, 0.0, 0.0}, gR[4] = {0.0, 0.0, 0.0, 0.0};
    hll_vjp(uL, uR, nrm.x, nrm.y, a.gamma, pb, gL, gR);
    if (kind == TENO_BC_TRANSMISSIVE) {
#pragma unroll
      for (int c = 0; c < 4; ++c) gL[c] += gR[c];
    } else if (kind == TENO_BC_REFLECTIVE) {
      const double gn = gR[1] * nrm.x + gR[2] * nrm.y;
      gL[0] += gR[0];
      gL[1] += gR[1] - 2.0 * gn * nrm.x;
      gL[2] += gR[2] - 2.0 * gn * nrm.y;
      gL[3] += gR[3];
    }
    const double w = len.x * FaceRule<NQ>::w[k];
    out2[oL] = make_double2(w * gL[0], w * gL[1]);
    out2[oL + 1] = make_double2(w * gL[2], w * gL[3]);
  }
}

// Phase 2 (one wavefront per tile, four lanes per cell): transpose of the
// reconstruction.  The adjoint of each stencil difference d_s = U_s - U_0
// goes to the tile's member slot of U_s, summed in LDS (one accumulator per
// distinct member and variable) in a fixed order.  Blocks stored rows by
// lane are read as the forward kernel reads them: lane g of a cell takes row
// 4j + g of group j for all four variables (the coefficient adjoints of the
// cell are shared across its four lanes first); blocks of entry pairs are
// read by lane v for variable v, row by row.  Within one LDS instruction the
// lanes that name the same member add in rounds that set-up assigns (in lane
// order for a group of rows, in cell order for one row), so no instruction
// has two lanes on one address and every sum is formed in the same order on
// every run.  The tile's sums are written once to tbar; the cell's own part
// (the -U_0 of its differences and its face points) goes to own[n][4].
struct AdjReconArgs {
  const double* __restrict__ fpbar;
  const uint16_t* __restrict__ flags;
  const double2* __restrict__ M;
  const int4* __restrict__ aslot;   // [n_tiles][rows4][16][4] uint16: slot | round << 9
  const int* __restrict__ tround;   // [n_tiles] rounds of the tile (largest round + 1)
  double* __restrict__ tbar;      // [n_tiles][ustride][4]
  double* __restrict__ own;       // [n_pad][4]
  int ustride;
  int n_cell, n_tiles, n_pad;
};

__device__ __forceinline__ unsigned quad_bcast_u(unsigned x, int k) {
  switch (k) {
    case 0: return (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x00, 0xF, 0xF, false);
    case 1: return (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x55, 0xF, 0xF, false);
    case 2: return (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0xAA, 0xF, 0xF, false);
    default: return (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0xFF, 0xF, 0xF, false);
  }
}

// wavefronts per block of the adjoint reconstruction (one tile each); one,
// as for the forward kernels, measured 4% faster on the backward pass
#ifndef TENO_ADJ_BLOCK_WAVES
#define TENO_ADJ_BLOCK_WAVES 1
#endif
constexpr int kAdjBlockWaves = TENO_ADJ_BLOCK_WAVES;

template <int P, int NQ>
__global__ __launch_bounds__(64 * kAdjBlockWaves) void k_adj_recon(AdjReconArgs a) {
  using O = OrderT<P>;
  constexpr int NU = O::NU;
  constexpr int NP = 3 * NQ;
  constexpr bool SL = lane_rows(kSmallCoef, true), LL = large_lane_rows(NU, true);
  static_assert(kTile == 16, "four lanes per cell");
  extern __shared__ double lds_acc[];  // kAdjBlockWaves wavefronts x ustride x 4
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile =
      __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * kAdjBlockWaves + wave);
  if (tile >= a.n_tiles) return;  // whole wavefront leaves together
  double* acc = lds_acc + (size_t)wave * a.ustride * 4;
  for (int i = lane; i < 4 * a.ustride; i += 64) acc[i] = 0.0;
  wave_lds_sync();
  const int c = lane / kLanesPerCell, v = lane % kLanesPerCell, g = v;
  const int cell = tile * kTile + c;
  const bool live = cell < a.n_cell;
  const int cl = live ? cell : tile * kTile;
  const unsigned nib = live ? ((a.flags[cl] >> (4 * v)) & 0xFu) : 0u;
  double gsum = 0.0;
  double ab[NU];
#pragma unroll
  for (int l = 0; l < NU; ++l) ab[l] = 0.0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const double gq = live ? a.fpbar[((size_t)q * a.n_pad + cl) * 4 + v] : 0.0;
    gsum += gq;
#pragma unroll
    for (int l = 0; l < NU; ++l) ab[l] = fma(FaceBasis<O::R, NQ>::P.v[q][l], gq, ab[l]);
  }
  // the tile's operator stream (dense: the adjoint runs on meshes in
  // conservative variables)
  const double* __restrict__ mt =
      reinterpret_cast<const double*>(a.M) + (size_t)tile * O::template JPD<true> * kTile;
  const uint16_t* __restrict__ sl =
      reinterpret_cast<const uint16_t*>(a.aslot + (size_t)tile * slot_int4(O::ROWS4));
  const int rounds = a.tround[tile];  // >= 1, the same for the whole wavefront
  auto slot_of = [&](int r) { return (int)sl[(r >> 2) * (kTile * 4) + c * 4 + (r & 3)]; };
  // adds d into accumulator column q of the row's member, in the row's round
  // (the first round unconditionally, so the slot word is loaded with the
  // row's operator entries rather than after them)
  auto add_in_round = [&](int w, int q, double d, bool on) {
    double* dst = &acc[(w & 511) * 4 + q];
    const int mine = w >> 9;
    int r = 0;
    do {
      if (on && mine == r) atomicAdd(dst, d);
    } while (++r < rounds);
  };
  const bool keepK = nib & 8u;
  const int cnt = (int)(nib & 1u) + (int)((nib >> 1) & 1u) + (int)((nib >> 2) & 1u);
  // the flags of the cell's four variables, on all four lanes
  unsigned nq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) nq[q] = quad_bcast_u(nib, q);
  // weight of stencil k (3 = large) for variable q: a small stencil counts
  // 1/cnt where step two kept it, the large one 1 where step one kept it
  auto weight = [&](int k, int q) {
    const unsigned f = nq[q];
    if (!live) return 0.0;
    if (k == 3) return (f & 8u) ? 1.0 : 0.0;
    const int cq = (int)(f & 1u) + (int)((f >> 1) & 1u) + (int)((f >> 2) & 1u);
    return (!(f & 8u) && ((f >> k) & 1u) && cq > 0) ? 1.0 / (double)cq : 0.0;
  };
  double dsum = 0.0;                    // rows read by variable (lane v)
  double dq[4] = {0.0, 0.0, 0.0, 0.0};  // rows read by lane: this lane's rows, per variable

  // rows by lane: a block of NR rows of L entries at block k of the stream,
  // with coefficient adjoints ab4 of all four variables and weights w
  auto lane_block = [&](auto kc, auto nrc, auto lc, const auto& ab4) {
    constexpr int K = decltype(kc)::value, NR = decltype(nrc)::value, L = decltype(lc)::value;
    constexpr int R0 = K == 3 ? 33 : kSmallRows * K;
    const double w[4] = {weight(K, 0), weight(K, 1), weight(K, 2), weight(K, 3)};
    const bool need = (w[0] != 0.0) | (w[1] != 0.0) | (w[2] != 0.0) | (w[3] != 0.0);
    if (!__any(need)) return;
    const double* __restrict__ mb = mt + (size_t)block_start(K, true) * kTile;
    static_for<0, (NR + 3) / 4>([&](auto jc) {
      constexpr int J = jc, rg = group_rows(NR, J);
      const int gg = g < rg ? g : rg - 1;
      const bool on = g < rg;
      const int s = 4 * J + gg;
      double m[L];
#pragma unroll
      for (int l = 0; l < L; ++l) m[l] = mb[4 * kTile * L * J + (l * kTile + c) * rg + gg];
      const int w0 = slot_of(R0 + s);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) t = fma(m[l], ab4[l][q], t);
        const double d = (on && w[q] != 0.0) ? t * w[q] : 0.0;
        dq[q] += d;
        add_in_round(w0, q, d, on && w[q] != 0.0);
      }
    });
  };

  // ---- small stencils ----
  if constexpr (SL) {
    double ab4[kSmallCoef][4];
#pragma unroll
    for (int l = 0; l < kSmallCoef; ++l) {
      ab4[l][0] = quad_bcast<0>(ab[l]);
      ab4[l][1] = quad_bcast<1>(ab[l]);
      ab4[l][2] = quad_bcast<2>(ab[l]);
      ab4[l][3] = quad_bcast<3>(ab[l]);
    }
    using I = std::integral_constant<int, kSmallRows>;
    using C = std::integral_constant<int, kSmallCoef>;
    lane_block(std::integral_constant<int, 0>{}, I{}, C{}, ab4);
    lane_block(std::integral_constant<int, 1>{}, I{}, C{}, ab4);
    lane_block(std::integral_constant<int, 2>{}, I{}, C{}, ab4);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const bool kept = live && !keepK && (nib & (1u << k)) && cnt > 0;
      if (kept) {
        const double wk = 1.0 / (double)cnt;
#pragma unroll
        for (int s = 0; s < kSmallRows; ++s) {
          double d = 0.0;
#pragma unroll
          for (int l = 0; l < kSmallCoef; ++l)
            d = fma(mt[(size_t)block_start(k, true) * kTile + block_offset(kSmallRows, kSmallCoef, true, c, s, l)],
                    ab[l], d);
          d *= wk;
          dsum += d;
          add_in_round(slot_of(small_row(k, s)), v, d, true);
        }
      }
    }
  }
  // ---- large stencil ----
  if constexpr (LL) {
    double ab4[NU][4];
#pragma unroll
    for (int l = 0; l < NU; ++l) {
      ab4[l][0] = quad_bcast<0>(ab[l]);
      ab4[l][1] = quad_bcast<1>(ab[l]);
      ab4[l][2] = quad_bcast<2>(ab[l]);
      ab4[l][3] = quad_bcast<3>(ab[l]);
    }
    lane_block(std::integral_constant<int, 3>{}, std::integral_constant<int, O::NL>{},
               std::integral_constant<int, NU>{}, ab4);
  } else if (live && keepK) {
#pragma unroll 1
    for (int s = 0; s < O::NL; ++s) {
      double d = 0.0;
#pragma unroll
      for (int l = 0; l < NU; ++l)
        d = fma(mt[(size_t)block_start(3, true) * kTile + large_block_offset(O::NL, NU, true, c, s, l)],
                ab[l], d);
      dsum += d;
      add_in_round(slot_of(large_row(s)), v, d, true);
    }
  }
  // the rows read by lane: variable v's sum over the cell's four lanes
  if constexpr (SL || LL) {
    const bool odd = lane & 1, hi = lane & 2;
    const double k0 = odd ? dq[1] : dq[0], k1 = odd ? dq[3] : dq[2];
    const double s0 = odd ? dq[0] : dq[1], s1 = odd ? dq[2] : dq[3];
    const double p0 = k0 + quad_perm_dpp<0xB1>(s0), p1 = k1 + quad_perm_dpp<0xB1>(s1);
    const double keep = hi ? p1 : p0, send = hi ? p0 : p1;
    dsum = (keep + quad_perm_dpp<0x4E>(send)) + dsum;
  }
  if (live) a.own[(size_t)cell * 4 + v] = gsum - dsum;
  wave_lds_sync();
  double* __restrict__ tb = a.tbar + (size_t)tile * a.ustride * 4;
  for (int i = lane; i < 4 * a.ustride; i += 64) tb[i] = acc[i];
}

// Phase 3 (four lanes per cell, lane q = variable q): U_bar[j] = own[j] +
// the tile sums of every tile member slot naming j (reverse list rev_ptr[j]
// .. rev_ptr[j+1]-1, by tile), in list order: no atomics.  Then out = U_bar
// + beta * extra (extra nullable).
__global__ __launch_bounds__(256) void k_adj_gather(const double* __restrict__ own,
                                                    const double* __restrict__ tbar,
                                                    const int32_t* __restrict__ rev_ptr,
                                                    const int32_t* __restrict__ rev_ent,
                                                    int n_cell, const double* extra, double beta,
                                                    double* out) {
  const int gid = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const int j = gid >> 2, q = gid & 3;
  if (j >= n_cell) return;
  const int b = rev_ptr[j], e = rev_ptr[j + 1];
  double s = 0.0;
  int t = b;
  for (; t + 3 < e; t += 4) {
    const int e0 = rev_ent[t], e1 = rev_ent[t + 1], e2 = rev_ent[t + 2], e3 = rev_ent[t + 3];
    const double x0 = tbar[(size_t)e0 * 4 + q], x1 = tbar[(size_t)e1 * 4 + q];
    const double x2 = tbar[(size_t)e2 * 4 + q], x3 = tbar[(size_t)e3 * 4 + q];
    s += x0;
    s += x1;
    s += x2;
    s += x3;
  }
  for (; t < e; ++t) s += tbar[(size_t)rev_ent[t] * 4 + q];
  double v = own[(size_t)j * 4 + q] + s;
  if (extra) v = v + beta * extra[(size_t)j * 4 + q];
  out[(size_t)j * 4 + q] = v;
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

// ---------------------------------------------------------------------------
// batches of independent meshes
// ---------------------------------------------------------------------------
// One mesh of a batch: the arguments of its three RK stages.
struct BatchMeshDev {
  ReconArgs r[3];          // reconstruction input of stage k
  FaceFluxArgs ff;         // face fluxes (the same buffers every stage)
  CellUpdateArgs cu[3];    // gather and update of stage k
  const double* U;         // cell averages at the start of the step
  const double* geo;
  double* dt;              // this mesh's step (device scalar)
  const int* bface;        // [n_bface]: face of each boundary face
  double gamma;
  int pq;                  // order * 10 + face points
  int n_cell;
  int n_bface;
};

// Runs reconstruct_tile for pq (any supported pair when PQ == 0, otherwise
// only PQ, so a per-order launch keeps that order's register budget).
template <int PQ>
__device__ __forceinline__ void batch_tile(int pq, const ReconArgs& a, int tile, int lane,
                                           int4* stage) {
  if (PQ != 0) pq = PQ;
  switch (pq) {
    case 32: reconstruct_tile<3, 2>(a, tile, lane, stage); break;
    case 42: reconstruct_tile<4, 2>(a, tile, lane, stage); break;
    case 53: reconstruct_tile<5, 3>(a, tile, lane, stage); break;
    case 63: reconstruct_tile<6, 3>(a, tile, lane, stage); break;
    case 33: if (PQ == 0 || PQ == 33) reconstruct_tile<3, 3>(a, tile, lane, stage); break;
    case 43: if (PQ == 0 || PQ == 43) reconstruct_tile<4, 3>(a, tile, lane, stage); break;
    case 52: if (PQ == 0 || PQ == 52) reconstruct_tile<5, 2>(a, tile, lane, stage); break;
    case 62: if (PQ == 0 || PQ == 62) reconstruct_tile<6, 2>(a, tile, lane, stage); break;
    default: break;
  }
}

// Persistent reconstruction over a work list of (mesh, tile) items: each
// wavefront takes the contiguous, cost-balanced item range
// [wave_start[w], wave_start[w+1]) and leaves when it is done.
template <int PQ>
__global__ __launch_bounds__(256) void k_batch_reconstruct(const BatchMeshDev* __restrict__ meshes,
                                                           const int2* __restrict__ items,
                                                           const int* __restrict__ wave_start,
                                                           int n_waves, int stage_k,
                                                           int lds_stride) {
  extern __shared__ int4 lds[];  // 4 wavefronts x lds_stride (the largest mesh's)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= n_waves) return;
  const int i0 = wave_start[w], i1 = wave_start[w + 1];
  for (int i = i0; i < i1; ++i) {
    const int2 it = items[i];
    const int m = __builtin_amdgcn_readfirstlane(it.x);
    const int tile = __builtin_amdgcn_readfirstlane(it.y);
    const BatchMeshDev& d = meshes[m];
    batch_tile<PQ>(d.pq, d.r[stage_k], tile, lane, lds + wave * lds_stride);
  }
}

// The same with one (mesh, tile) item per wavefront and no loop.  In the
// persistent form the compiler hoists the constant tables' addresses out of
// the item loop and holds them, spilling scalar registers into vector ones
// (141 VGPRs at order 5 against 104 for one mesh); without the loop it keeps
// the single-mesh kernel's budget.
// Blocks of kReconBlockWaves wavefronts, as for one mesh.
template <int PQ>
__global__ __launch_bounds__(64 * kReconBlockWaves)
void k_batch_reconstruct_one(const BatchMeshDev* __restrict__ meshes,
                             const int2* __restrict__ items, int n_items, int stage_k,
                             int lds_stride) {
  extern __shared__ int4 lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = xcd_remap(blockIdx.x, gridDim.x) * kReconBlockWaves + wave;
  if (w >= n_items) return;
  const int2 it = items[w];
  const int m = __builtin_amdgcn_readfirstlane(it.x);
  const int tile = __builtin_amdgcn_readfirstlane(it.y);
  const BatchMeshDev& d = meshes[m];
  batch_tile<PQ>(d.pq, d.r[stage_k], tile, lane, lds + wave * lds_stride);
}

// Persistent face fluxes over (mesh, 64-face chunk) items.
__global__ __launch_bounds__(256) void k_batch_face_flux(const BatchMeshDev* __restrict__ meshes,
                                                         const int2* __restrict__ items,
                                                         const int* __restrict__ wave_start,
                                                         int n_waves) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= n_waves) return;
  const int i0 = wave_start[w], i1 = wave_start[w + 1];
  for (int i = i0; i < i1; ++i) {
    const int2 it = items[i];
    const int m = __builtin_amdgcn_readfirstlane(it.x);
    const BatchMeshDev& d = meshes[m];
    const int f = it.y * 64 + lane;
    if (f >= d.ff.n_face) continue;
    if (d.pq % 10 == 2) face_flux<2>(d.ff, f);
    else face_flux<3>(d.ff, f);
  }
}

// Boundary faces over (mesh, 64-face chunk) items, one item per wavefront,
// after k_batch_face_flux: every face, then the boundary faces rewritten
// with their conditions, as for one mesh.
__global__ __launch_bounds__(256) void k_batch_boundary_flux(const BatchMeshDev* __restrict__ meshes,
                                                             const int2* __restrict__ items,
                                                             int n_items) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (w >= n_items) return;
  const int2 it = items[w];
  const int m = __builtin_amdgcn_readfirstlane(it.x);
  const BatchMeshDev& d = meshes[m];
  const int b = it.y * 64 + lane;
  if (b >= d.n_bface) return;
  if (d.pq % 10 == 2) face_flux<2, true>(d.ff, d.bface[b], b);
  else face_flux<3, true>(d.ff, d.bface[b], b);
}

// Persistent gather + stage update over (mesh, 64-cell chunk) items.
__global__ __launch_bounds__(256) void k_batch_cell_update(const BatchMeshDev* __restrict__ meshes,
                                                           const int2* __restrict__ items,
                                                           const int* __restrict__ wave_start,
                                                           int n_waves, int stage_k) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= n_waves) return;
  const int i0 = wave_start[w], i1 = wave_start[w + 1];
  for (int i = i0; i < i1; ++i) {
    const int2 it = items[i];
    const int m = __builtin_amdgcn_readfirstlane(it.x);
    const BatchMeshDev& d = meshes[m];
    const int t = it.y * 64 + lane;
    if (t >= d.n_cell) continue;
    cell_update<true>(d.cu[stage_k], t);
  }
}

// Per-mesh dt: one block per (mesh, 256-cell block) item, then one block per mesh.
__global__ __launch_bounds__(256) void k_batch_dt_partial(const BatchMeshDev* __restrict__ meshes,
                                                          const int2* __restrict__ items,
                                                          double* __restrict__ partial) {
  __shared__ double sh[4];
  const int2 it = items[blockIdx.x];
  const BatchMeshDev& d = meshes[it.x];
  const int t = it.y * 256 + threadIdx.x;
  const double lim = t < d.n_cell ? cell_dt_limit(d.U, d.geo, t, d.gamma) : INFINITY;
  const double m = block_min(lim, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_batch_dt_final(const BatchMeshDev* __restrict__ meshes,
                                                        const int* __restrict__ item_start,
                                                        const double* __restrict__ partial,
                                                        double cfl) {
  __shared__ double sh[4];
  double x = INFINITY;
  for (int i = item_start[blockIdx.x] + threadIdx.x; i < item_start[blockIdx.x + 1]; i += 256)
    x = fmin(x, partial[i]);
  const double m = block_min(x, sh);
  if (threadIdx.x == 0) *meshes[blockIdx.x].dt = cfl * m;
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
