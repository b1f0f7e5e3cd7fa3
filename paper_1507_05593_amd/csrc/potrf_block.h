// Cholesky of one (<= 64) diagonal block with its explicit inverse, as a device
// function for a 256-thread workgroup: the body of the POTRF launch, and the tail of the
// trailing-update product launch whose tile is the next diagonal block (that workgroup
// factors the block right after storing it).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tasks.h"

namespace rsc {

typedef double v4d __attribute__((ext_vector_type(4)));

// 1 / sqrt(d) for a positive finite d: the hardware estimate r refined once by the
// binomial series of (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - d r^2, through the
// e^2 term (the relative error goes from |e| to about e^3, below FP64 rounding for the
// estimate's |e| ~ 1e-7), four dependent operations.
__device__ __forceinline__ double rsqrt_f64(double d) {
  const double r = __builtin_amdgcn_rsq(d);
  const double e = fma(-(d * r), r, 1.0);
  return fma(r * e, fma(0.375, e, 0.5), r);
}

// Cholesky of one (<= 64) diagonal block together with its explicit inverse.
// mode 0: a pivot that is not positive and finite records the supernode in
//         status[0] (smallest id wins) and is replaced by 1 so the sweep stays finite.
// mode 1 (orthonormalisation): a pivot <= 1e-14 * scale marks the column dependent:
//         its L column becomes the unit vector and its row and column of the inverse
//         become zero;
// mode 2: the same with the threshold 1e-8 * scale.
// Past the block edge (nb < 64) the tile is the identity.
//
// Blocked right-looking elimination over four 16-column block steps, the tile in LDS:
//   1. wave 0 factors the 16 x 16 diagonal block and forms its inverse in registers
//      (each lane holds four rows of one column of the symmetric block and of the
//      inverse; one column at a time, the pivot and the column broadcast across lanes);
//   2. the rows below: P = A_below D^{-T}, one 16-row block per wave (FP64 MFMA);
//   3. the trailing lower blocks: A -= P P^T, blocks dealt round robin to the waves.
// The inverse's off-diagonal blocks then follow block row by block row:
//   W_ij = -D_i^{-1} sum_{m = j}^{i-1} L_im W_mj.
// MFMA v_mfma_f64_16x16x4f64: A operand (row lane % 16, k lane / 16), B operand
// (column lane % 16, k lane / 16), result element e at (row lane / 16 + 4e, column lane % 16).
// Lane C of each 16-lane row, broadcast to the row (DPP row_newbcast, two 32-bit moves).
template <int C>
__device__ __forceinline__ double bcast16(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + C, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + C, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Lane l's value of x (l uniform), through two 32-bit readlanes.
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Column C of the 16 x 16 diagonal block.  Lane (j, g) = (lane % 16, lane / 16) holds rows
// 4s + g (s < 4) of column j of the symmetric block (v[s]) and of the inverse (wv[s]).
// The pivot comes from lane (C, C % 4) by readlane; A(j, C) = A(C, j) and W(C, j) from
// lane (j, C % 4) by a shuffle; A(4s + g, C) from lane C of the lane's own 16-lane row by
// DPP row broadcast, so each lane updates its four rows.
template <int C>
__device__ __forceinline__ void diag_step(double (&v)[4], double (&wv)[4], int j, int g, int kk, int nb,
                                          int mode, double dscale, bool& bad) {
  constexpr int gC = C & 3, sC = C >> 2;
  double d = readlane_f64(v[sC], 16 * gC + C);
  const double ajc = __shfl(v[sC], 16 * gC + j, 64);
  const double wcr = __shfl(wv[sC], 16 * gC + j, 64);
  bool dk = false;
  if (kk + C >= nb) {
    d = 1.0;                                       // past the block edge: identity
  } else if (mode == 0) {
    if (!(d > 0.0) || !isfinite(d)) { bad = true; d = 1.0; }
  } else if (!(d > dscale) || !isfinite(d)) {
    dk = true;
    d = 1.0;
  }
  const double rp = rsqrt_f64(d);
  const double piv = d * rp;
  const double sc = dk ? 0.0 : rp;
  const double ljc = (j > C) ? ajc * sc : 0.0;
  const double wcj = wcr * sc;                     // row C of the inverse, scaled
  if (g == gC) wv[sC] = wcj;
  const double al = (j == C) ? sc : 1.0;
  const double ga = sc * ljc, de = sc * wcj;
  if (j == C && g == gC) v[sC] = piv;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (4 * s + 3 <= C) continue;                  // every row of the slot is done
    const double x = bcast16<C>(v[s]);             // A(4s + g, C)
    const bool below = 4 * s + g > C;
    const double nv = fma(-x, ga, v[s] * al), nw = fma(-x, de, wv[s]);
    v[s] = below ? nv : v[s];
    wv[s] = below ? nw : wv[s];
  }
  if constexpr (C < 15) diag_step<C + 1>(v, wv, j, g, kk, nb, mode, dscale, bad);
}

constexpr int kPitch = 65;   // LDS row pitch of a 64-edge block (NB + 1 in general)

template <int PITCH>
__device__ __forceinline__ v4d mma16(v4d acc, const double* X, int xr, int xc, const double* Y, int yr,
                                     int yc, bool ytrans, int lane) {
  // acc += X(xr.., xc..) Y^T over 16 k: Y element (col j, k) read at Y(yr + j, yc + k), or at
  // Y(yr + k, yc + j) when ytrans
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 16; ks += 4) {
    const double a = X[(xr + li) * PITCH + xc + ks + lk];
    const double b = ytrans ? Y[(yr + ks + lk) * PITCH + yc + li] : Y[(yr + li) * PITCH + yc + ks + lk];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// One diagonal block (nb <= NB, NB = 32 or 64) for a 256-thread workgroup; A and W are its
// LDS blocks (NB x (NB + 1) doubles each; A(r, c) at r * (NB + 1) + c, the inverse W in
// the same layout).  The inverse is stored as a 64 x 64 block whatever NB.
template <int NB>
__device__ inline void potrf_block(const PotrfTask& T, double* __restrict__ arena, int32_t* __restrict__ status,
                                   double* __restrict__ A, double* __restrict__ W) {
  constexpr int PI = NB + 1, NL = NB * NB / 256;      // pitch, loads per thread
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nb = T.nb;
  const int nbk = (nb + 15) >> 4, nbb16 = 16 * nbk;   // 16-column blocks that hold the block
  double* P = arena + T.panel;
  const int64_t base = T.d0 + (int64_t)T.d0 * T.ld;
  {
    // all loads in flight together (addresses clamped into the block), then LDS
    double t[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int idx = tid + 256 * u, r = idx % NB, c = idx / NB;
      t[u] = P[base + min(r, nb - 1) + (int64_t)min(c, nb - 1) * T.ld];
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int idx = tid + 256 * u, r = idx % NB, c = idx / NB;
      A[r * PI + c] = (r < nb && c < nb && r >= c) ? t[u] : ((r == c) ? 1.0 : 0.0);
      W[r * PI + c] = (r == c && r >= nbb16) ? 1.0 : 0.0;   // blocks past nb: identity
    }
  }
  const double dscale = (T.mode >= 1) ? arena[T.scale_off] * (T.mode == 2 ? 1e-8 : 1e-14) : 0.0;
  __syncthreads();
  bool bad = false;
  for (int kb = 0; kb < nbk; ++kb) {
    const int kk = 16 * kb;
    if (w == 0) {
      // lane (j, g) holds rows 4s + g of column j of the symmetric block (read from the
      // lower triangle) and of the inverse (see diag_step)
      const int j = li, g = lk;
      double v[4], wv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + g;
        v[q] = A[(kk + (i > j ? i : j)) * PI + kk + (i > j ? j : i)];
        wv[q] = (i == j) ? 1.0 : 0.0;
      }
      diag_step<0>(v, wv, j, g, kk, nb, T.mode, dscale, bad);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + g;
        if (i >= j) A[(kk + i) * PI + kk + j] = v[q];
        W[(kk + i) * PI + kk + j] = wv[q];
      }
    }
    __syncthreads();
    if (kb == nbk - 1) break;
    // rows below: P = A_below D^{-T} (block row rb by wave rb - kb - 1)
    {
      const int rb = kb + 1 + w;
      if (rb < nbk) {
        v4d acc = {0, 0, 0, 0};
        acc = mma16<PI>(acc, A, 16 * rb, kk, W, kk, kk, false, lane);
#pragma unroll
        for (int e = 0; e < 4; ++e) A[(16 * rb + lk + 4 * e) * PI + kk + li] = acc[e];
      }
    }
    __syncthreads();
    // trailing lower blocks (ib, jb), kb < jb <= ib < nbk
    {
      int t = 0;
      for (int ib = kb + 1; ib < nbk; ++ib)
        for (int jb = kb + 1; jb <= ib; ++jb, ++t) {
          if ((t & 3) != w) continue;
          v4d acc = {0, 0, 0, 0};
          acc = mma16<PI>(acc, A, 16 * ib, kk, A, 16 * jb, kk, false, lane);
#pragma unroll
          for (int e = 0; e < 4; ++e) A[(16 * ib + lk + 4 * e) * PI + 16 * jb + li] -= acc[e];
        }
    }
    __syncthreads();
  }
  // off-diagonal blocks of the inverse, block row by block row (block jb by wave jb)
  for (int ib = 1; ib < nbk; ++ib) {
    if (w < ib) {
      const int jb = w;
      v4d t = {0, 0, 0, 0};
      for (int mb = jb; mb < ib; ++mb) t = mma16<PI>(t, A, 16 * ib, 16 * mb, W, 16 * mb, 16 * jb, true, lane);
      // W_ij = -D_i^{-1} T: the B operand (column li, k = 4e + lk) is t[e] of this lane
      v4d acc = {0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double a = W[(16 * ib + li) * PI + 16 * ib + 4 * e + lk];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, t[e], acc, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) W[(16 * ib + lk + 4 * e) * PI + 16 * jb + li] = -acc[e];
    }
    __syncthreads();
  }
  if (bad && tid == 0) atomicMin(&status[0], T.sn);
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    if (r < nb && c <= r) P[base + r + (int64_t)c * T.ld] = A[r * PI + c];
  }
  double* inv = arena + T.inv;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    inv[r + 64 * c] = W[r * PI + c];
  }
  if (T.mrow > 0) {
    // a one-block panel: its identity rows become M = W^T at once (no solve launch)
    double* M = P + T.mrow;
    for (int idx = tid; idx < NB * NB; idx += 256) {
      const int r = idx % NB, c = idx / NB;
      if (r < nb && c < nb) M[r + (int64_t)c * T.ld] = W[c * PI + r];
    }
  }
}

// LDS bytes of potrf_block<64>'s two blocks
constexpr size_t kPotrfSmem = 2 * 64 * kPitch * sizeof(double);

}  // namespace rsc
