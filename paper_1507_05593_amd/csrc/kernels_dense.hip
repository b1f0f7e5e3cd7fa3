// gfx950 kernels of the numeric factorization: assembly, Schur-complement updates,
// diagonal-block Cholesky, tile GEMMs, Gaussian sampling, Jacobi eigensolver.
//
// Matrix-core layouts (CDNA4, 64-lane waves):
//   v_mfma_f64_16x16x4f64: A(i,k) from lane i + 16k, B(k,j) from lane j + 16k,
//                          D(i,j) in lane j + 16 (i mod 4), element i / 4.
//   v_mfma_f32_16x16x4f32 / v_mfma_f32_16x16x32_bf16: same operand pattern (the bf16
//                          form packs k = 8 (lane/16) + e, e < 8), D(i,j) in lane
//                          j + 16 (i / 4), element i mod 4.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"
#include "tasks.h"

namespace rsc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// ---------------------------------------------------------------- elementwise

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// arena[slot[p]] = values[p] for every stored entry with a target slot (>= 0).
__global__ void k_assemble(const double* __restrict__ values, const int64_t* __restrict__ slot,
                           int64_t nnz, double* __restrict__ arena) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    int64_t s = slot[p];
    if (s >= 0) arena[s] = values[p];
  }
}

__global__ void k_scatter_const(const int64_t* __restrict__ slot, int64_t n, double v,
                                double* __restrict__ arena) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    arena[slot[p]] = v;
}

// ---------------------------------------------------------------- FP64 MFMA tile GEMM

// One 64x64 output tile per 256-thread workgroup; wave w owns the 32x32 quarter
// (w / 2, w % 2) as 2x2 blocks of 16x16, accumulated by v_mfma_f64_16x16x4f64 with
// operands read straight from the arena (L2-resident tiles).
__global__ __launch_bounds__(256) void k_gemm_f64(const GemmTask* __restrict__ tasks,
                                                  double* __restrict__ arena,
                                                  const int32_t* __restrict__ ilim) {
  const GemmTask T = tasks[blockIdx.x];
  const int lane = lane_id(), w = wave_id();
  const int wr = w >> 1, wc = w & 1;
  const int n = T.nlim >= 0 ? min(T.n, ilim[T.nlim]) : T.n;
  const int K = T.klim >= 0 ? min(T.k, ilim[T.klim]) : T.k;
  if (T.j0 >= n) return;
  const int li = lane & 15, lk = lane >> 4;
  int rows[2], cols[2];
  bool rv[2], cv[2];
  for (int b = 0; b < 2; ++b) {
    rows[b] = T.i0 + wr * 32 + b * 16 + li;
    cols[b] = T.j0 + wc * 32 + b * 16 + li;
    rv[b] = rows[b] < T.m;
    cv[b] = cols[b] < n;
  }
  const double* A = arena + T.a;
  const double* B = arena + T.b;
  v4d acc[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) acc[x][y] = (v4d){0.0, 0.0, 0.0, 0.0};
  const bool active = (T.i0 + wr * 32 < T.m) && (T.j0 + wc * 32 < n);
  if (active) {
    int64_t ar[2], bc[2];
    for (int b = 0; b < 2; ++b) {
      ar[b] = (int64_t)rows[b] * T.ais;
      bc[b] = (int64_t)cols[b] * T.bjs;
    }
    int k0 = 0;
    for (; k0 + 16 <= K; k0 += 16) {
      double av[4][2], bv[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t kk = k0 + 4 * u + lk;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          av[u][b] = rv[b] ? A[ar[b] + kk * T.aks] : 0.0;
          bv[u][b] = cv[b] ? B[bc[b] + kk * T.bks] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][x], bv[u][y], acc[x][y], 0, 0, 0);
    }
    for (; k0 < K; k0 += 4) {
      const int64_t kk = k0 + lk;
      const bool kv = kk < K;
      double av[2], bv[2];
      for (int b = 0; b < 2; ++b) {
        av[b] = (rv[b] && kv) ? A[ar[b] + kk * T.aks] : 0.0;
        bv[b] = (cv[b] && kv) ? B[bc[b] + kk * T.bks] : 0.0;
      }
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
  }
  // every read of A/B (which may alias C in the in-place triangular solve) is done
  __syncthreads();
  if (!active) return;
  double* C = arena + T.c;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      for (int e = 0; e < 4; ++e) {
        const int i = T.i0 + wr * 32 + x * 16 + lk + 4 * e;
        const int j = T.j0 + wc * 32 + y * 16 + li;
        if (i < T.m && j < n) {
          double* cp = C + i + (int64_t)j * T.ldc;
          const double v = T.alpha * acc[x][y][e];
          *cp = (T.beta == 0.0) ? v : v + T.beta * *cp;
        }
      }
}

// ---------------------------------------------------------------- Schur update

// Target-tile ownership: the workgroup holds one 64x64 tile of a supernode panel in
// LDS, subtracts every descendant's product X(a:b) X(c:d)^T (scattered through the
// relative map) in entry order, and writes the tile back once.  No atomics: the
// result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_update_f64(const UpdTile* __restrict__ tiles,
                                                    const UpdEntry* __restrict__ ents,
                                                    const int32_t* __restrict__ relmap,
                                                    double* __restrict__ arena,
                                                    const int32_t* __restrict__ ilim) {
  __shared__ double tile[64][65];
  __shared__ int32_t rmap[64], cmap[64];
  const UpdTile T = tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wr = w >> 1, wc = w & 1, li = lane & 15, lk = lane >> 4;
  double* P = arena + T.panel;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    tile[r][c] = (r < T.nrows && c < T.ncols) ? P[(T.row0 + r) + (int64_t)(T.col0 + c) * T.ld] : 0.0;
  }
  for (int e = T.e0; e < T.e1; ++e) {
    const UpdEntry E = ents[e];
    const int nr = E.b - E.a, nc = E.d - E.c;
    const int K = E.kdim >= 0 ? E.kdim : ilim[-1 - E.kdim];
    if (tid < 64) {
      rmap[tid] = tid < nr ? relmap[E.map + E.a + tid] - T.row0 : 0;
    } else if (tid < 128) {
      const int t = tid - 64;
      cmap[t] = t < nc ? relmap[E.map + E.c + t] - T.col0 : 0;
    }
    __syncthreads();
    const bool active = (wr * 32 < nr) && (wc * 32 < nc) && K > 0;
    if (active) {
      const double* X = arena + E.x;
      v4d acc[2][2];
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = (v4d){0.0, 0.0, 0.0, 0.0};
      int ra[2], rc[2];
      bool va[2], vc[2];
      for (int b = 0; b < 2; ++b) {
        ra[b] = wr * 32 + b * 16 + li;
        rc[b] = wc * 32 + b * 16 + li;
        va[b] = ra[b] < nr;
        vc[b] = rc[b] < nc;
        ra[b] += E.a;
        rc[b] += E.c;
      }
      int k0 = 0;
      for (; k0 + 16 <= K; k0 += 16) {
        double av[4][2], bv[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t col = (int64_t)(k0 + 4 * u + lk) * E.ldx;
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            av[u][b] = va[b] ? X[ra[b] + col] : 0.0;
            bv[u][b] = vc[b] ? X[rc[b] + col] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][x], bv[u][y], acc[x][y], 0, 0, 0);
      }
      for (; k0 < K; k0 += 4) {
        const int kk = k0 + lk;
        const bool kv = kk < K;
        const int64_t col = (int64_t)kk * E.ldx;
        double av[2], bv[2];
        for (int b = 0; b < 2; ++b) {
          av[b] = (va[b] && kv) ? X[ra[b] + col] : 0.0;
          bv[b] = (vc[b] && kv) ? X[rc[b] + col] : 0.0;
        }
        for (int x = 0; x < 2; ++x)
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
      }
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
          for (int e2 = 0; e2 < 4; ++e2) {
            const int pr = wr * 32 + x * 16 + lk + 4 * e2;
            const int pc = wc * 32 + y * 16 + li;
            if (pr < nr && pc < nc) tile[rmap[pr]][cmap[pc]] -= acc[x][y][e2];
          }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    if (r < T.nrows && c < T.ncols) P[(T.row0 + r) + (int64_t)(T.col0 + c) * T.ld] = tile[r][c];
  }
}

// ---------------------------------------------------------------- diagonal block Cholesky

// Cholesky of one (<= 64) diagonal block in LDS, then its explicit inverse.
// mode 0: a pivot that is not positive and finite records the supernode in
//         status[0] (smallest id wins) and is replaced by 1 so the sweep stays finite.
// mode 1 (orthonormalisation): a pivot <= 1e-14 * scale marks the column dependent:
//         its L column and its row of the inverse become zero.
__global__ __launch_bounds__(256) void k_potrf_f64(const PotrfTask* __restrict__ tasks,
                                                   double* __restrict__ arena,
                                                   int32_t* __restrict__ status) {
  __shared__ double L[64][65];
  __shared__ double W[64][65];
  __shared__ int32_t drop[64];
  const PotrfTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int nb = T.nb;
  double* P = arena + T.panel;
  const int64_t base = T.d0 + (int64_t)T.d0 * T.ld;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    L[r][c] = (r < nb && c < nb && r >= c) ? P[base + r + (int64_t)c * T.ld] : 0.0;
  }
  if (tid < 64) drop[tid] = 0;
  __shared__ double dscale;
  if (tid == 0) dscale = (T.mode == 1) ? arena[T.scale_off] : 0.0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid == 0) {
      double d = L[k][k];
      if (T.mode == 0) {
        if (!(d > 0.0) || !isfinite(d)) {
          atomicMin(&status[0], T.sn);
          d = 1.0;
        }
        L[k][k] = sqrt(d);
      } else {
        if (!(d > 1e-14 * dscale) || !isfinite(d)) {
          drop[k] = 1;
          L[k][k] = 1.0;
        } else {
          L[k][k] = sqrt(d);
        }
      }
    }
    __syncthreads();
    const double piv = L[k][k];
    const bool dk = drop[k] != 0;
    for (int i = k + 1 + tid; i < nb; i += 256) L[i][k] = dk ? 0.0 : L[i][k] / piv;
    __syncthreads();
    const int m = nb - k - 1;
    for (int idx = tid; idx < m * m; idx += 256) {
      const int i = k + 1 + idx % m, j = k + 1 + idx / m;
      if (i >= j) L[i][j] -= L[i][k] * L[j][k];
    }
    __syncthreads();
  }
  // write L back (lower triangle incl. diagonal; dropped columns hold 0 below a unit diagonal)
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int r = idx % nb, c = idx / nb;
    if (r >= c) P[base + r + (int64_t)c * T.ld] = L[r][c];
  }
  // explicit inverse, one column per thread (forward substitution)
  if (tid < 64) {
    const int t = tid;
    for (int i = 0; i < 64; ++i) W[i][t] = 0.0;
    if (t < nb && !drop[t]) {
      W[t][t] = 1.0 / L[t][t];
      for (int i = t + 1; i < nb; ++i) {
        if (drop[i]) continue;
        double s = 0.0;
        for (int q = t; q < i; ++q) s += L[i][q] * W[q][t];
        W[i][t] = -s / L[i][i];
      }
    }
  }
  __syncthreads();
  double* inv = arena + T.inv;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    inv[r + 64 * c] = W[r][c];
  }
}

// ---------------------------------------------------------------- Gaussian sample

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

// Entry (row, col) of supernode j's sample from counter (row, col / 4, 0, 0);
// Box-Muller pairs (w0, w1) -> columns 4t, 4t+1 and (w2, w3) -> 4t+2, 4t+3.
__global__ void k_philox(const PhiloxTask* __restrict__ tasks, double* __restrict__ arena,
                         int round_bf16) {
  const PhiloxTask T = tasks[blockIdx.y];
  const int ngrp = (T.cols + 3) / 4;
  const int64_t total = (int64_t)T.rows * ngrp;
  const double two32 = 2.3283064365386963e-10;   // 2^-32
  const double twopi = 2.0 * 3.141592653589793;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(id / ngrp), g = (int)(id % ngrp);
    uint32_t c[4] = {(uint32_t)row, (uint32_t)g, 0u, 0u};
    philox4x32_10(c, T.k0, T.k1);
    double out[4];
    for (int h = 0; h < 2; ++h) {
      const double u1 = ((double)c[2 * h] + 1.0) * two32;
      const double u2 = (double)c[2 * h + 1] * two32;
      const double rad = sqrt(-2.0 * log(u1));
      const double th = twopi * u2;
      out[2 * h] = rad * cos(th);
      out[2 * h + 1] = rad * sin(th);
    }
    for (int e = 0; e < 4; ++e) {
      const int col = 4 * g + e;
      if (col < T.cols) {
        double v = out[e];
        if (round_bf16) v = (double)(float)(__bf16)(float)v;
        arena[T.out + row + (int64_t)col * T.rows] = v;
      }
    }
  }
}

// ---------------------------------------------------------------- Gram preparation

// Column-drop scale of an orthonormalisation panel: the largest diagonal entry of
// its n x n Gram block (at arena[g], leading dimension ld), stored at arena[out].
__global__ void k_gram_scale(const int64_t* __restrict__ g, const int32_t* __restrict__ ld,
                             const int32_t* __restrict__ n, const int64_t* __restrict__ out,
                             double* __restrict__ arena) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  double m = 0.0;
  for (int i = threadIdx.x; i < n[p]; i += 256) {
    const double d = arena[g[p] + i + (int64_t)i * ld[p]];
    m = fmax(m, isfinite(d) ? d : 0.0);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) arena[out[p]] = red[0];
}

// ---------------------------------------------------------------- Jacobi eigensolver

// Cyclic Jacobi with the round-robin parallel ordering on a 64x64 symmetric matrix in
// LDS (Golub and Van Loan, symmetric Schur decomposition); accumulates the rotations
// into Q (initialised by the caller).  Runs sweeps until no rotation is applied.
__device__ void jacobi64(double (*A)[65], double (*Q)[65], double scale) {
  __shared__ double cs[32], sn[32];
  __shared__ int pp[32], qq[32];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const double tiny = 1e-300 + 1e-15 * scale;
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < 63; ++rnd) {
      if (tid < 32) {
        // circle method: position 0 fixed, positions 1..63 rotate
        auto at = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + rnd) % 63); };
        int p = at(tid), q = at(63 - tid);
        if (p > q) { int t = p; p = q; q = t; }
        const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-16 * sqrt(fabs(app) * fabs(aqq)) && fabs(apq) > tiny) {
          const double th = (aqq - app) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          rotated = 1;
        }
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int idx = tid; idx < 32 * 64; idx += 256) {
        const int r = idx & 31, j = idx >> 5;
        const double c = cs[r], s = sn[r];
        if (s == 0.0) continue;
        const int p = pp[r], q = qq[r];
        const double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - s * aq;
        A[q][j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, Q <- Q J
      for (int idx = tid; idx < 32 * 64; idx += 256) {
        const int r = idx & 31, i = idx >> 5;
        const double c = cs[r], s = sn[r];
        if (s == 0.0) continue;
        const int p = pp[r], q = qq[r];
        const double ap = A[i][p], aq = A[i][q];
        A[i][p] = c * ap - s * aq;
        A[i][q] = s * ap + c * aq;
        const double qp = Q[i][p], qv = Q[i][q];
        Q[i][p] = c * qp - s * qv;
        Q[i][q] = s * qp + c * qv;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
}

__device__ __forceinline__ void pair_blocks(int rnd, int pair, int nbk, int& I, int& J) {
  auto at = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + rnd) % (nbk - 1)); };
  I = at(pair);
  J = at(nbk - 1 - pair);
  if (I > J) { int t = I; I = J; J = t; }
}

// Small problems (npad == 64): the whole matrix in LDS, solved to convergence.
__global__ __launch_bounds__(256) void k_jacobi_small(const EigTask* __restrict__ tasks,
                                                      double* __restrict__ arena) {
  __shared__ double A[64][65];
  __shared__ double Q[64][65];
  const EigTask T = tasks[blockIdx.x];
  if (T.npad != 64) return;
  const int tid = threadIdx.x;
  double* G = arena + T.g;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    A[r][c] = G[r + 64 * c];
    Q[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi64(A, Q, arena[T.scale]);
  double* Z = arena + T.z;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    Z[r + 64 * c] = Q[r][c];
    G[r + 64 * c] = A[r][c];
  }
}

// Block Jacobi round, phase 1: for each block pair (I, J) of this round solve the
// 64x64 subproblem [[G_II, G_IJ], [G_JI, G_JJ]] and store its rotation (64x64).
// A pair whose coupling block is already negligible stores nothing and is skipped.
__global__ __launch_bounds__(256) void k_jacobi_pairs(const EigTask* __restrict__ tasks,
                                                      double* __restrict__ arena,
                                                      int32_t* __restrict__ ints, int rnd) {
  __shared__ double A[64][65];
  __shared__ double Q[64][65];
  __shared__ int big;
  const EigTask T = tasks[blockIdx.y];
  const int pair = blockIdx.x;
  if (T.npad <= 64 || pair >= T.nbk / 2) return;
  int I, J;
  pair_blocks(rnd % (T.nbk - 1), pair, T.nbk, I, J);
  const int tid = threadIdx.x;
  const double* G = arena + T.g;
  const int ld = T.npad;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    const int gr = (r < 32 ? I * 32 + r : J * 32 + r - 32);
    const int gc = (c < 32 ? I * 32 + c : J * 32 + c - 32);
    A[r][c] = G[gr + (int64_t)gc * ld];
    Q[r][c] = (r == c) ? 1.0 : 0.0;
  }
  if (tid == 0) big = 0;
  __syncthreads();
  const double floor_abs = 1e-300 + 1e-15 * arena[T.scale];
  for (int idx = tid; idx < 32 * 32; idx += 256) {
    const int r = idx & 31, c = 32 + (idx >> 5);
    const double a = A[r][c];
    if (fabs(a) > 1e-16 * sqrt(fabs(A[r][r]) * fabs(A[c][c])) && fabs(a) > floor_abs) big = 1;
  }
  __syncthreads();
  int32_t* flag = ints + T.flagslot + pair;
  if (!big) {
    if (tid == 0) *flag = 0;
    return;
  }
  if (tid == 0) *flag = 1;
  jacobi64(A, Q, arena[T.scale]);
  double* R = arena + T.rot + (int64_t)pair * 64 * 64;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    R[r + 64 * c] = Q[r][c];
  }
}

// Block Jacobi round, phase 2: G <- P^T G P for the block-diagonal rotation P of the
// round, one (pair a, pair b) 64x64 block per workgroup; blockIdx.x = a * (nbk/2) + b.
__global__ __launch_bounds__(256) void k_jacobi_apply_g(const EigTask* __restrict__ tasks,
                                                        double* __restrict__ arena,
                                                        const int32_t* __restrict__ ints, int rnd) {
  __shared__ double X[64][65];
  __shared__ double Y[64][65];
  const EigTask T = tasks[blockIdx.y];
  if (T.npad <= 64) return;
  const int np = T.nbk / 2;
  const int pa = blockIdx.x / np, pb = blockIdx.x % np;
  if (pa >= np) return;
  const int fa = ints[T.flagslot + pa], fb = ints[T.flagslot + pb];
  if (!fa && !fb) return;
  int Ia, Ja, Ib, Jb;
  pair_blocks(rnd % (T.nbk - 1), pa, T.nbk, Ia, Ja);
  pair_blocks(rnd % (T.nbk - 1), pb, T.nbk, Ib, Jb);
  const int tid = threadIdx.x;
  double* G = arena + T.g;
  const int ld = T.npad;
  const double* Ra = arena + T.rot + (int64_t)pa * 4096;
  const double* Rb = arena + T.rot + (int64_t)pb * 4096;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    const int gr = (r < 32 ? Ia * 32 + r : Ja * 32 + r - 32);
    const int gc = (c < 32 ? Ib * 32 + c : Jb * 32 + c - 32);
    X[r][c] = G[gr + (int64_t)gc * ld];
  }
  __syncthreads();
  // Y = Ra^T X (if pair a rotated), else Y = X
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    double s;
    if (fa) {
      s = 0.0;
      for (int t = 0; t < 64; ++t) s += Ra[t + 64 * r] * X[t][c];
    } else {
      s = X[r][c];
    }
    Y[r][c] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    double s;
    if (fb) {
      s = 0.0;
      for (int t = 0; t < 64; ++t) s += Y[r][t] * Rb[t + 64 * c];
    } else {
      s = Y[r][c];
    }
    const int gr = (r < 32 ? Ia * 32 + r : Ja * 32 + r - 32);
    const int gc = (c < 32 ? Ib * 32 + c : Jb * 32 + c - 32);
    G[gr + (int64_t)gc * ld] = s;
  }
}

// Block Jacobi round, phase 3: Z <- Z P on the columns of each rotated pair;
// blockIdx.x = pair * (npad / 64) + row block.
__global__ __launch_bounds__(256) void k_jacobi_apply_z(const EigTask* __restrict__ tasks,
                                                        double* __restrict__ arena,
                                                        const int32_t* __restrict__ ints, int rnd) {
  __shared__ double X[64][65];
  const EigTask T = tasks[blockIdx.y];
  if (T.npad <= 64) return;
  const int nrb = T.npad / 64;
  const int pair = blockIdx.x / nrb, rb = blockIdx.x % nrb;
  if (pair >= T.nbk / 2) return;
  if (!ints[T.flagslot + pair]) return;
  int I, J;
  pair_blocks(rnd % (T.nbk - 1), pair, T.nbk, I, J);
  const int tid = threadIdx.x;
  double* Z = arena + T.z;
  const int ld = T.npad;
  const double* R = arena + T.rot + (int64_t)pair * 4096;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    const int gc = (c < 32 ? I * 32 + c : J * 32 + c - 32);
    X[r][c] = Z[rb * 64 + r + (int64_t)gc * ld];
  }
  __syncthreads();
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    double s = 0.0;
    for (int t = 0; t < 64; ++t) s += X[r][t] * R[t + 64 * c];
    const int gc = (c < 32 ? I * 32 + c : J * 32 + c - 32);
    Z[rb * 64 + r + (int64_t)gc * ld] = s;
  }
}

// Z = I (npad x npad) before the rounds of a block Jacobi solve.
__global__ void k_eig_init(const EigTask* __restrict__ tasks, double* __restrict__ arena) {
  const EigTask T = tasks[blockIdx.y];
  const int64_t nn = (int64_t)T.npad * T.npad;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nn;
       i += (int64_t)gridDim.x * blockDim.x)
    arena[T.z + i] = (i % T.npad == i / T.npad) ? 1.0 : 0.0;
}

// Eigenvalues are the diagonal of the converged G.  Sort descending (rank by
// counting, ties by index), keep q = #{sqrt(lambda_i) > tol * sqrt(lambda_max)}, and
// write the kept eigenvectors, in order, as the first q columns of zq (n x n; the
// rest zero).
__global__ __launch_bounds__(256) void k_eig_select(const EigTask* __restrict__ tasks,
                                                    double* __restrict__ arena,
                                                    int32_t* __restrict__ ints) {
  const EigTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const double* G = arena + T.g;
  const double* Z = arena + T.z;
  double* zq = arena + T.zq;
  double* lam = arena + T.lam;
  const int n = T.n, ld = T.npad;
  __shared__ double lmax;
  __shared__ int q;
  if (tid == 0) {
    double m = 0.0;
    bool bad = false;
    for (int i = 0; i < n; ++i) {
      const double d = G[i + (int64_t)i * ld];
      if (!isfinite(d)) bad = true;
      m = fmax(m, d);
    }
    lmax = bad ? 0.0 : m;
    q = 0;
  }
  __syncthreads();
  const double smax = sqrt(fmax(lmax, 0.0));
  for (int i = tid; i < n; i += 256) {
    const double li = G[i + (int64_t)i * ld];
    int rank = 0;
    for (int t = 0; t < n; ++t) {
      const double lt = G[t + (int64_t)t * ld];
      rank += (lt > li) || (lt == li && t < i);
    }
    lam[rank] = li;
    const bool keep = smax > 0.0 && sqrt(fmax(li, 0.0)) > T.tol * smax;
    if (keep) atomicAdd(&q, 1);
    for (int r = 0; r < n; ++r) zq[r + (int64_t)rank * n] = keep ? Z[r + (int64_t)i * ld] : 0.0;
  }
  __syncthreads();
  if (tid == 0) ints[T.qslot] = q;
}

// ---------------------------------------------------------------- launchers

static inline int grid_for(int64_t n, int block = 256, int cap = 8192) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}
void launch_assemble(const double* values, const int64_t* slot, int64_t nnz, double* arena,
                     hipStream_t s) {
  if (nnz > 0) hipLaunchKernelGGL(k_assemble, dim3(grid_for(nnz)), dim3(256), 0, s, values, slot, nnz, arena);
}
void launch_scatter_const(const int64_t* slot, int64_t n, double v, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_const, dim3(grid_for(n)), dim3(256), 0, s, slot, n, v, arena);
}
void launch_gemm_f64(const GemmTask* t, int n, double* arena, const int32_t* ilim, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gemm_f64, dim3(n), dim3(256), 0, s, t, arena, ilim);
}
void launch_update_f64(const UpdTile* t, int n, const UpdEntry* e, const int32_t* relmap,
                       double* arena, const int32_t* ilim, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_update_f64, dim3(n), dim3(256), 0, s, t, e, relmap, arena, ilim);
}
void launch_potrf_f64(const PotrfTask* t, int n, double* arena, int32_t* status, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_potrf_f64, dim3(n), dim3(256), 0, s, t, arena, status);
}
void launch_philox(const PhiloxTask* t, int n, int64_t max_work, double* arena, int bf16,
                   hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_philox, dim3(grid_for(max_work, 256, 4096), n), dim3(256), 0, s, t, arena, bf16);
}
void launch_gram_scale(const int64_t* g, const int32_t* ld, const int32_t* nn, const int64_t* out,
                       int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gram_scale, dim3(n), dim3(256), 0, s, g, ld, nn, out, arena);
}
void launch_jacobi_small(const EigTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_jacobi_small, dim3(n), dim3(256), 0, s, t, arena);
}
void launch_jacobi_round(const EigTask* t, int n, int max_pairs, int max_rowblocks, double* arena,
                         int32_t* ints, int rnd, hipStream_t s) {
  if (n <= 0 || max_pairs <= 0) return;
  hipLaunchKernelGGL(k_jacobi_pairs, dim3(max_pairs, n), dim3(256), 0, s, t, arena, ints, rnd);
  hipLaunchKernelGGL(k_jacobi_apply_g, dim3(max_pairs * max_pairs, n), dim3(256), 0, s, t, arena,
                     (const int32_t*)ints, rnd);
  hipLaunchKernelGGL(k_jacobi_apply_z, dim3(max_pairs * max_rowblocks, n), dim3(256), 0, s, t,
                     arena, (const int32_t*)ints, rnd);
}
void launch_eig_init(const EigTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_eig_init, dim3(64, n), dim3(256), 0, s, t, arena);
}
void launch_eig_select(const EigTask* t, int n, double* arena, int32_t* ints, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_eig_select, dim3(n), dim3(256), 0, s, t, arena, ints);
}

}  // namespace rsc
