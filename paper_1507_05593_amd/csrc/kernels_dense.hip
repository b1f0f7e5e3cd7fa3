// gfx950 kernels of the numeric factorization: assembly, fills, identity scatter,
// diagonal-block Cholesky, Gaussian sampling, Gram scale and the spectral-truncation
// helpers (Newton-Schulz projector iteration in LDS, projector trace, basis compaction).
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
#include <type_traits>

#include "kernels.h"
#include "potrf_block.h"
#include "tasks.h"

namespace rsc {

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

// arena[slot[t]] = values[idx[t]]: the entries of one level's off-diagonal blocks.
__global__ void k_assemble_pairs(const double* __restrict__ values, const int64_t* __restrict__ idx,
                                 const int64_t* __restrict__ slot, int64_t n, double* __restrict__ arena) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    arena[slot[t]] = values[idx[t]];
}

__global__ void k_scatter_const(const int64_t* __restrict__ slot, int64_t n, double v,
                                double* __restrict__ arena) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    arena[slot[p]] = v;
}

// ---------------------------------------------------------------- diagonal block Cholesky

// NB = 32 for launches whose blocks all have at most 32 columns (a quarter of the LDS,
// so several times as many workgroups per compute unit), else 64.
template <int NB>
__global__ __launch_bounds__(256) void k_potrf_f64(const PotrfTask* __restrict__ tasks,
                                                   double* __restrict__ arena,
                                                   int32_t* __restrict__ status) {
  __shared__ double A[NB * (NB + 1)];
  __shared__ double W[NB * (NB + 1)];
  potrf_block<NB>(tasks[blockIdx.x], arena, status, A, W);
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
// Box-Muller pairs (w0, w1) -> columns 4t, 4t+1 and (w2, w3) -> 4t+2, 4t+3.  F32: the
// transform in FP32 (the mixed forms, whose products round the sample to BF16 or FP32
// anyway), else in FP64.
template <bool F32>
__global__ void k_philox(const PhiloxTask* __restrict__ tasks, double* __restrict__ arena) {
  const PhiloxTask T = tasks[blockIdx.y];
  const int ngrp = (T.cols + 3) / 4;
  const int64_t total = (int64_t)T.rows * ngrp;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * blockDim.x) {
    // consecutive threads on consecutive rows: each of the four column stores is
    // coalesced (the values depend only on the counter (row, g), not on the thread)
    const int row = (int)(id % T.rows), g = (int)(id / T.rows);
    uint32_t c[4] = {(uint32_t)row, (uint32_t)g, T.c2, 0u};
    philox4x32_10(c, T.k0, T.k1);
    double out[4];
    for (int h = 0; h < 2; ++h) {
      if constexpr (F32) {
        const float two32 = 2.3283064365386963e-10f;   // 2^-32
        const float u1 = ((float)c[2 * h] + 1.0f) * two32;
        const float u2 = (float)c[2 * h + 1] * two32;
        const float rad = sqrtf(-2.0f * logf(u1));
        float sn, cs;
        sincosf(6.283185307179586f * u2, &sn, &cs);
        out[2 * h] = (double)(rad * cs);
        out[2 * h + 1] = (double)(rad * sn);
      } else {
        const double two32 = 2.3283064365386963e-10;  // 2^-32
        const double u1 = ((double)c[2 * h] + 1.0) * two32;
        const double u2 = (double)c[2 * h + 1] * two32;
        const double rad = sqrt(-2.0 * log(u1));
        const double th = 2.0 * 3.141592653589793 * u2;
        out[2 * h] = rad * cos(th);
        out[2 * h + 1] = rad * sin(th);
      }
    }
    for (int e = 0; e < 4; ++e) {
      const int col = 4 * g + e;
      if (col < T.cols) arena[T.out + row + (int64_t)col * T.rows] = out[e];
    }
  }
}

// ---------------------------------------------------------------- Gram preparation

// Column-drop scale of an orthonormalisation panel: the largest diagonal entry of
// its n x n Gram block (at arena[g], leading dimension ld), stored at arena[out].
// m[p] > 0 (the rows of the sampled block Y whose Gram matrix this is): shifted
// Cholesky-QR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020) -- the shift
// s = 11 (m n + n (n + 1)) u ||Y||_F^2, u = 2^-53, ||Y||_F^2 = trace(G), is added to the
// diagonal first, so that G + s I is positive definite despite the rounding of G and
// the pass keeps every direction of Y (the scale then includes the shift).
__global__ void k_gram_scale(const int64_t* __restrict__ g, const int32_t* __restrict__ ld,
                             const int32_t* __restrict__ n, const int32_t* __restrict__ m,
                             const int64_t* __restrict__ out, double* __restrict__ arena) {
  __shared__ double red[256], tr[256];
  const int p = blockIdx.x;
  double mx = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < n[p]; i += 256) {
    const double d = arena[g[p] + i + (int64_t)i * ld[p]];
    mx = fmax(mx, isfinite(d) ? d : 0.0);
    t += isfinite(d) ? d : 0.0;
  }
  red[threadIdx.x] = mx;
  tr[threadIdx.x] = t;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
      tr[threadIdx.x] += tr[threadIdx.x + s];
    }
    __syncthreads();
  }
  double shift = 0.0;
  if (m[p] > 0) {
    const double nn = (double)n[p];
    shift = 11.0 * ((double)m[p] * nn + nn * (nn + 1.0)) * 1.1102230246251565e-16 * tr[0];
    for (int i = threadIdx.x; i < n[p]; i += 256) arena[g[p] + i + (int64_t)i * ld[p]] += shift;
  }
  if (threadIdx.x == 0) arena[out[p]] = red[0] + shift;
}

// ---------------------------------------------------------------- spectral truncation

// Truncation of V (r x l) at sigma_i > tol sigma_1 through the spectral projector of
// its Gram matrix G = V^T V onto the eigenvalues lambda > theta = tol^2 lambda_max:
// X0 = (G - theta I)(G + theta I)^{-1} maps lambda to (lambda - theta)/(lambda + theta)
// in (-1, 1); Newton-Schulz iterations X <- X (3 I - X^2) / 2 drive it to sign(G - theta I);
// P = (I + X) / 2.  Per-problem scalars (arena sc[0..7]): trace, lambda_max, theta,
// scale (largest diagonal of G + theta I).

__device__ double block_sum256(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_sum1024(double v) {
  __shared__ double red[1024];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// trace(G) and S = G / trace(G) (zero when the trace is not positive).
__global__ __launch_bounds__(256) void k_trunc_prep(const TruncTask* __restrict__ tasks,
                                                    double* __restrict__ arena) {
  // grid (blocks, tasks): every block forms tr G the same way, then scales its share
  const TruncTask T = tasks[blockIdx.y];
  const int l = T.l;
  const double* G = arena + T.g;
  double t = 0.0;
  for (int i = threadIdx.x; i < l; i += 256) t += G[i + (int64_t)i * l];
  t = block_sum256(t);
  if (blockIdx.x == 0 && threadIdx.x == 0) arena[T.sc] = t;
  const double inv = (t > 0.0 && isfinite(t)) ? 1.0 / t : 0.0;
  double* S = arena + T.sa;
  const int64_t ll = (int64_t)l * l;
#pragma unroll 4
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < ll; e += (int64_t)gridDim.x * 256) S[e] = G[e] * inv;
}

// lambda_max by power iteration with S32 = (G / tr G)^32 (already in sb), Rayleigh
// quotient with G; theta = tol^2 lambda_max (the panel [G + theta I; I] is filled by
// k_trunc_mfill).
__global__ __launch_bounds__(1024) void k_trunc_power(const TruncTask* __restrict__ tasks,
                                                     double* __restrict__ arena) {
  __shared__ double v[2048], w[2048];   // l <= 2048 (checked by the planner)
  const TruncTask T = tasks[blockIdx.x];
  const int l = T.l;
  const double* S = arena + T.sb;
  const double* G = arena + T.g;
  for (int i = threadIdx.x; i < l; i += 1024) {
    // fixed, non-structured start vector
    uint32_t h = (uint32_t)i * 2654435761u + 0x9E3779B9u;
    h ^= h >> 15; h *= 2246822519u; h ^= h >> 13;
    v[i] = 0.5 + (double)(h & 0xFFFF) / 65536.0;
  }
  __syncthreads();
  for (int it = 0; it < 4; ++it) {
    for (int i = threadIdx.x; i < l; i += 1024) {
      double a = 0.0;
#pragma unroll 8
      for (int k = 0; k < l; ++k) a += S[i + (int64_t)k * l] * v[k];
      w[i] = a;
    }
    __syncthreads();
    double nn = 0.0;
    for (int i = threadIdx.x; i < l; i += 1024) nn += w[i] * w[i];
    nn = block_sum1024(nn);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int i = threadIdx.x; i < l; i += 1024) v[i] = w[i] * inv;
    __syncthreads();
  }
  double num = 0.0, den = 0.0;
  for (int i = threadIdx.x; i < l; i += 1024) {
    double a = 0.0;
#pragma unroll 8
    for (int k = 0; k < l; ++k) a += G[i + (int64_t)k * l] * v[k];
    num += v[i] * a;
    den += v[i] * v[i];
  }
  num = block_sum1024(num);
  den = block_sum1024(den);
  double lam = (den > 0.0) ? num / den : 0.0;
  if (!isfinite(lam) || lam < 0.0) lam = 0.0;
  const double theta = T.tol * T.tol * lam;
  if (threadIdx.x == 0) { arena[T.sc + 1] = lam; arena[T.sc + 2] = theta; }
}

// The same power iteration for large l, one launch per matrix-vector product over a grid
// (64-row blocks, tasks): step it < 4 forms w_it = S32 v with v = w_{it-1} / |w_{it-1}| (the
// start vector of k_trunc_power for it = 0); step 4 forms the Rayleigh quotient's partial
// sums v^T (G v) and v^T v of each row block with v = w_3 / |w_3|.  The vectors alternate
// between the first two l-blocks of the work block at wout (free until the projector
// iteration), the partial sums go to sc[64 + 2 rb] and sc[65 + 2 rb]; every workgroup
// forms the norm of the previous vector in the same order, so they all scale alike.
__global__ __launch_bounds__(256) void k_trunc_pmv(const TruncTask* __restrict__ tasks,
                                                   double* __restrict__ arena, int it) {
  __shared__ double v[2048];            // l <= 2048 (checked by the planner)
  __shared__ double red[4][64];
  const TruncTask T = tasks[blockIdx.y];
  const int l = T.l, r0 = 64 * blockIdx.x;
  if (r0 >= l) return;
  if (it == 0) {
    for (int i = threadIdx.x; i < l; i += 256) {
      uint32_t h = (uint32_t)i * 2654435761u + 0x9E3779B9u;
      h ^= h >> 15; h *= 2246822519u; h ^= h >> 13;
      v[i] = 0.5 + (double)(h & 0xFFFF) / 65536.0;
    }
  } else {
    const double* wp = arena + T.wout + (int64_t)((it - 1) & 1) * l;
    double nn = 0.0;
    for (int i = threadIdx.x; i < l; i += 256) nn += wp[i] * wp[i];
    nn = block_sum256(nn);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int i = threadIdx.x; i < l; i += 256) v[i] = wp[i] * inv;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = r0 + lane;
  const double* Mx = arena + (it < 4 ? T.sb : T.g);
  double acc = 0.0;
  if (i < l) {
    const int per = (l + 3) / 4, k0 = w * per, k1 = min(l, k0 + per);
#pragma unroll 8
    for (int k = k0; k < k1; ++k) acc += Mx[i + (int64_t)k * l] * v[k];
  }
  red[w][lane] = acc;
  __syncthreads();
  if (w != 0) return;
  const double y = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  if (it < 4) {
    if (i < l) arena[T.wout + (int64_t)(it & 1) * l + i] = y;
    return;
  }
  double num = i < l ? v[i] * y : 0.0, den = i < l ? v[i] * v[i] : 0.0;
  for (int o = 32; o > 0; o >>= 1) {
    num += __shfl_xor(num, o, 64);
    den += __shfl_xor(den, o, 64);
  }
  if (lane == 0) {
    arena[T.sc + 64 + 2 * blockIdx.x] = num;
    arena[T.sc + 65 + 2 * blockIdx.x] = den;
  }
}

// lambda_max and theta from k_trunc_pmv's partial sums (row blocks in order).
__global__ void k_trunc_pfin(const TruncTask* __restrict__ tasks, int n, double* __restrict__ arena) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const TruncTask T = tasks[t];
  double num = 0.0, den = 0.0;
  for (int rb = 0; rb < (T.l + 63) / 64; ++rb) {
    num += arena[T.sc + 64 + 2 * rb];
    den += arena[T.sc + 65 + 2 * rb];
  }
  double lam = (den > 0.0) ? num / den : 0.0;
  if (!isfinite(lam) || lam < 0.0) lam = 0.0;
  arena[T.sc + 1] = lam;
  arena[T.sc + 2] = T.tol * T.tol * lam;
}

// The Cholesky panel [G + theta I; I] (ld 2l) of the truncation and its drop scale (the
// largest diagonal entry); grid (blocks, tasks).
__global__ __launch_bounds__(256) void k_trunc_mfill(const TruncTask* __restrict__ tasks,
                                                     double* __restrict__ arena) {
  const TruncTask T = tasks[blockIdx.y];
  const int l = T.l;
  const double theta = arena[T.sc + 2];
  const double* G = arena + T.g;
  double* M = arena + T.mpan;
  const int64_t ld = 2 * (int64_t)l, ll = (int64_t)l * l;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < ll; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % l), j = (int)(e / l);
    M[i + j * ld] = G[e] + (i == j ? theta : 0.0);
    M[l + i + j * ld] = (i == j) ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0) {
    double mx = 0.0;
    for (int i = threadIdx.x; i < l; i += 256) mx = fmax(mx, G[i + (int64_t)i * l] + theta);
    __shared__ double red[256];
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
      if (threadIdx.x < s2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s2]);
      __syncthreads();
    }
    if (threadIdx.x == 0) arena[T.sc + 3] = red[0];
  }
}

// X0 = I - 2 theta H with H = (G + theta I)^{-1} (in sb), into sa.
__global__ __launch_bounds__(256) void k_trunc_x0(const TruncTask* __restrict__ tasks,
                                                  double* __restrict__ arena) {
  const TruncTask T = tasks[blockIdx.y];
  const int l = T.l;
  const double theta = arena[T.sc + 2];
  const double* H = arena + T.sb;
  double* X = arena + T.sa;
  const int64_t ll = (int64_t)l * l;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < ll; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % l), j = (int)(e / l);
    X[e] = (i == j ? 1.0 : 0.0) - 2.0 * theta * H[e];
  }
}

// P = (I + X) / 2 in place (a grid of workgroups per supernode).
__global__ __launch_bounds__(256) void k_trunc_p(const TruncTask* __restrict__ tasks,
                                                 double* __restrict__ arena) {
  const TruncTask T = tasks[blockIdx.y];
  const int l = T.l;
  double* X = arena + T.sa;
  const int64_t ll = (int64_t)l * l;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < ll; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % l), j = (int)(e / l);
    X[e] = 0.5 * ((i == j ? 1.0 : 0.0) + X[e]);
  }
}

// Newton-Schulz iteration of the spectral projector, X <- 1.5 X - 0.5 X (X X), all
// `steps` steps in one workgroup (NW waves) per supernode with LMIN < l <= LMAX: X and
// Y = X X live in LDS (element type T, order L = l rounded up to 16, pitch L + 4 so that
// the sixteen lanes of a fragment fall in distinct banks), each product over the blocks
// on and below the diagonal (MFMA 16x16x4, blocks dealt to the waves in turn; a wave
// steps all its blocks together through k, so their MFMA chains interleave) and
// mirrored, so both iterates stay exactly symmetric -- which lets both operands be read
// column-wise: A(i, k) = X(k, i).  Other supernodes are left to the other launches.
// Reads X0 from sa and leaves the last iterate there (FP64).
template <typename T, int LMIN, int LMAX, int NW>
__global__ __launch_bounds__(64 * NW) void k_trunc_ns(const TruncTask* __restrict__ tasks,
                                                      double* __restrict__ arena, NsSchedule ns) {
  constexpr int NB = LMAX / 16, NBLK = NB * (NB + 1) / 2, MAXB = (NBLK + NW - 1) / NW, PITCH = LMAX + 4;
  typedef typename std::conditional<sizeof(T) == 8, v4d, v4f>::type AccT;
  __shared__ T X[LMAX * PITCH], Y[LMAX * PITCH];
  const TruncTask Tk = tasks[blockIdx.x];
  const int l = Tk.l;
  if (l <= LMIN || l > LMAX) return;
  const int L = (l + 15) & ~15, nb = L >> 4, nblk = nb * (nb + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* S = arena + Tk.sa;
  for (int e = tid; e < L * L; e += 64 * NW) {
    const int i = e % L, j = e / L;
    X[i + j * PITCH] = (i < l && j < l) ? (T)S[i + (int64_t)j * l] : (T)0;
  }
  // this wave's blocks: q = w + NW u in row-major order of the lower block triangle
  int bi[MAXB], bj[MAXB];
  int nmine = 0;
#pragma unroll
  for (int u = 0; u < MAXB; ++u) {
    const int q = w + NW * u;
    int r = 0;
    while ((r + 1) * (r + 2) / 2 <= q) ++r;
    bi[u] = r; bj[u] = q - r * (r + 1) / 2;
    if (q < nblk) nmine = u + 1;
  }
  AccT acc[MAXB];
  // acc[u] = (P Q)(block u) for symmetric P, Q: lane (li, lk) supplies P(16 bi + li, k)
  // = P[k + (16 bi + li) PITCH] and Q(k, 16 bj + li) = Q[k + (16 bj + li) PITCH]
  auto product = [&](const T* P, const T* Q) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < MAXB; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[u][e] = 0;
    for (int k0 = 0; k0 < L; k0 += 4) {
      T a[MAXB], b[MAXB];
#pragma unroll
      for (int u = 0; u < MAXB; ++u) {
        if (u >= nmine) break;
        a[u] = P[k0 + lk + (16 * bi[u] + li) * PITCH];
        b[u] = Q[k0 + lk + (16 * bj[u] + li) * PITCH];
      }
#pragma unroll
      for (int u = 0; u < MAXB; ++u) {
        if (u >= nmine) break;
        if constexpr (sizeof(T) == 8)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc[u], 0, 0, 0);
        else
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc[u], 0, 0, 0);
      }
    }
  };
  // result element e of block u: row 16 bi + ri, column 16 bj + rj
  auto pos = [&](int u, int e, int& i, int& j) __attribute__((always_inline)) {
    if constexpr (sizeof(T) == 8) i = 16 * bi[u] + lk + 4 * e;
    else i = 16 * bi[u] + 4 * lk + e;
    j = 16 * bj[u] + li;
  };
  __syncthreads();
  for (int it = 0; it < ns.steps; ++it) {
    const double a = ns.alpha[it];
    const T ca = (T)(1.5 * a), cc = (T)(-0.5 * a * a * a);
    product(X, X);                                   // Y = X X
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
      if (u >= nmine) break;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int i, j;
        pos(u, e, i, j);
        if (i >= j) Y[i + j * PITCH] = acc[u][e];
        if (i > j) Y[j + i * PITCH] = acc[u][e];
      }
    }
    __syncthreads();
    product(X, Y);                                   // Z = X (X X), kept in registers
    __syncthreads();                                 // every read of X is done
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
      if (u >= nmine) break;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int i, j;
        pos(u, e, i, j);
        const T v = ca * X[i + j * PITCH] + cc * acc[u][e];
        if (i >= j) X[i + j * PITCH] = v;
        if (i > j) X[j + i * PITCH] = v;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < l * l; e += 64 * NW) {
    const int i = e % l, j = e / l;
    S[e] = (double)X[i + j * PITCH];
  }
}

void launch_trunc_ns(const TruncTask* t, int n, bool fp32, double* arena, const NsSchedule& ns, hipStream_t s) {
  if (n <= 0) return;
  if (fp32) {
    hipLaunchKernelGGL((k_trunc_ns<float, 0, 64, 4>), dim3(n), dim3(256), 0, s, t, arena, ns);
    hipLaunchKernelGGL((k_trunc_ns<float, 64, kNsMaxF32, 8>), dim3(n), dim3(512), 0, s, t, arena, ns);
  } else {
    hipLaunchKernelGGL((k_trunc_ns<double, 0, kNsMaxF64, 4>), dim3(n), dim3(256), 0, s, t, arena, ns);
  }
}


// Kept rank and basis.  The orthonormalisation of P Omega2 (all l columns, rows
// [l, 2l) of the basis panel, ld 2l) zeroed every column that fell in the span of
// the earlier ones, so the surviving columns span range(P): they are copied, in
// order, to the front of the l x l block at wout (ld l) and their count is q.  An
// eigenvalue that sits on the threshold leaves P with an intermediate eigenvalue;
// its direction then survives whole instead of displacing a kept one.  q = 0 for a
// zero or non-finite Gram matrix.
// Basis compaction of the truncation, in three launches.  Flags (grid (columns / 16,
// tasks)): column k of W survives if it has any non-zero (or non-finite) entry; the flag
// goes to sb[k].  Scan (one workgroup per task): survivors are numbered in column order,
// the destination (or -1) goes to sb[l + k] and their count q_j to the rank slot (0 when
// tr G was zero or not finite).  Copy (grid (columns / 16, tasks)): surviving columns to
// the front of wout (ld l).
__global__ __launch_bounds__(256) void k_trunc_flags(const TruncTask* __restrict__ tasks,
                                                     double* __restrict__ arena) {
  const TruncTask T = tasks[blockIdx.y];
  const int l = T.l;
  const int64_t ld = 2 * (int64_t)l;
  const double* W = arena + T.wpan + l;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int u = 0; u < 4; ++u) {
    const int k = blockIdx.x * 16 + 4 * w + u;
    if (k >= l) break;
    const double* col = W + (int64_t)k * ld;
    int nz = 0;
    for (int i = lane; i < l; i += 64) nz |= (col[i] != 0.0);
    const unsigned long long m = __ballot(nz);
    if (lane == 0) arena[T.sb + k] = m ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_trunc_compact(const TruncTask* __restrict__ tasks,
                                                       double* __restrict__ arena,
                                                       int32_t* __restrict__ ints) {
  __shared__ int32_t part[256];
  const TruncTask T = tasks[blockIdx.x];
  const int l = T.l;
  const int tid = threadIdx.x;
  double* flag = arena + T.sb;
  // exclusive scan: thread t owns columns [t cs, (t + 1) cs)
  const int cs = (l + 255) / 256;
  const int k0 = min(l, tid * cs), k1 = min(l, k0 + cs);
  int own = 0;
  for (int k = k0; k < k1; ++k) own += (flag[k] != 0.0);
  part[tid] = own;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const int q = part[255];
  int dst = part[tid] - own;
  for (int k = k0; k < k1; ++k) {
    const bool keep = flag[k] != 0.0;
    flag[l + k] = keep ? (double)dst : -1.0;
    dst += keep;
  }
  if (tid == 0) {
    const double gt = arena[T.sc];
    ints[T.qslot] = (gt > 0.0 && isfinite(gt)) ? q : 0;
  }
}

__global__ __launch_bounds__(256) void k_trunc_copy(const TruncTask* __restrict__ tasks,
                                                    double* __restrict__ arena) {
  const TruncTask T = tasks[blockIdx.y];
  const int l = T.l;
  const int64_t ld = 2 * (int64_t)l;
  const double* W = arena + T.wpan + l;
  double* out = arena + T.wout;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int u = 0; u < 4; ++u) {
    const int k = blockIdx.x * 16 + 4 * w + u;
    if (k >= l) break;
    const int d = (int)arena[T.sb + l + k];
    if (d < 0) continue;
    const double* col = W + (int64_t)k * ld;
    double* o = out + (int64_t)d * l;
    for (int i = lane; i < l; i += 64) o[i] = col[i];
  }
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
void launch_assemble_pairs(const double* values, const int64_t* idx, const int64_t* slot, int64_t n,
                           double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_assemble_pairs, dim3(grid_for(n)), dim3(256), 0, s, values, idx, slot, n, arena);
}
void launch_scatter_const(const int64_t* slot, int64_t n, double v, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_const, dim3(grid_for(n)), dim3(256), 0, s, slot, n, v, arena);
}
void launch_potrf_f64(const PotrfTask* t, int n, int nbmax, double* arena, int32_t* status, hipStream_t s) {
  if (n <= 0) return;
  if (nbmax <= 32) hipLaunchKernelGGL(k_potrf_f64<32>, dim3(n), dim3(256), 0, s, t, arena, status);
  else hipLaunchKernelGGL(k_potrf_f64<64>, dim3(n), dim3(256), 0, s, t, arena, status);
}
void launch_philox(const PhiloxTask* t, int n, int64_t max_work, double* arena, bool f32,
                   hipStream_t s) {
  if (n <= 0) return;
  const dim3 grid(grid_for(max_work, 256, 4096), n);
  if (f32) hipLaunchKernelGGL(k_philox<true>, grid, dim3(256), 0, s, t, arena);
  else hipLaunchKernelGGL(k_philox<false>, grid, dim3(256), 0, s, t, arena);
}
void launch_gram_scale(const int64_t* g, const int32_t* ld, const int32_t* nn, const int32_t* mm,
                       const int64_t* out, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gram_scale, dim3(n), dim3(256), 0, s, g, ld, nn, mm, out, arena);
}
void launch_trunc_prep(const TruncTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_prep, dim3(64, n), dim3(256), 0, s, t, arena);
}
void launch_trunc_mfill(const TruncTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_mfill, dim3(64, n), dim3(256), 0, s, t, arena);
}
void launch_trunc_flags(const TruncTask* t, int n, int lmax, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_flags, dim3((lmax + 15) / 16, n), dim3(256), 0, s, t, arena);
}
void launch_trunc_copy(const TruncTask* t, int n, int lmax, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_copy, dim3((lmax + 15) / 16, n), dim3(256), 0, s, t, arena);
}
void launch_trunc_power(const TruncTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_power, dim3(n), dim3(1024), 0, s, t, arena);
}
void launch_trunc_pmv(const TruncTask* t, int n, int lmax, int it, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_pmv, dim3((lmax + 63) / 64, n), dim3(256), 0, s, t, arena, it);
}
void launch_trunc_pfin(const TruncTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_pfin, dim3((n + 63) / 64), dim3(64), 0, s, t, n, arena);
}
void launch_trunc_x0(const TruncTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_x0, dim3(64, n), dim3(256), 0, s, t, arena);
}
void launch_trunc_p(const TruncTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_p, dim3(64, n), dim3(256), 0, s, t, arena);
}
void launch_trunc_compact(const TruncTask* t, int n, double* arena, int32_t* ints, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_trunc_compact, dim3(n), dim3(256), 0, s, t, arena, ints);
}

}  // namespace rsc
