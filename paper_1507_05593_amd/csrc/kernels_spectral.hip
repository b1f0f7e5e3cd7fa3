// gfx950 kernels of the spectral coordinates (paper Sec. 4.3): the graph Laplacian of the
// pattern times a block of three vectors, block inner products with a fixed reduction
// order (partial sums per row chunk, then summed in chunk order), block updates, the
// 3 x 3 Cholesky-QR steps, and a one-workgroup Jacobi eigen-decomposition of the
// projected block-tridiagonal matrix.  Every block of three vectors is column-major with
// leading dimension n.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace rsc {

namespace {

__device__ __forceinline__ double wsum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

// Y = L X: for row i, (number of stored off-diagonal entries) x_i minus their x_j.
__global__ __launch_bounds__(256) void k_lap3(const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colind, int64_t n,
                                              const double* __restrict__ X, double* __restrict__ Y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int deg = 0;
  for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    const int64_t j = colind[p];
    if (j == i) continue;
    ++deg;
    s0 += X[j];
    s1 += X[j + n];
    s2 += X[j + 2 * n];
  }
  Y[i] = deg * X[i] - s0;
  Y[i + n] = deg * X[i + n] - s1;
  Y[i + 2 * n] = deg * X[i + 2 * n] - s2;
}

// Partial inner products of one chunk of kSpChunk rows and one group of kSpGroup
// columns (grid: chunks x groups): part[(chunk * ncols + c) * 3 + k] = sum over the chunk's
// rows of Q(i, c) W(i, k), c < ncols, k < 3.  ncols < 0: one column, the weights i + 1.
// Each thread keeps its rows' W in registers and the group's 3 kSpGroup sums; lanes are
// summed by a fixed butterfly, then the four waves in order.
__global__ __launch_bounds__(256) void k_bdots(const double* __restrict__ Q, int64_t ldq, int ncols,
                                               const double* __restrict__ W, int64_t n,
                                               double* __restrict__ part) {
  __shared__ double red[3 * kSpGroup][4];
  constexpr int R = kSpChunk / 256;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t r0 = blockIdx.x * (int64_t)kSpChunk;
  const int nc = ncols < 0 ? 1 : ncols;
  const int g0 = blockIdx.y * kSpGroup, g1 = min(nc, g0 + kSpGroup);
  double w0[R], w1[R], w2[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int64_t i = r0 + tid + 256 * u;
    const bool in = i < n;
    w0[u] = in ? W[i] : 0.0;
    w1[u] = in ? W[i + n] : 0.0;
    w2[u] = in ? W[i + 2 * n] : 0.0;
  }
  double acc[3 * kSpGroup];
#pragma unroll
  for (int t = 0; t < 3 * kSpGroup; ++t) acc[t] = 0.0;
#pragma unroll
  for (int g = 0; g < kSpGroup; ++g) {
    const int c = g0 + g;
    if (c >= g1) break;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = r0 + tid + 256 * u;
      const double q = (i < n) ? (ncols < 0 ? (double)(i + 1) : Q[i + c * ldq]) : 0.0;
      acc[3 * g] = fma(q, w0[u], acc[3 * g]);
      acc[3 * g + 1] = fma(q, w1[u], acc[3 * g + 1]);
      acc[3 * g + 2] = fma(q, w2[u], acc[3 * g + 2]);
    }
  }
#pragma unroll
  for (int t = 0; t < 3 * kSpGroup; ++t) {
    const double v = wsum64(acc[t]);
    if (lane == 0) red[t][w] = v;
  }
  __syncthreads();
  const int nout = 3 * (g1 - g0);
  if (tid < nout)
    part[((int64_t)blockIdx.x * nc + g0) * 3 + tid] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
}

// out[(r0 + o / 3) + (c0 + o % 3) ld] = the sum over the chunks of part[.. o], o < nout:
// one wave per output, lane l adding chunks l, l + 64, ... in order, then a fixed butterfly.
__global__ __launch_bounds__(256) void k_bsum(const double* __restrict__ part, int nchunks, int nout,
                                              double* __restrict__ out, int ld, int r0, int c0) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= nout) return;
  double s = 0.0;
  for (int b = lane; b < nchunks; b += 64) s += part[(int64_t)b * nout + o];
  s = wsum64(s);
  if (lane == 0) out[(r0 + o / 3) + (int64_t)(c0 + o % 3) * ld] = s;
}

// W -= Q(:, 0:ncols) C, C ncols x 3 (ld ncols).
__global__ __launch_bounds__(256) void k_bupd(const double* __restrict__ Q, int64_t ldq, int ncols,
                                              const double* __restrict__ C, double* __restrict__ W,
                                              int64_t n) {
  __shared__ double cs[3 * kSpMaxCols];
  for (int t = threadIdx.x; t < 3 * ncols; t += blockDim.x) cs[t] = C[t];
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int c = 0; c < ncols; ++c) {
    const double q = Q[i + c * ldq];
    a0 = fma(q, cs[c], a0);
    a1 = fma(q, cs[c + ncols], a1);
    a2 = fma(q, cs[c + 2 * ncols], a2);
  }
  W[i] -= a0;
  W[i + n] -= a1;
  W[i + 2 * n] -= a2;
}

// Cholesky of the 3 x 3 Gram matrix G = R^T R (one thread): Rinv = R^{-1}; pass 0 keeps R
// in racc, pass 1 multiplies it in (racc = R racc, the factor of two Cholesky-QR passes)
// and, when T is given, stores it as the block (r0, c0) of T and its transpose at (c0, r0).
// A pivot that is not positive and finite (the Krylov space is exhausted) sets *flag.
__global__ void k_chol3(const double* __restrict__ G, double* __restrict__ rinv, double* __restrict__ racc,
                        int pass, double* __restrict__ T, int ldt, int r0, int c0, int32_t* __restrict__ flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double g[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) g[a][b] = G[a + 3 * b];
  double r[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    double d = g[a][a];
    for (int k = 0; k < a; ++k) d -= r[k][a] * r[k][a];
    if (!(d > 0.0) || !isfinite(d)) { ok = false; d = 1.0; }
    r[a][a] = sqrt(d);
    for (int b = a + 1; b < 3; ++b) {
      double e = g[a][b];
      for (int k = 0; k < a; ++k) e -= r[k][a] * r[k][b];
      r[a][b] = e / r[a][a];
    }
  }
  if (!ok) *flag = 1;
  // inverse of the upper-triangular R
  double v[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int b = 0; b < 3; ++b) {
    v[b][b] = 1.0 / r[b][b];
    for (int a = b - 1; a >= 0; --a) {
      double e = 0.0;
      for (int k = a + 1; k <= b; ++k) e += r[a][k] * v[k][b];
      v[a][b] = -e / r[a][a];
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) rinv[a + 3 * b] = v[a][b];
  double m[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      if (pass == 0) {
        m[a][b] = r[a][b];
      } else {
        double e = 0.0;
        for (int k = 0; k < 3; ++k) e += r[a][k] * racc[k + 3 * b];
        m[a][b] = e;
      }
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) racc[a + 3 * b] = m[a][b];
  if (pass == 1 && T)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        T[(r0 + a) + (int64_t)(c0 + b) * ldt] = m[a][b];
        T[(c0 + b) + (int64_t)(r0 + a) * ldt] = m[a][b];
      }
}

// W = W Rinv (Rinv 3 x 3, column-major).
__global__ __launch_bounds__(256) void k_bscale(double* __restrict__ W, int64_t n, const double* __restrict__ rinv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x0 = W[i], x1 = W[i + n], x2 = W[i + 2 * n];
  W[i] = x0 * rinv[0];
  W[i + n] = x0 * rinv[3] + x1 * rinv[4];
  W[i + 2 * n] = x0 * rinv[6] + x1 * rinv[7] + x2 * rinv[8];
}

__global__ __launch_bounds__(256) void k_bcopy(const double* __restrict__ src, double* __restrict__ dst, int64_t len,
                                               double v, int fill) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < len) dst[i] = fill ? v : src[i];
}

// Eigen-decomposition of the symmetric N x N matrix T (ld ldt, N <= kSpMaxN) by cyclic
// Jacobi rotations in one workgroup, the matrix in LDS and the rotations' product in V.
// Each round rotates Np/2 disjoint index pairs at once (a fixed round-robin schedule over
// Np - 1 rounds per sweep, Np = N rounded up to even, the extra index an inert diagonal
// entry larger than any eigenvalue); the pair (p, q) is rotated by J = [c s; -s c] with
// t = s / c the smaller root of t^2 + 2 theta t - 1 = 0, theta = (T_qq - T_pp) / (2 T_pq),
// which zeroes T_pq.  A' = J^T A J acts on the 2 x 2 blocks (pair k rows, pair k' columns)
// one at a time, so a round is one pass over those blocks.  Sweeps stop when the
// off-diagonal mass falls below 1e-32 of the whole.  Output: the eigenvectors as the
// columns of V (Np x Np, ld Np), the eigenvalues in evals, and in sel the indices of the
// three smallest (ascending).
__global__ __launch_bounds__(256) void k_jacobi(const double* __restrict__ T, int N, int ldt,
                                                double* __restrict__ V, double* __restrict__ evals,
                                                int32_t* __restrict__ sel) {
  extern __shared__ double A[];   // Np x (Np + 1), A(p, q) at p + q (Np + 1)
  __shared__ double cs[kSpMaxN / 2 + 1], sn[kSpMaxN / 2 + 1];
  __shared__ int pp[kSpMaxN / 2 + 1], qq[kSpMaxN / 2 + 1];
  __shared__ double red[8];
  __shared__ int go;
  const int Np = N + (N & 1), L = Np + 1, half = Np / 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < Np * Np; e += nt) {
    const int p = e % Np, q = e / Np;
    A[p + q * L] = (p < N && q < N) ? T[p + (int64_t)q * ldt] : ((p == q) ? DBL_MAX / 4 : 0.0);
    V[e] = (p == q) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, all = 0.0;
    for (int e = tid; e < N * N; e += nt) {
      const int p = e % N, q = e / N;
      const double a = A[p + q * L];
      all += a * a;
      if (p != q) off += a * a;
    }
    off = wsum64(off);
    all = wsum64(all);
    if ((tid & 63) == 0) { red[tid >> 6] = off; red[4 + (tid >> 6)] = all; }
    __syncthreads();
    if (tid == 0) go = ((red[0] + red[1]) + (red[2] + red[3]) > 1e-32 * ((red[4] + red[5]) + (red[6] + red[7]))) ? 1 : 0;
    __syncthreads();
    if (!go) break;
    for (int rd = 0; rd < Np - 1; ++rd) {
      if (tid < half) {
        // round-robin pairs: index 0 fixed, the others rotated by rd
        const int a = tid, b = Np - 1 - tid;
        int p = a == 0 ? 0 : ((a - 1 + rd) % (Np - 1)) + 1;
        int q = ((b - 1 + rd) % (Np - 1)) + 1;
        if (p > q) { const int x = p; p = q; q = x; }
        const double apq = A[p + q * L];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300) {
          const double th = (A[q + q * L] - A[p + p * L]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        cs[tid] = c; sn[tid] = s; pp[tid] = p; qq[tid] = q;
      }
      __syncthreads();
      // 2 x 2 blocks (rows of pair k, columns of pair kk): J_k^T A J_kk
      for (int e = tid; e < half * half; e += nt) {
        const int k = e % half, kk = e / half;
        const int p = pp[k], q = qq[k], p2 = pp[kk], q2 = qq[kk];
        const double c = cs[k], s = sn[k], c2 = cs[kk], s2 = sn[kk];
        const double a = A[p + p2 * L], b = A[p + q2 * L], d = A[q + p2 * L], f = A[q + q2 * L];
        // rows: [c -s; s c] applied to (row p, row q)
        const double ra = c * a - s * d, rb = c * b - s * f, rd2 = s * a + c * d, rf = s * b + c * f;
        // columns: (col p2, col q2) [c2 s2; -s2 c2]
        A[p + p2 * L] = c2 * ra - s2 * rb;
        A[p + q2 * L] = s2 * ra + c2 * rb;
        A[q + p2 * L] = c2 * rd2 - s2 * rf;
        A[q + q2 * L] = s2 * rd2 + c2 * rf;
      }
      // V J: rows j, columns of pair k
      for (int e = tid; e < half * Np; e += nt) {
        const int j = e % Np, k = e / Np;
        const int p = pp[k], q = qq[k];
        const double c = cs[k], s = sn[k];
        const double u = V[j + p * Np], v = V[j + q * Np];
        V[j + p * Np] = c * u - s * v;
        V[j + q * Np] = s * u + c * v;
      }
      __syncthreads();
    }
  }
  for (int p = tid; p < N; p += nt) evals[p] = A[p + p * L];
  if (tid == 0) {
    int s0 = -1, s1 = -1, s2 = -1;
    for (int p = 0; p < N; ++p) {
      const double d = A[p + p * L];
      if (s0 < 0 || d < A[s0 + s0 * L]) { s2 = s1; s1 = s0; s0 = p; }
      else if (s1 < 0 || d < A[s1 + s1 * L]) { s2 = s1; s1 = p; }
      else if (s2 < 0 || d < A[s2 + s2 * L]) { s2 = p; }
    }
    sel[0] = s0; sel[1] = s1; sel[2] = s2;
  }
}

// Y(:, k) = Q(:, 1 : 1 + nc) V(0 : nc, sel[k]), k < 3 (V ld ldv).
__global__ __launch_bounds__(256) void k_ritz(const double* __restrict__ Q, int64_t ldq, int nc,
                                              const double* __restrict__ V, int ldv,
                                              const int32_t* __restrict__ sel,
                                              double* __restrict__ Y, int64_t n) {
  __shared__ double vs[3 * kSpMaxN];
  for (int t = threadIdx.x; t < 3 * nc; t += blockDim.x) vs[t] = V[(t % nc) + (int64_t)sel[t / nc] * ldv];
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int c = 0; c < nc; ++c) {
    const double q = Q[i + (1 + c) * ldq];
    a0 = fma(q, vs[c], a0);
    a1 = fma(q, vs[c + nc], a1);
    a2 = fma(q, vs[c + 2 * nc], a2);
  }
  Y[i] = a0;
  Y[i + n] = a1;
  Y[i + 2 * n] = a2;
}

// Column k of Y negated when sums[k] < 0.
__global__ __launch_bounds__(256) void k_bsign(double* __restrict__ Y, int64_t n, const double* __restrict__ sums) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k)
    if (sums[k] < 0.0) Y[i + k * n] = -Y[i + k * n];
}

static inline unsigned sp_blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_lap3(const int64_t* rowptr, const int32_t* colind, int64_t n, const double* X, double* Y,
                 hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_lap3, dim3(sp_blocks(n)), dim3(256), 0, s, rowptr, colind, n, X, Y);
}
void launch_bdots(const double* Q, int64_t ldq, int ncols, const double* W, int64_t n, double* part,
                  hipStream_t s) {
  const int nchunks = (int)((n + kSpChunk - 1) / kSpChunk);
  const int ngroups = ((ncols < 0 ? 1 : ncols) + kSpGroup - 1) / kSpGroup;
  if (nchunks > 0 && ngroups > 0)
    hipLaunchKernelGGL(k_bdots, dim3(nchunks, ngroups), dim3(256), 0, s, Q, ldq, ncols, W, n, part);
}
void launch_bsum(const double* part, int nchunks, int nout, double* out, int ld, int r0, int c0, hipStream_t s) {
  if (nout > 0) hipLaunchKernelGGL(k_bsum, dim3((nout + 3) / 4), dim3(256), 0, s, part, nchunks, nout, out, ld, r0, c0);
}
void launch_bupd(const double* Q, int64_t ldq, int ncols, const double* C, double* W, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_bupd, dim3(sp_blocks(n)), dim3(256), 0, s, Q, ldq, ncols, C, W, n);
}
void launch_chol3(const double* G, double* rinv, double* racc, int pass, double* T, int ldt, int r0, int c0,
                  int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_chol3, dim3(1), dim3(64), 0, s, G, rinv, racc, pass, T, ldt, r0, c0, flag);
}
void launch_bscale(double* W, int64_t n, const double* rinv, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_bscale, dim3(sp_blocks(n)), dim3(256), 0, s, W, n, rinv);
}
void launch_bcopy(const double* src, double* dst, int64_t len, double v, bool fill, hipStream_t s) {
  if (len > 0) hipLaunchKernelGGL(k_bcopy, dim3(sp_blocks(len)), dim3(256), 0, s, src, dst, len, v, fill ? 1 : 0);
}
void launch_jacobi(const double* T, int N, int ldt, double* V, double* evals, int32_t* sel, hipStream_t s) {
  const int Np = N + (N & 1);
  const size_t lds = sizeof(double) * (size_t)Np * (Np + 1);
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), lds, s, T, N, ldt, V, evals, sel);
}
void launch_ritz(const double* Q, int64_t ldq, int nc, const double* V, int ldv, const int32_t* sel, double* Y,
                 int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_ritz, dim3(sp_blocks(n)), dim3(256), 0, s, Q, ldq, nc, V, ldv, sel, Y, n);
}
void launch_bsign(double* Y, int64_t n, const double* sums, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_bsign, dim3(sp_blocks(n)), dim3(256), 0, s, Y, n, sums);
}

}  // namespace rsc
