// gfx950 kernels of the solve phase: the two supernodal triangular sweeps with the
// stored factor (paper Sec. 1: two triangular solves), CSR SpMV, wavefront
// reductions for the CG scalars (Sec. 5.2, 6.1.1), and the solve adjoint.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "kernels.h"
#include "tasks.h"

namespace rsc {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide deterministic sum (fixed reduction tree) of 256 threads.
__device__ double block_sum(double v) {
  __shared__ double red[4];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- sweeps

// The factor operands of the sweeps (L^O_j, V_j, W_j = M_j U_j, the inverse diagonal
// blocks) are read through F: the arena itself (TF = double), or in the mixed forms its
// FP32 copy (TF = float: L^O_j, V_j and W_j at their arena offsets, the inverse blocks M_j compact,
// written once the factorization is complete); the vectors and every sum stay FP64.

// out[t] = sum_{m < K} X(t, m) v[m] for up to 64 rows: lane = row (coalesced column
// reads), the 4 waves split the inner dimension and their partial sums are added in
// a fixed order.
template <typename TF>
__global__ __launch_bounds__(256) void k_gemv_n(const GemvTask* __restrict__ tasks,
                                                double* __restrict__ arena, const TF* __restrict__ F,
                                                const int32_t* __restrict__ ilim) {
  __shared__ double part[4][64];
  const GemvTask T = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int K = T.kdim >= 0 ? T.kdim : min(ilim[-1 - T.kdim], T.kmax);
  double acc = 0.0;
  if (lane < T.rows) {
    const int per = (K + 3) / 4;
    const int m0 = w * per, m1 = min(K, m0 + per);
    const TF* X = F + T.x + lane;
    const double* v = arena + T.v;
#pragma unroll 8
    for (int m = m0; m < m1; ++m) acc += (double)X[(int64_t)m * T.ldx] * v[m];
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && lane < T.rows)
    arena[T.out + lane] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// Backward diagonal solve chunk: rows i in [i0, i0 + 64) (lanes) of M (w - s) over the
// columns [t0, t1) (kind 0), or of -W u over W's columns [t0, t1) below the device rank
// (kind 1); the vector is staged in LDS (s or u added up from the column dots' partial
// blocks when they were cut into row chunks), the four waves take consecutive column
// quarters, and their sums are added in a fixed order into one partial block (at slots
// past those it reads).
template <typename TF>
__global__ __launch_bounds__(256) void k_row_part(const RowChunk* __restrict__ chunks,
                                                  const double* __restrict__ arena, const TF* __restrict__ F,
                                                  const int32_t* __restrict__ ilim,
                                                  double* __restrict__ part) {
  __shared__ double v[kRowChunkMax];
  __shared__ double red[4][64];
  const RowChunk T = chunks[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t1 = T.kind ? min(T.t1, min(ilim[T.qslot], T.kmax)) : T.t1;
  const int n = max(0, t1 - T.t0);
  for (int t = threadIdx.x; t < n; t += 256) {
    const int col = T.t0 + t;
    double sv = 0.0;                       // s or u from the column dots' partial blocks
    if (T.sns > 0) {
      const double* pp = part + ((int64_t)T.sbase + (int64_t)(col >> 4) * T.sns) * 64 + (col & 15);
      for (int q = 0; q < T.sns; ++q) sv += pp[(int64_t)q * 64];
    }
    if (T.kind) {
      v[t] = T.sns > 0 ? sv : arena[T.w + col];
    } else {
      const double a = arena[T.w + col];
      v[t] = T.s >= 0 ? a - arena[T.s + col] : (T.sns > 0 ? a - sv : a);
    }
  }
  __syncthreads();
  const int i = T.i0 + lane;
  double acc = 0.0;
  if (i < T.c) {
    const int per = (n + 3) / 4;
    const int ta = T.t0 + w * per, tb = min(t1, ta + per);
    const TF* M = F + T.m + i;
#pragma unroll 8
    for (int t = T.kind ? ta : max(ta, i); t < tb; ++t) acc += (double)M[(int64_t)t * T.ld] * v[t - T.t0];
  }
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0) {
    const double sum = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    part[(int64_t)T.slot * 64 + lane] = T.kind ? -sum : sum;
  }
}

// Applies the partial blocks of one vector block in slot order (see PartApply).
__global__ __launch_bounds__(64) void k_part_apply(const PartApply* __restrict__ tasks,
                                                   const double* __restrict__ part,
                                                   double* __restrict__ arena) {
  const PartApply T = tasks[blockIdx.x];
  const int r = threadIdx.x;
  if (r >= T.nrows) return;
  double s = 0.0;
  for (int q = 0; q < T.ns; ++q) s += part[(int64_t)(T.s0 + q) * 64 + r];
  if (T.mode == 0) arena[T.dst + r] -= s;
  else arena[T.dst + r] = s;
}

// dst[begin + t] = src[idx[begin + t]] for t < count: the off-diagonal rows of one
// supernode gathered once per sweep into a contiguous vector.
__global__ void k_gather_rows(const int64_t* __restrict__ tasks, const int64_t* __restrict__ idx,
                              const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t b = tasks[2 * blockIdx.x], n = tasks[2 * blockIdx.x + 1];
  for (int64_t t = threadIdx.x; t < n; t += 256) dst[b + t] = src[idx[b + t]];
}

// Column dots, 16 columns per workgroup: wave w takes columns col0 + 4w .. col0 + 4w + 3,
// one per 16-lane group, the group's lanes striding the rows (one 128-byte line per
// group and load, unrolled so several loads are in flight); then a fixed butterfly
// within each group.  Short columns (the many small supernodes) keep most lanes busy.
template <typename TF>
__global__ __launch_bounds__(256) void k_coldot(const ColDotTask* __restrict__ tasks,
                                                double* __restrict__ arena, const TF* __restrict__ F,
                                                const int64_t* __restrict__ gidx,
                                                const int32_t* __restrict__ ilim,
                                                double* __restrict__ part) {
  const ColDotTask T = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int ncols = T.ncols >= 0 ? T.ncols : min(ilim[-1 - T.ncols], T.kmax);
  const double* in = arena + T.in;
  const int col = T.col0 + w * 4 + g;
  double acc = 0.0;
  if (col < ncols) {
    const int rows = min(T.tri ? col + 1 : T.rows, T.r1);
    const TF* X = F + T.x + (int64_t)col * T.ldx;
    if (T.idx >= 0) {
      const int64_t* ix = gidx + T.idx;
#pragma unroll 8
      for (int t = T.r0 + r; t < rows; t += 16) acc += (double)X[t] * in[ix[t]];
    } else {
#pragma unroll 8
      for (int t = T.r0 + r; t < rows; t += 16) acc += (double)X[t] * in[t];
    }
  }
  for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (r == 0) {
    if (T.slot >= 0) part[(int64_t)T.slot * 64 + (col - T.col0)] = acc;
    else if (col < ncols) arena[T.out + col] = acc;
  }
}

// y[rows[t]] -= sum of part[contrib[p]], p in [ptr[t], ptr[t+1]), in list order.
__global__ void k_row_gather(const int64_t* __restrict__ rows, const int64_t* __restrict__ ptr,
                             const int64_t* __restrict__ contrib, int64_t nrows,
                             const double* __restrict__ part, double* __restrict__ y) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  double s = 0.0;
  for (int64_t p = ptr[t]; p < ptr[t + 1]; ++p) s += part[contrib[p]];
  y[rows[t]] -= s;
}

// Small-supernode sweep levels (SweepTask): one workgroup of 64 or 256 threads per
// supernode runs the whole level step of a sweep, its vectors in LDS.  Column dots use
// 16 lanes per column (a fixed butterfly at the end), row products one thread per row
// (column-major operands: the threads of a column read consecutive entries).
__device__ __forceinline__ double sum16(double acc) {
  for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  return acc;
}

// Forward step:  y_C minus the descendants' contributions (pulled from zr in list order),
// w_C = (L^D_j)^{-1} y_C = M_j^T y_C, and t = L^O_j w_C or V_j (U_j^T w_C) = V_j (W_j^T y_C)
// stored in the supernode's zr slots, from which its ancestors pull.  LDS: y_C, w_C (cpad
// each), W^T y.
template <typename TF>
__global__ __launch_bounds__(256) void k_sweep_fwd(const SweepTask* __restrict__ tasks,
                                                   const double* __restrict__ y, double* __restrict__ w,
                                                   double* __restrict__ zr, const TF* __restrict__ F,
                                                   const int32_t* __restrict__ ilim,
                                                   const int64_t* __restrict__ pull_ptr,
                                                   const int64_t* __restrict__ pull_idx, int32_t cpad) {
  extern __shared__ double sm[];
  const SweepTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int g = tid >> 4, gl = tid & 15, ng = nt >> 4;
  double* yc = sm;
  double* wc = sm + cpad;
  double* tq = sm + 2 * cpad;
  for (int i = tid; i < T.c; i += nt) {
    const int64_t row = T.first + i;
    double s = y[row];
    for (int64_t p = pull_ptr[row]; p < pull_ptr[row + 1]; ++p) s -= zr[pull_idx[p]];
    yc[i] = s;
  }
  __syncthreads();
  for (int col = g; col < T.c; col += ng) {
    const TF* X = F + T.m + (int64_t)col * T.ld;
    double acc = 0.0;
    for (int t = gl; t <= col; t += 16) acc += (double)X[t] * yc[t];
    acc = sum16(acc);
    if (gl == 0) {
      wc[col] = acc;
      w[T.first + col] = acc;
    }
  }
  __syncthreads();
  const double* v = wc;
  int K = T.c;
  if (T.u >= 0) {
    K = min(ilim[T.qslot], T.kmax);
    for (int k = g; k < K; k += ng) {
      const TF* W = F + T.u + (int64_t)k * T.c;
      double acc = 0.0;
      for (int i = gl; i < T.c; i += 16) acc += (double)W[i] * yc[i];
      acc = sum16(acc);
      if (gl == 0) tq[k] = acc;
    }
    __syncthreads();
    v = tq;
  }
  for (int i = tid; i < T.r; i += nt) {
    const TF* X = F + T.x + i;
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < K; ++k) acc += (double)X[(int64_t)k * T.r] * v[k];
    zr[T.rows + i] = acc;
  }
}

// Backward step:  z_R gathered from zz, s = (L^O_j)^T z_R or U_j (V_j^T z_R), and
// z_C = (L^D_j)^{-T} (w_C - s) = M_j (w_C - s) into zz -- for a compressed supernode
// M_j w_C - W_j (V_j^T z_R).  LDS: w_C - s (cpad), V^T z_R (lpad), z_R.
template <typename TF>
__global__ __launch_bounds__(256) void k_sweep_bwd(const SweepTask* __restrict__ tasks,
                                                   const double* __restrict__ w, double* __restrict__ zz,
                                                   const TF* __restrict__ F,
                                                   const int32_t* __restrict__ ilim,
                                                   const int64_t* __restrict__ rows_idx, int32_t cpad,
                                                   int32_t lpad) {
  extern __shared__ double sm[];
  const SweepTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int g = tid >> 4, gl = tid & 15, ng = nt >> 4;
  double* v = sm;
  double* uq = sm + cpad;
  double* zR = sm + cpad + lpad;
  for (int i = tid; i < T.r; i += nt) zR[i] = zz[rows_idx[T.rows + i]];
  __syncthreads();
  if (T.u < 0) {
    for (int col = g; col < T.c; col += ng) {
      const TF* X = F + T.x + (int64_t)col * T.r;
      double acc = 0.0;
      for (int i = gl; i < T.r; i += 16) acc += (double)X[i] * zR[i];
      acc = sum16(acc);
      if (gl == 0) v[col] = w[T.first + col] - acc;
    }
  } else {
    const int K = min(ilim[T.qslot], T.kmax);
    for (int k = g; k < K; k += ng) {
      const TF* V = F + T.x + (int64_t)k * T.r;
      double acc = 0.0;
      for (int i = gl; i < T.r; i += 16) acc += (double)V[i] * zR[i];
      acc = sum16(acc);
      if (gl == 0) uq[k] = acc;
    }
    for (int i = tid; i < T.c; i += nt) v[i] = w[T.first + i];
  }
  __syncthreads();
  const int K = T.u >= 0 ? min(ilim[T.qslot], T.kmax) : 0;
  for (int i = tid; i < T.c; i += nt) {
    const TF* M = F + T.m + i;
    double acc = 0.0;
#pragma unroll 8
    for (int t = i; t < T.c; ++t) acc += (double)M[(int64_t)t * T.ld] * v[t];
    if (K > 0) {
      const TF* W = F + T.u + i;
      double wu = 0.0;
#pragma unroll 8
      for (int k = 0; k < K; ++k) wu += (double)W[(int64_t)k * T.c] * uq[k];
      acc -= wu;
    }
    zz[T.first + i] = acc;
  }
}

__global__ void k_gather_perm(int64_t n, const int64_t* __restrict__ perm,
                              const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_scatter_perm(int64_t n, const int64_t* __restrict__ perm,
                               const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[perm[i]] = src[i];
}

// ---------------------------------------------------------------- CG vectors

// Ap = A p on one chunk of rows (one thread per row), partial = p . Ap for the chunk.
__global__ __launch_bounds__(256) void k_spmv_dot(const Chunk* __restrict__ chunks,
                                                  const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind,
                                                  const double* __restrict__ vals,
                                                  const double* __restrict__ p,
                                                  double* __restrict__ Ap,
                                                  double* __restrict__ partial) {
  const Chunk C = chunks[blockIdx.x];
  const int64_t i = C.begin + threadIdx.x;
  double d = 0.0;
  if (i < C.end) {
    // a row's entries eight at a time: the index and value loads of a group, then its
    // gathers, are in flight together; the products are added in entry order as before
    double s = 0.0;
    const int64_t q0 = rowptr[i], q1 = rowptr[i + 1];
    for (int64_t qb = q0; qb < q1; qb += 8) {
      int32_t cq[8];
      double vq[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = qb + u < q1;
        cq[u] = in ? colind[qb + u] : (int32_t)i;
        vq[u] = in ? vals[qb + u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double t = vq[u] * p[cq[u]];
        if (qb + u < q1) s += t;
      }
    }
    Ap[i] = s;
    d = p[i] * s;
  }
  d = block_sum(d);
  if (threadIdx.x == 0) partial[blockIdx.x] = d;
}

__global__ __launch_bounds__(256) void k_dot_partial(const Chunk* __restrict__ chunks,
                                                     const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ partial) {
  const Chunk C = chunks[blockIdx.x];
  const int64_t i = C.begin + threadIdx.x;
  double d = (i < C.end) ? a[i] * b[i] : 0.0;
  d = block_sum(d);
  if (threadIdx.x == 0) partial[blockIdx.x] = d;
}

// partial = sum over the chunk of (b - Ax)^2 (true residual).
__global__ __launch_bounds__(256) void k_resid_partial(const Chunk* __restrict__ chunks,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ ax,
                                                       double* __restrict__ partial) {
  const Chunk C = chunks[blockIdx.x];
  const int64_t i = C.begin + threadIdx.x;
  double d = 0.0;
  if (i < C.end) {
    const double t = b[i] - ax[i];
    d = t * t;
  }
  d = block_sum(d);
  if (threadIdx.x == 0) partial[blockIdx.x] = d;
}

// out[s] = sum of the partials of segment s (one workgroup per segment, fixed
// strided assignment and reduction tree: deterministic).
__global__ __launch_bounds__(256) void k_seg_sum(const int32_t* __restrict__ seg_ptr, int32_t nseg,
                                                 const double* __restrict__ partial,
                                                 double* __restrict__ out) {
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int c = seg_ptr[s] + threadIdx.x; c < seg_ptr[s + 1]; c += 256) acc += partial[c];
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[s] = acc;
}

// A system's sum of chunk partials (as k_seg_sum) followed by the CG scalar step that
// uses it, one workgroup per system: kind 0, p^T A p then alpha = r^T z / p^T A p (and
// the "any system active" flag cleared for this iteration's test); kind 1, r^T r then
// the convergence test |r| / |b| <= rtol, which counts the iteration; kind 2, the new
// r^T z then beta.  A non-positive p^T A p or r^T z stops the system and flags a
// breakdown.
__global__ __launch_bounds__(256) void k_seg_step(const int32_t* __restrict__ seg_ptr,
                                                  const double* __restrict__ partial, PcgScalars sc,
                                                  double rtol, double* __restrict__ arena,
                                                  int32_t* __restrict__ ints, int kind) {
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int c = seg_ptr[s] + threadIdx.x; c < seg_ptr[s + 1]; c += 256) acc += partial[c];
  acc = block_sum(acc);
  if (threadIdx.x != 0) return;
  int32_t* active = ints + sc.active;
  if (kind == 0) {
    arena[sc.pAp + s] = acc;
    if (s == 0) ints[sc.any] = 0;
    const double rz = arena[sc.rz + s];
    double a = 0.0;
    if (active[s]) {
      if (!(acc > 0.0) || !(rz > 0.0)) {
        ints[sc.breakdown] = 1;
        active[s] = 0;
      } else {
        a = rz / acc;
      }
    }
    arena[sc.alpha + s] = a;
  } else if (kind == 1) {
    arena[sc.rr + s] = acc;
    if (!active[s]) return;
    ints[sc.iters + s] += 1;
    const double rel = sqrt(acc) / arena[sc.bnorm + s];
    arena[sc.rel + s] = rel;
    if (rel <= rtol || !isfinite(rel)) active[s] = 0;
    else atomicOr(ints + sc.any, 1);
  } else {
    arena[sc.rznew + s] = acc;
    if (!active[s]) { arena[sc.beta + s] = 0.0; return; }
    const double rzo = arena[sc.rz + s];
    if (!(acc > 0.0) || !(rzo > 0.0)) {
      ints[sc.breakdown] = 1;
      active[s] = 0;
      arena[sc.beta + s] = 0.0;
      return;
    }
    arena[sc.beta + s] = acc / rzo;
    arena[sc.rz + s] = acc;
  }
}

__global__ __launch_bounds__(256) void k_pcg_xr(const Chunk* __restrict__ chunks, PcgScalars sc,
                                                double* __restrict__ arena,
                                                const int32_t* __restrict__ ints,
                                                double* __restrict__ partial) {
  const Chunk C = chunks[blockIdx.x];
  const int64_t i = C.begin + threadIdx.x;
  const double a = arena[sc.alpha + C.seg];
  double d = 0.0;
  if (i < C.end) {
    double* x = arena + sc.x;
    double* r = arena + sc.r;
    const double* p = arena + sc.p;
    const double* Ap = arena + sc.Ap;
    if (ints[sc.active + C.seg]) {
      x[i] += a * p[i];
      r[i] -= a * Ap[i];
    }
    d = r[i] * r[i];
  }
  d = block_sum(d);
  if (threadIdx.x == 0) partial[blockIdx.x] = d;
}

__global__ __launch_bounds__(256) void k_pcg_p(const Chunk* __restrict__ chunks, PcgScalars sc,
                                               double* __restrict__ arena,
                                               const int32_t* __restrict__ ints, int first) {
  const Chunk C = chunks[blockIdx.x];
  const int64_t i = C.begin + threadIdx.x;
  if (i >= C.end) return;
  double* p = arena + sc.p;
  if (first) {              // p = z (p holds no value yet: never read it)
    p[i] = arena[sc.z + i];
    return;
  }
  if (!ints[sc.active + C.seg]) return;
  p[i] = arena[sc.z + i] + arena[sc.beta + C.seg] * p[i];
}

// Start of CG: x = 0, r = b, bnorm = ||b|| (set by the caller), iters = 0, active = bnorm > 0.
__global__ void k_pcg_start(int32_t nseg, PcgScalars sc, double* __restrict__ arena,
                            int32_t* __restrict__ ints) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) { ints[sc.breakdown] = 0; }
  if (s >= nseg) return;
  const double bb = arena[sc.bnorm + s];
  arena[sc.bnorm + s] = sqrt(bb);
  ints[sc.active + s] = bb > 0.0 ? 1 : 0;
  ints[sc.iters + s] = 0;
  arena[sc.rel + s] = bb > 0.0 ? 1.0 : 0.0;
}

__global__ void k_copy(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------- adjoint

__global__ void k_grad_values(int64_t n, const int64_t* __restrict__ rowptr,
                              const int32_t* __restrict__ colind, const double* __restrict__ lam,
                              const double* __restrict__ x, double* __restrict__ g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double li = lam[i];
  for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) g[q] = -li * x[colind[q]];
}

__global__ void k_grad_faces(int64_t nf, const int32_t* __restrict__ fi,
                             const int32_t* __restrict__ fj, const double* __restrict__ lam,
                             const double* __restrict__ x, double* __restrict__ g) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int i = fi[f], j = fj[f];
  g[f] = (j >= 0) ? -(lam[i] - lam[j]) * (x[i] - x[j]) : -lam[i] * x[i];
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_gemv_n(const GemvTask* t, int n, double* arena, const float* f32, const int32_t* ilim,
                   hipStream_t s) {
  if (n <= 0) return;
  if (f32) hipLaunchKernelGGL(k_gemv_n<float>, dim3(n), dim3(256), 0, s, t, arena, f32, ilim);
  else hipLaunchKernelGGL(k_gemv_n<double>, dim3(n), dim3(256), 0, s, t, arena, (const double*)arena, ilim);
}
void launch_row_part(const RowChunk* c, int n, const double* arena, const float* f32,
                     const int32_t* ilim, double* part, hipStream_t s) {
  if (n <= 0) return;
  if (f32) hipLaunchKernelGGL(k_row_part<float>, dim3(n), dim3(256), 0, s, c, arena, f32, ilim, part);
  else hipLaunchKernelGGL(k_row_part<double>, dim3(n), dim3(256), 0, s, c, arena, arena, ilim, part);
}

// FP32 copy of the factor operands the sweeps read, at the arena's offsets: one task per
// block of at most 64 columns and kConvRows rows (see ConvTask).
__global__ __launch_bounds__(256) void k_to_f32(const ConvTask* __restrict__ tasks,
                                                const double* __restrict__ arena,
                                                float* __restrict__ f32) {
  const ConvTask T = tasks[blockIdx.x];
  if (T.rows >= 256) {
    for (int c = 0; c < T.cols; ++c) {
      const int64_t o = T.off + (int64_t)c * T.ld, d = T.dst + (int64_t)c * T.dld;
#pragma unroll 4
      for (int t = threadIdx.x; t < T.rows; t += 256) f32[d + t] = (float)arena[o + t];
    }
  } else {                                  // short columns: every thread busy
    const int n = T.rows * T.cols;
    for (int e = threadIdx.x; e < n; e += 256) {
      const int c = e / T.rows, t = e - c * T.rows;
      f32[T.dst + (int64_t)c * T.dld + t] = (float)arena[T.off + (int64_t)c * T.ld + t];
    }
  }
}
void launch_to_f32(const ConvTask* t, int n, const double* arena, float* f32, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(n), dim3(256), 0, s, t, arena, f32);
}

// FP64 copy of a block (the rows of an interior supernode's L^O_k inside its block, from
// the level pool to the factor's own storage): one task per block of at most 64 columns.
__global__ __launch_bounds__(256) void k_copy_f64(const ConvTask* __restrict__ tasks, double* __restrict__ arena) {
  const ConvTask T = tasks[blockIdx.x];
  const int n = T.rows * T.cols;
  for (int e = threadIdx.x; e < n; e += 256) {
    const int c = e / T.rows, t = e - c * T.rows;
    arena[T.dst + (int64_t)c * T.dld + t] = arena[T.off + (int64_t)c * T.ld + t];
  }
}
void launch_copy_f64(const ConvTask* t, int n, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy_f64, dim3(n), dim3(256), 0, s, t, arena);
}
void launch_part_apply(const PartApply* t, int n, const double* part, double* arena, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_part_apply, dim3(n), dim3(64), 0, s, t, part, arena);
}
void launch_gather_rows(const int64_t* tasks, int n, const int64_t* idx, const double* src,
                        double* dst, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gather_rows, dim3(n), dim3(256), 0, s, tasks, idx, src, dst);
}
void launch_coldot(const ColDotTask* t, int n, double* arena, const float* f32, const int64_t* gidx,
                   const int32_t* ilim, double* part, hipStream_t s) {
  if (n <= 0) return;
  if (f32) hipLaunchKernelGGL(k_coldot<float>, dim3(n), dim3(256), 0, s, t, arena, f32, gidx, ilim, part);
  else hipLaunchKernelGGL(k_coldot<double>, dim3(n), dim3(256), 0, s, t, arena, (const double*)arena, gidx, ilim, part);
}
void launch_row_gather(const int64_t* rows, const int64_t* ptr, const int64_t* contrib,
                       int64_t nrows, const double* part, double* y, hipStream_t s) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_row_gather, dim3(blocks_for(nrows)), dim3(256), 0, s, rows, ptr, contrib,
                       nrows, part, y);
}
void launch_sweep_fwd(const SweepTask* t, int n, int nt, int cpad, int lpad, double* arena,
                      const float* f32, int64_t a_y, int64_t a_w, int64_t a_zr, const int32_t* ilim,
                      const int64_t* pull_ptr, const int64_t* pull_idx, hipStream_t s) {
  if (n <= 0) return;
  const size_t lds = sizeof(double) * (size_t)(2 * cpad + lpad);
  if (f32)
    hipLaunchKernelGGL(k_sweep_fwd<float>, dim3(n), dim3(nt), lds, s, t, arena + a_y, arena + a_w,
                       arena + a_zr, f32, ilim, pull_ptr, pull_idx, cpad);
  else
    hipLaunchKernelGGL(k_sweep_fwd<double>, dim3(n), dim3(nt), lds, s, t, arena + a_y, arena + a_w,
                       arena + a_zr, (const double*)arena, ilim, pull_ptr, pull_idx, cpad);
}
void launch_sweep_bwd(const SweepTask* t, int n, int nt, int cpad, int lpad, int rmax, double* arena,
                      const float* f32, int64_t a_w, int64_t a_zz, const int32_t* ilim,
                      const int64_t* rows_idx, hipStream_t s) {
  if (n <= 0) return;
  const size_t lds = sizeof(double) * (size_t)(cpad + lpad + rmax);
  if (f32)
    hipLaunchKernelGGL(k_sweep_bwd<float>, dim3(n), dim3(nt), lds, s, t, arena + a_w, arena + a_zz,
                       f32, ilim, rows_idx, cpad, lpad);
  else
    hipLaunchKernelGGL(k_sweep_bwd<double>, dim3(n), dim3(nt), lds, s, t, arena + a_w, arena + a_zz,
                       (const double*)arena, ilim, rows_idx, cpad, lpad);
}
// Interior blocks (Sec. 5.1): a step of a solve with a block's own factor L^B =
// L(C^B, C^B), one workgroup (256 threads) per supernode, the supernodes of one
// elimination-tree level in one launch.  The block's off-diagonal rows beyond it are not
// stored; the sweeps reach them through A's coupling entries and these solves (eq.
// interiorBlockMult):
//  !FWD (levels from the block's root down): t_k = M_k (w_k - L^O_k(in)^T t_in), t = (L^B)^{-T} w;
//   FWD (levels up to the root): s_k = M_k^T (s_k - the pulled products of its
//        descendants), then L^O_k(in) s_k into the k's row slots of zr (pulled by the
//        supernodes owning those rows, in a fixed order); the root then takes w -= s over
//        the block's columns: s = (L^B)^{-1} s.
// Factor operands from `fac` (the FP64 arena or its FP32 copy), vectors FP64.
template <typename TF, bool FWD>
__global__ void __launch_bounds__(256) k_interior(const IntSn* __restrict__ sns, const TF* __restrict__ fac,
                                                  const int64_t* __restrict__ rows,
                                                  const int64_t* __restrict__ pull_ptr,
                                                  const int64_t* __restrict__ pull_idx, double* __restrict__ w,
                                                  double* __restrict__ t, double* __restrict__ zr) {
  __shared__ double in[kIntMaxC];
  __shared__ double out[kIntMaxC];
  __shared__ double red[4][64];
  const IntSn q = sns[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (!FWD) {
    // in = w_k - L^O_k(in)^T t_in: t over the rows gathered into LDS (`out`) a chunk at a
    // time, then a wave per column, its lanes down the rows
    for (int i = tid; i < q.c; i += 256) in[i] = w[q.first + i];
    for (int r0 = 0; r0 < q.rh; r0 += kIntMaxC) {
      const int nr = min(kIntMaxC, q.rh - r0);
      __syncthreads();
      for (int r = tid; r < nr; r += 256) out[r] = t[rows[q.rows + r0 + r]];
      __syncthreads();
      for (int col = wv; col < q.c; col += 4) {
        const TF* L = fac + q.lo + r0 + (int64_t)col * q.rh;
        double acc = 0.0;
#pragma unroll 4
        for (int r = lane; r < nr; r += 64) acc += (double)L[r] * out[r];
        acc = wave_sum(acc);
        if (lane == 0) in[col] -= acc;
      }
    }
    __syncthreads();
    // t_k = M_k in, 64 rows at a time: the lanes on the rows, the waves on every fourth
    // column (one coalesced column segment per step), then the four parts added
    for (int i0 = 0; i0 < q.c; i0 += 64) {
      const int i = i0 + lane;
      double acc = 0.0;
      if (i < q.c) {
#pragma unroll 4
        for (int m = i0 + wv; m < q.c; m += 4) acc += (double)fac[q.m + i + (int64_t)m * q.mld] * in[m];
      }
      red[wv][lane] = acc;      // (M upper: the terms m < i are zeros of M)
      __syncthreads();
      if (wv == 0 && i < q.c) t[q.first + i] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
      __syncthreads();
    }
  } else {
    // in = s_k minus the products its descendants in the block left in zr for its rows
    for (int i = tid; i < q.c; i += 256) {
      const int64_t row = q.first + i;
      double v = t[row];
      for (int64_t e = pull_ptr[row]; e < pull_ptr[row + 1]; ++e) v -= zr[pull_idx[e]];
      in[i] = v;
    }
    __syncthreads();
    // s_k = M_k^T in: a wave per column i of M, its lanes down the rows m <= i
    for (int i = wv; i < q.c; i += 4) {
      double acc = 0.0;
#pragma unroll 2
      for (int m = lane; m <= i; m += 64) acc += (double)fac[q.m + m + (int64_t)i * q.mld] * in[m];
      acc = wave_sum(acc);
      if (lane == 0) { out[i] = acc; t[q.first + i] = acc; }
    }
    __syncthreads();
    // its products for the rows inside the block, one slot per row of R_k
    for (int r = tid; r < q.rh; r += 256) {
      const TF* L = fac + q.lo + r;
      double acc = 0.0;
#pragma unroll 8
      for (int i = 0; i < q.c; ++i) acc += (double)L[(int64_t)i * q.rh] * out[i];
      zr[q.rows + r] = acc;
    }
    if (q.root) {
      __syncthreads();
      for (int64_t i = q.a + tid; i < q.b; i += 256) w[i] -= t[i];
    }
  }
}

void launch_interior(const IntSn* sns, int n, bool fwd, const double* arena, const float* f32,
                     const int64_t* rows, const int64_t* pull_ptr, const int64_t* pull_idx, double* w,
                     double* t, double* zr, hipStream_t s) {
  if (n <= 0) return;
  if (f32) {
    if (fwd) hipLaunchKernelGGL((k_interior<float, true>), dim3(n), dim3(256), 0, s, sns, f32, rows, pull_ptr, pull_idx, w, t, zr);
    else hipLaunchKernelGGL((k_interior<float, false>), dim3(n), dim3(256), 0, s, sns, f32, rows, pull_ptr, pull_idx, w, t, zr);
  } else {
    if (fwd) hipLaunchKernelGGL((k_interior<double, true>), dim3(n), dim3(256), 0, s, sns, arena, rows, pull_ptr, pull_idx, w, t, zr);
    else hipLaunchKernelGGL((k_interior<double, false>), dim3(n), dim3(256), 0, s, sns, arena, rows, pull_ptr, pull_idx, w, t, zr);
  }
}

// Coupling products with A over interior blocks: for target i,
// out[tgt[i]] (-)= sum_e vals[vidx[e]] vec[xidx[e]] over e in [ptr[i], ptr[i+1]) (in list
// order); `sub` subtracts from out, else it is assigned.  A thread per target.
__global__ void k_coupling(const int64_t* __restrict__ tgt, const int64_t* __restrict__ ptr,
                           const int64_t* __restrict__ vidx, const int64_t* __restrict__ xidx, int64_t n,
                           const double* __restrict__ vals, const double* __restrict__ vec,
                           double* __restrict__ out, int sub) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) acc += vals[vidx[e]] * vec[xidx[e]];
  const int64_t o = tgt[i];
  out[o] = sub ? out[o] - acc : acc;
}

void launch_coupling(const int64_t* tgt, const int64_t* ptr, const int64_t* vidx, const int64_t* xidx,
                     int64_t n, const double* vals, const double* vec, double* out, bool sub, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_coupling, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tgt, ptr, vidx, xidx, n,
                     vals, vec, out, sub ? 1 : 0);
}

void launch_gather_perm(int64_t n, const int64_t* perm, const double* src, double* dst, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gather_perm, dim3(blocks_for(n)), dim3(256), 0, s, n, perm, src, dst);
}
void launch_scatter_perm(int64_t n, const int64_t* perm, const double* src, double* dst, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_perm, dim3(blocks_for(n)), dim3(256), 0, s, n, perm, src, dst);
}
void launch_spmv_dot(const Chunk* c, int nc, const int64_t* rowptr, const int32_t* colind,
                     const double* vals, const double* p, double* Ap, double* partial, hipStream_t s) {
  if (nc > 0)
    hipLaunchKernelGGL(k_spmv_dot, dim3(nc), dim3(256), 0, s, c, rowptr, colind, vals, p, Ap, partial);
}
void launch_dot_partial(const Chunk* c, int nc, const double* a, const double* b, double* partial,
                        hipStream_t s) {
  if (nc > 0) hipLaunchKernelGGL(k_dot_partial, dim3(nc), dim3(256), 0, s, c, a, b, partial);
}
void launch_resid_partial(const Chunk* c, int nc, const double* b, const double* ax,
                          double* partial, hipStream_t s) {
  if (nc > 0) hipLaunchKernelGGL(k_resid_partial, dim3(nc), dim3(256), 0, s, c, b, ax, partial);
}
void launch_seg_sum(const int32_t* seg_ptr, int32_t nseg, const double* partial, double* out,
                    hipStream_t s) {
  if (nseg > 0) hipLaunchKernelGGL(k_seg_sum, dim3(nseg), dim3(256), 0, s, seg_ptr, nseg, partial, out);
}
void launch_seg_step(const int32_t* seg_ptr, int32_t nseg, const double* partial, const PcgScalars& sc,
                     double rtol, double* arena, int32_t* ints, int kind, hipStream_t s) {
  if (nseg > 0)
    hipLaunchKernelGGL(k_seg_step, dim3(nseg), dim3(256), 0, s, seg_ptr, partial, sc, rtol, arena, ints, kind);
}
void launch_pcg_xr(const Chunk* c, int nc, const PcgScalars& sc, double* arena, const int32_t* ints,
                   double* partial, hipStream_t s) {
  if (nc > 0) hipLaunchKernelGGL(k_pcg_xr, dim3(nc), dim3(256), 0, s, c, sc, arena, ints, partial);
}
void launch_pcg_p(const Chunk* c, int nc, const PcgScalars& sc, double* arena, const int32_t* ints,
                  int first, hipStream_t s) {
  if (nc > 0) hipLaunchKernelGGL(k_pcg_p, dim3(nc), dim3(256), 0, s, c, sc, arena, ints, first);
}
void launch_pcg_start(int32_t nseg, const PcgScalars& sc, double* arena, int32_t* ints, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_start, dim3((nseg + 255) / 256), dim3(256), 0, s, nseg, sc, arena, ints);
}
void launch_copy(int64_t n, const double* a, double* b, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(256), 0, s, n, a, b);
}
void launch_grad_values(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* lam,
                        const double* x, double* g, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_grad_values, dim3(blocks_for(n)), dim3(256), 0, s, n, rowptr, colind, lam, x, g);
}
void launch_grad_faces(int64_t nf, const int32_t* fi, const int32_t* fj, const double* lam,
                       const double* x, double* g, hipStream_t s) {
  if (nf > 0) hipLaunchKernelGGL(k_grad_faces, dim3(blocks_for(nf)), dim3(256), 0, s, nf, fi, fj, lam, x, g);
}


// Partial-sum blocks of the allocation-free preconditioner apply: a file-scope device
// array, one copy on every GPU the library runs on, held until the process ends.  In
// host code its name is not a device address; apply_scratch() looks the address up once
// per device (with that device current) and every later use goes through that pointer.
static __device__ __align__(256) double apply_scratch_buf[kApplyScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t apply_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(apply_scratch_buf));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace rsc
