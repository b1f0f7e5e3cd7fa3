// LDS-staged MFMA tile GEMM for gfx950 (all precisions, two tile sizes).
//
// One TM x TM output tile per workgroup: TM = 64 with 4 waves (each a 32 x 32 quarter
// as 2 x 2 MFMA blocks of 16 x 16) or TM = 128 with 8 waves (each a 32 x 64 strip as
// 2 x 4 blocks); wave w sits at row strip w / 2, column half w % 2.
// K advances in chunks of 32: the A and B chunks (TM x 32 each) are read from the FP64
// arena with coalesced loads whatever their layout (the contiguous dimension is mapped
// to consecutive threads), converted once to the matrix-core type and written to LDS;
// the next chunk's global loads are issued into registers before the current chunk's
// MFMAs.  The 128 tile halves the operand bytes per flop; the 64 tile gives four times
// as many workgroups for launches too small to fill the chip with 128 tiles.
//   kF64:    v_mfma_f64_16x16x4f64          (LDS tiles [k][i], FP64)
//   kF32:    v_mfma_f32_16x16x4f32          (LDS tiles [k][i], FP32)
//   kBF16x3: v_mfma_f32_16x16x32_bf16 x 3   (LDS tiles [i][k], hi and lo parts)
//   kBF16:   v_mfma_f32_16x16x32_bf16       (LDS tiles [i][k], hi part)
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "potrf_block.h"
#include "tasks.h"

namespace rsc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

enum StMode { sF64 = 0, sF32 = 1, sBF16x3 = 2, sBF16 = 3 };

constexpr int KC = 32;          // K chunk
constexpr int PADB = 40;        // row pitch (bf16) of [i][k] tiles: 80 bytes, 16-byte aligned

template <int MODE, int TM> struct Stage;

template <int TM> struct Stage<sF64, TM> {
  double a[KC][TM + 4], b[KC][TM + 4];
  __device__ void put_a(int i, int k, double v) { a[k][i] = v; }
  __device__ void put_b(int j, int k, double v) { b[k][j] = v; }
};
template <int TM> struct Stage<sF32, TM> {
  float a[KC][TM + 4], b[KC][TM + 4];
  __device__ void put_a(int i, int k, double v) { a[k][i] = (float)v; }
  __device__ void put_b(int j, int k, double v) { b[k][j] = (float)v; }
};
template <int TM> struct Stage<sBF16x3, TM> {
  __bf16 ah[TM][PADB], al[TM][PADB], bh[TM][PADB], bl[TM][PADB];
  __device__ void put_a(int i, int k, double v) {
    const float f = (float)v; const __bf16 h = (__bf16)f;
    ah[i][k] = h; al[i][k] = (__bf16)(f - (float)h);
  }
  __device__ void put_b(int j, int k, double v) {
    const float f = (float)v; const __bf16 h = (__bf16)f;
    bh[j][k] = h; bl[j][k] = (__bf16)(f - (float)h);
  }
};
template <int TM> struct Stage<sBF16, TM> {
  __bf16 ah[TM][PADB], bh[TM][PADB];
  __device__ void put_a(int i, int k, double v) { ah[i][k] = (__bf16)(float)v; }
  __device__ void put_b(int j, int k, double v) { bh[j][k] = (__bf16)(float)v; }
};

template <int MODE> struct Acc { typedef v4f T; };
template <> struct Acc<sF64> { typedef v4d T; };

// Global loads of one TM x 32 operand chunk by NT threads (TM * 32 / NT values per
// thread), coalesced along the operand's contiguous dimension.  Element (r, k) is at
// base + r * rs + k * ks, valid for r < rmax, k < kmax.
template <int TM, int NT>
struct ChunkLoader {
  static constexpr int NV = TM * 32 / NT, RP = TM / 64;
  double v[NV];
  __device__ static void pos(int u, bool rcont, int& r, int& k) {
    const int t = threadIdx.x;
    if (rcont) { r = (t & 63) + 64 * (u % RP); k = (t >> 6) + (NT / 64) * (u / RP); }
    else       { k = t & 31; r = (t >> 5) + (NT / 32) * u; }
  }
  __device__ void load(const double* base, int64_t rs, int64_t ks, int rmax, int kmax, int k0,
                       bool rcont) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      int r, k;
      pos(u, rcont, r, k);
      const int kk = k0 + k;
      v[u] = (r < rmax && kk < kmax) ? base[r * rs + (int64_t)kk * ks] : 0.0;
    }
  }
  template <class S>
  __device__ void store_a(S& st, bool rcont) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      int r, k;
      pos(u, rcont, r, k);
      st.put_a(r, k, v[u]);
    }
  }
  template <class S>
  __device__ void store_b(S& st, bool rcont) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      int r, k;
      pos(u, rcont, r, k);
      st.put_b(r, k, v[u]);
    }
  }
};

// Wave layout of a TM x TM tile: waves at row strips of RW rows and column halves.
template <int TM> struct Layout {
  static constexpr int NW = (TM == 128) ? 8 : 4;   // waves per workgroup
  static constexpr int NT = 64 * NW;               // threads
  static constexpr int RW = 2 * TM / NW;           // rows per wave strip (32)
  static constexpr int CW = TM / 2;                // columns per wave half
  static constexpr int BR = RW / 16, BC = CW / 16; // MFMA blocks per wave
};

template <int MODE, int TM>
__device__ __forceinline__ void mma_chunk(Stage<MODE, TM>& st,
                                          typename Acc<MODE>::T (&acc)[Layout<TM>::BR][Layout<TM>::BC],
                                          int wr, int wc, int lane) {
  using Ly = Layout<TM>;
  constexpr int BR = Ly::BR, BC = Ly::BC;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = wr * Ly::RW, c0 = wc * Ly::CW;
  if constexpr (MODE == sF64 || MODE == sF32) {
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      if constexpr (MODE == sF64) {
        double av[BR], bv[BC];
#pragma unroll
        for (int b = 0; b < BR; ++b) av[b] = st.a[ks + lk][r0 + b * 16 + li];
#pragma unroll
        for (int b = 0; b < BC; ++b) bv[b] = st.b[ks + lk][c0 + b * 16 + li];
#pragma unroll
        for (int x = 0; x < BR; ++x)
#pragma unroll
          for (int y = 0; y < BC; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
      } else {
        float av[BR], bv[BC];
#pragma unroll
        for (int b = 0; b < BR; ++b) av[b] = st.a[ks + lk][r0 + b * 16 + li];
#pragma unroll
        for (int b = 0; b < BC; ++b) bv[b] = st.b[ks + lk][c0 + b * 16 + li];
#pragma unroll
        for (int x = 0; x < BR; ++x)
#pragma unroll
          for (int y = 0; y < BC; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[x], bv[y], acc[x][y], 0, 0, 0);
      }
    }
  } else {
    v8bf ah[BR], bh[BC];
#pragma unroll
    for (int b = 0; b < BR; ++b) ah[b] = *reinterpret_cast<const v8bf*>(&st.ah[r0 + b * 16 + li][8 * lk]);
#pragma unroll
    for (int b = 0; b < BC; ++b) bh[b] = *reinterpret_cast<const v8bf*>(&st.bh[c0 + b * 16 + li][8 * lk]);
    if constexpr (MODE == sBF16x3) {
      v8bf al[BR], bl[BC];
#pragma unroll
      for (int b = 0; b < BR; ++b) al[b] = *reinterpret_cast<const v8bf*>(&st.al[r0 + b * 16 + li][8 * lk]);
#pragma unroll
      for (int b = 0; b < BC; ++b) bl[b] = *reinterpret_cast<const v8bf*>(&st.bl[c0 + b * 16 + li][8 * lk]);
#pragma unroll
      for (int x = 0; x < BR; ++x)
#pragma unroll
        for (int y = 0; y < BC; ++y) {
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], bh[y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bl[y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bh[y], acc[x][y], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int x = 0; x < BR; ++x)
#pragma unroll
        for (int y = 0; y < BC; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bh[y], acc[x][y], 0, 0, 0);
    }
  }
}

// Result element (i, j) of block (x, y) held by this lane as element e.
template <int MODE>
__device__ __forceinline__ void res_pos(int lane, int e, int& i, int& j) {
  if constexpr (MODE == sF64) i = (lane >> 4) + 4 * e;    // f64: row lane/16 + 4e
  else i = 4 * (lane >> 4) + e;                           // f32 accumulators: row 4 (lane/16) + e
  j = lane & 15;
}

// Accumulates P = A(r0.., :) B(c0.., :)^T for the workgroup's TM x TM tile over k < K.
template <int MODE, int TM>
__device__ void tile_product(Stage<MODE, TM>& st,
                             typename Acc<MODE>::T (&acc)[Layout<TM>::BR][Layout<TM>::BC],
                             const double* A, int64_t ars, int64_t aks, int amax,
                             const double* B, int64_t brs, int64_t bks, int bmax, int K) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool acont = (ars == 1), bcont = (brs == 1);
  ChunkLoader<TM, Layout<TM>::NT> la, lb;
  if (K > 0) {
    la.load(A, ars, aks, amax, K, 0, acont);
    lb.load(B, brs, bks, bmax, K, 0, bcont);
  }
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();                       // previous chunk's MFMAs done with the LDS tiles
    la.store_a(st, acont);
    lb.store_b(st, bcont);
    __syncthreads();
    if (k0 + KC < K) {                     // next chunk in flight during the MFMAs
      la.load(A, ars, aks, amax, K, k0 + KC, acont);
      lb.load(B, brs, bks, bmax, K, k0 + KC, bcont);
    }
    mma_chunk<MODE, TM>(st, acc, wr, wc, lane);
  }
}

// Epilogue slab: 64 columns of the tile as accumulator values, column-major with an
// odd pitch; it reuses the operand stage's LDS.
template <int MODE> struct AccElem { typedef float T; };
template <> struct AccElem<sF64> { typedef double T; };
template <int TM> constexpr int kSlabPitch = TM + 1;
template <int MODE, int TM>
constexpr size_t kGemmSmem = sizeof(Stage<MODE, TM>) > 64 * kSlabPitch<TM> * sizeof(typename AccElem<MODE>::T)
                                 ? sizeof(Stage<MODE, TM>)
                                 : 64 * kSlabPitch<TM> * sizeof(typename AccElem<MODE>::T);

// POST (FP64, 64 tiles): a task with potrf1 > 0 holds a panel's next diagonal block; its
// workgroup factors the block (potrf_block) once the tile is stored, so the POTRF of the
// next panel step runs inside this launch instead of after it.
template <int MODE, int TM, bool POST>
constexpr size_t kStagedSmem = (POST && kPotrfSmem > kGemmSmem<MODE, TM>) ? kPotrfSmem : kGemmSmem<MODE, TM>;

template <int MODE, int TM, bool POST>
__global__ __launch_bounds__(Layout<TM>::NT, (TM == 64 && MODE == sF64) ? (POST ? 2 : 3) : 1) void k_gemm_staged(const GemmTask* __restrict__ tasks,
                                                               double* __restrict__ arena,
                                                               const int32_t* __restrict__ ilim,
                                                               double* __restrict__ part,
                                                               const PotrfTask* __restrict__ ptasks,
                                                               int32_t* __restrict__ status) {
  using Ly = Layout<TM>;
  using AE = typename AccElem<MODE>::T;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kStagedSmem<MODE, TM, POST>];
  Stage<MODE, TM>& st = *reinterpret_cast<Stage<MODE, TM>*>(smem);
  const GemmTask T = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int n = T.nlim >= 0 ? min(T.n, ilim[T.nlim]) : T.n;
  const int K = T.klim >= 0 ? min(T.k, ilim[T.klim]) : T.k;
  if (T.j0 >= n) return;
  typename Acc<MODE>::T acc[Ly::BR][Ly::BC];
#pragma unroll
  for (int x = 0; x < Ly::BR; ++x)
#pragma unroll
    for (int y = 0; y < Ly::BC; ++y)
      for (int e = 0; e < 4; ++e) acc[x][y][e] = 0;
  int kb = 0, ke = K;
  if (T.kz > 1) {                          // K slice ks of kz (chunk aligned)
    const int per = ((K + T.kz - 1) / T.kz + KC - 1) / KC * KC;
    kb = min(K, T.ks * per);
    ke = min(K, kb + per);
  }
  const double* A = arena + T.a + (int64_t)T.i0 * T.ais + (int64_t)kb * T.aks;
  const double* B = arena + T.b + (int64_t)T.j0 * T.bjs + (int64_t)kb * T.bks;
  tile_product<MODE, TM>(st, acc, A, T.ais, T.aks, T.m - T.i0, B, T.bjs, T.bks, n - T.j0, ke - kb);
  // C = alpha P (+ beta D), 64 columns at a time through LDS so that C and D are read
  // and written one contiguous column (up to TM rows) per wave instruction
  AE* slab = reinterpret_cast<AE*>(smem);
  double* C = arena + T.c;
  const int mrows = min(TM, T.m - T.i0);
  for (int s0 = 0; s0 < TM; s0 += 64) {
    __syncthreads();                       // A/B may alias C; the stage (or the last slab) is free
    if (wc * Ly::CW < s0 + 64 && wc * Ly::CW + Ly::CW > s0) {
#pragma unroll
      for (int x = 0; x < Ly::BR; ++x)
#pragma unroll
        for (int y = 0; y < Ly::BC; ++y)
          for (int e = 0; e < 4; ++e) {
            int ii, jj;
            res_pos<MODE>(lane, e, ii, jj);
            const int i = wr * Ly::RW + x * 16 + ii;
            const int j = wc * Ly::CW + y * 16 + jj - s0;
            slab[j * kSlabPitch<TM> + i] = acc[x][y][e];
          }
    }
    __syncthreads();
    if (T.kz > 1) {                        // a K slice: the raw partial tile (no alpha, beta)
      for (int idx = threadIdx.x; idx < TM * 64; idx += Ly::NT) {
        const int i = idx % TM, j = idx / TM;
        part[T.part + i + (int64_t)(s0 + j) * TM] = (double)slab[j * kSlabPitch<TM> + i];
      }
      continue;
    }
    const int ncol = min(64, n - T.j0 - s0);
    // symmetric C: elements on or below the diagonal directly, their mirror images below
    const int dj = T.j0 + s0 - T.i0;         // global column - row = j - i + dj
    for (int idx = threadIdx.x; idx < TM * 64; idx += Ly::NT) {
      const int i = idx % TM, j = idx / TM;
      if (i < mrows && j < ncol && !(T.sym && j + dj > i)) {
        const int64_t o = (T.i0 + i) + (int64_t)(T.j0 + s0 + j) * T.ldc;
        const double v = T.alpha * (double)slab[j * kSlabPitch<TM> + i];
        if (T.beta == 0.0) C[o] = v;
        else C[o] = v + T.beta * ((T.d >= 0) ? arena[T.d + o] : C[o]);
      }
    }
    if (T.sym) {
      // the transpose, rows of C along consecutive threads; D is symmetric too
      __syncthreads();                     // the direct writes (which D may not alias) are done
      for (int idx = threadIdx.x; idx < TM * 64; idx += Ly::NT) {
        const int j = idx % 64, i = idx / 64;
        if (i < mrows && j < ncol && j + dj < i) {
          const int64_t o = (T.j0 + s0 + j) + (int64_t)(T.i0 + i) * T.ldc;
          const int64_t od = (T.i0 + i) + (int64_t)(T.j0 + s0 + j) * T.ldc;
          const double v = T.alpha * (double)slab[j * kSlabPitch<TM> + i];
          if (T.beta == 0.0) C[o] = v;
          else C[o] = v + T.beta * ((T.d >= 0) ? arena[T.d + od] : C[od]);
        }
      }
    }
  }
  if constexpr (POST) {
    if (T.potrf1 > 0) {
      __syncthreads();                     // the tile's stores, then its factorization
      double* blk = reinterpret_cast<double*>(smem);
      potrf_block<64>(ptasks[T.potrf1 - 1], arena, status, blk, blk + 64 * kPitch);
    }
  }
}

// Sum of the kz (<= 8) K-slice partial tiles of one output tile, then the same store as a
// whole-K product: C = alpha S (+ beta D), mirrored for symmetric C.  1024 threads, four
// elements each; every element's kz partials are loaded together and added in slice
// order (the missing slices as exact zeros).
template <int TM>
__global__ __launch_bounds__(1024) void k_gemm_reduce(const GemmTask* __restrict__ tasks,
                                                      double* __restrict__ arena,
                                                      const int32_t* __restrict__ ilim,
                                                      const double* __restrict__ part) {
  const GemmTask T = tasks[blockIdx.x];
  const int n = T.nlim >= 0 ? min(T.n, ilim[T.nlim]) : T.n;
  if (T.j0 >= n) return;
  double* C = arena + T.c;
  const int mrows = min(TM, T.m - T.i0), ncol = min(TM, n - T.j0);
  const int dj = T.j0 - T.i0;
  const int64_t tt = (int64_t)TM * TM;
  auto sum = [&](int i, int j) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = q < T.kz ? part[T.part + q * tt + i + (int64_t)j * TM] : 0.0;
    double acc = v[0];
#pragma unroll
    for (int q = 1; q < 8; ++q) acc += v[q];
    return acc;
  };
  for (int idx = threadIdx.x; idx < TM * TM; idx += 1024) {
    const int i = idx % TM, j = idx / TM;
    if (i < mrows && j < ncol && !(T.sym && j + dj > i)) {
      const int64_t o = (T.i0 + i) + (int64_t)(T.j0 + j) * T.ldc;
      const double v = T.alpha * sum(i, j);
      if (T.beta == 0.0) C[o] = v;
      else C[o] = v + T.beta * ((T.d >= 0) ? arena[T.d + o] : C[o]);
    }
  }
  if (T.sym) {
    __syncthreads();                       // the direct writes are done
    for (int idx = threadIdx.x; idx < TM * TM; idx += 1024) {
      const int j = idx % TM, i = idx / TM;
      if (i < mrows && j < ncol && j + dj < i) {
        const int64_t o = (T.j0 + j) + (int64_t)(T.i0 + i) * T.ldc;
        const int64_t od = (T.i0 + i) + (int64_t)(T.j0 + j) * T.ldc;
        const double v = T.alpha * sum(i, j);
        if (T.beta == 0.0) C[o] = v;
        else C[o] = v + T.beta * ((T.d >= 0) ? arena[T.d + od] : C[od]);
      }
    }
  }
}

// ------------------------------------------------------------------ Schur update
//
// Operands of the Schur update (L^O_k, or V_k of a compressed supernode) are read from a
// compact row-major copy written once when the operand is final: row t holds the
// operand's K columns in chunks of 32 -- FP64 values (sF64, 256 bytes), FP32 values
// (sF32, one 128-byte line), or 32 BF16 high parts followed by the 32 low parts
// (sBF16x3, one line) -- zero beyond the operand's kept columns.  A lane then takes its
// 8 consecutive k values of a row with one, two or four 16-byte loads.

// One 64-row block of one operand per workgroup: the 64 x 32 chunk is read column by
// column (coalesced), transposed through LDS and written as rows.
template <int MODE>
__global__ __launch_bounds__(256) void k_compact_rows(const CompactTask* __restrict__ tasks,
                                                      const double* __restrict__ arena,
                                                      const int32_t* __restrict__ ilim,
                                                      double* __restrict__ xc, float* __restrict__ f32) {
  __shared__ double t[KC][65];
  const CompactTask T = tasks[blockIdx.x];
  const int K = T.kdim >= 0 ? T.kdim : ilim[-1 - T.kdim];
  const int tid = threadIdx.x;
  const double* src = arena + T.src;
  const int r = tid >> 2, kq = 8 * (tid & 3);     // writer: row r, values kq .. kq + 7
  for (int c0 = 0; c0 < T.kp; c0 += KC) {
    __syncthreads();
    if (c0 < K) {                          // eight loads in flight together (clamped addresses)
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = tid + 256 * u, rr = idx & 63, k = idx >> 6;
        v[u] = src[min(rr, T.nrows - 1) + (int64_t)min(c0 + k, K - 1) * T.ld];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = tid + 256 * u, rr = idx & 63, k = idx >> 6;
        const bool in = rr < T.nrows && c0 + k < K;
        t[k][rr] = in ? v[u] : 0.0;
        // the sweeps' FP32 copy of the same block, column-major at the arena's offsets
        if (f32 && in && T.f32 >= 0) f32[T.f32 + rr + (int64_t)(c0 + k) * T.ld] = (float)v[u];
      }
    } else {
      for (int idx = tid; idx < 64 * KC; idx += 256) t[idx >> 6][idx & 63] = 0.0;
    }
    __syncthreads();
    if (r < T.nrows) {
      if constexpr (MODE == sBF16x3) {
        __bf16* row = reinterpret_cast<__bf16*>(xc + T.dst) + (int64_t)r * 2 * T.kp + 2 * c0;
        v8bf hi, lo;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float f = (float)t[kq + u][r];
          const __bf16 h = (__bf16)f;
          hi[u] = h; lo[u] = (__bf16)(f - (float)h);
        }
        *reinterpret_cast<v8bf*>(row + kq) = hi;
        *reinterpret_cast<v8bf*>(row + KC + kq) = lo;
      } else if constexpr (MODE == sF64) {
        double* row = xc + T.dst + (int64_t)r * T.kp + c0 + kq;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double2 d;
          d.x = t[kq + 2 * u][r];
          d.y = t[kq + 2 * u + 1][r];
          *reinterpret_cast<double2*>(row + 2 * u) = d;
        }
      } else {
        float* row = reinterpret_cast<float*>(xc + T.dst) + (int64_t)r * T.kp + c0;
        v4f a, b;
#pragma unroll
        for (int u = 0; u < 4; ++u) { a[u] = (float)t[kq + u][r]; b[u] = (float)t[kq + 4 + u][r]; }
        *reinterpret_cast<v4f*>(row + kq) = a;
        *reinterpret_cast<v4f*>(row + kq + 4) = b;
      }
    }
  }
}

// A wave's share of one entry: rows [r0, r0 + nr) and [c0, c0 + nc) (each <= 32) of the
// entry's operand, k < K.
struct WaveWork {
  UpdEntry E;
  int r0, nr, c0, nc, K;
};

// Operand registers of one 32-column chunk of a wave's product.  Lane (li, lk) holds k
// values 8 lk .. 8 lk + 7 of rows li and 16 + li (one bf16 MFMA takes them at once; for
// the 16x16x4 FP32 / FP64 MFMAs, step u takes k = 8 lk + u, the same permutation of k on
// both operands).
template <int MODE> struct WaveOps;
template <> struct WaveOps<sF64> { double a[2][8], b[2][8]; };
template <> struct WaveOps<sF32> { v4f a[2][2], b[2][2]; };
template <> struct WaveOps<sBF16x3> { v8bf ah[2], al[2], bh[2], bl[2]; };

// Vector-memory instructions issued by one wave_load.
template <int MODE> constexpr int kWaveLoads = MODE == sF64 ? 16 : 8;

// Waits until at most N vector-memory loads of the wave are outstanding (expcnt and
// lgkmcnt fields at their maxima, so only vmcnt is waited on).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N < 64, "vmcnt field");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x70 | 0xF00);
}

// Relative-map entries (target positions) of a wave's result rows and columns.
struct WaveMaps {
  int r[2][4], c[2];
};

// Rows past nr (nc) are loaded from row nr - 1 (nc - 1): in-bounds, unconditional loads
// that need no select before their use, and whose products land only in result rows or
// columns that the scatter skips.  Columns past K within the chunk are zero in the copy.
// Operand rows ia .. ia + na - 1 and ib .. ib + nb - 1 of the compact copy at double
// offset xo (row length ldx elements), columns k0 .. k0 + 31.
template <int MODE>
__device__ __forceinline__ void wave_load(WaveOps<MODE>& o, const double* __restrict__ xbase, int64_t xo, int ldx,
                                          int ia, int na, int ib, int nb, int k0, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int i = 16 * x + li;
    const int64_t ra = (int64_t)(ia + min(i, na - 1)) * ldx;
    const int64_t rb = (int64_t)(ib + min(i, nb - 1)) * ldx;
    if constexpr (MODE == sF64) {
      const double* pa = xbase + xo + ra + k0 + 8 * lk;
      const double* pb = xbase + xo + rb + k0 + 8 * lk;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const double2 za = *reinterpret_cast<const double2*>(pa + 2 * h);
        const double2 zb = *reinterpret_cast<const double2*>(pb + 2 * h);
        o.a[x][2 * h] = za.x; o.a[x][2 * h + 1] = za.y;
        o.b[x][2 * h] = zb.x; o.b[x][2 * h + 1] = zb.y;
      }
    } else if constexpr (MODE == sF32) {
      const float* X = reinterpret_cast<const float*>(xbase + xo);
      const float* pa = X + ra + k0 + 8 * lk;
      const float* pb = X + rb + k0 + 8 * lk;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        o.a[x][h] = *reinterpret_cast<const v4f*>(pa + 4 * h);
        o.b[x][h] = *reinterpret_cast<const v4f*>(pb + 4 * h);
      }
    } else {
      const __bf16* X = reinterpret_cast<const __bf16*>(xbase + xo);
      const __bf16* pa = X + ra + 2 * k0 + 8 * lk;
      const __bf16* pb = X + rb + 2 * k0 + 8 * lk;
      o.ah[x] = *reinterpret_cast<const v8bf*>(pa);
      o.al[x] = *reinterpret_cast<const v8bf*>(pa + KC);
      o.bh[x] = *reinterpret_cast<const v8bf*>(pb);
      o.bl[x] = *reinterpret_cast<const v8bf*>(pb + KC);
    }
  }
}

template <int MODE>
__device__ __forceinline__ void wave_mma(typename Acc<MODE>::T (&acc)[2][2], const WaveOps<MODE>& o, int br,
                                         int bc) {
  if constexpr (MODE == sF64) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          if (x < br && y < bc) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[x][u], o.b[y][u], acc[x][y], 0, 0, 0);
  } else if constexpr (MODE == sF32) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          if (x < br && y < bc)
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[x][u >> 2][u & 3], o.b[y][u >> 2][u & 3], acc[x][y], 0, 0, 0);
  } else {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        if (x < br && y < bc) {
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.al[x], o.bh[y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.ah[x], o.bl[y], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.ah[x], o.bh[y], acc[x][y], 0, 0, 0);
        }
  }
}

// Raw relative-map entries of a wave's result rows and columns (clamped like wave_load).
template <int MODE>
__device__ __forceinline__ void wave_maps(const int32_t* __restrict__ relmap, const WaveWork& W, int lane,
                                          WaveMaps& m) {
  const int32_t* rm = relmap + W.E.map;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int ii, jj;
      res_pos<MODE>(lane, e, ii, jj);
      m.r[x][e] = rm[W.E.a + W.r0 + min(16 * x + ii, W.nr - 1)];
    }
#pragma unroll
  for (int y = 0; y < 2; ++y) m.c[y] = rm[W.E.c + W.c0 + min(16 * y + (lane & 15), W.nc - 1)];
}

// Subtracts a wave's block from the LDS tile at the tile-local target positions kept in
// the wave's LDS slot: one byte each, rows r[x][0..3] in word x and columns c[0], c[1] in
// word 2 of lane l (word k at slot[64 k + l]).
template <int MODE>
__device__ __forceinline__ void wave_scatter(double* tile, const typename Acc<MODE>::T (&acc)[2][2],
                                             const uint32_t* slot, int nr, int nc, int lane) {
  int pr[2][4], pc[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const uint32_t v = slot[64 * x + lane];
#pragma unroll
    for (int e = 0; e < 4; ++e) pr[x][e] = (v >> (8 * e)) & 255;
  }
  {
    const uint32_t v = slot[128 + lane];
    pc[0] = v & 255;
    pc[1] = (v >> 8) & 255;
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int ii, jj;
        res_pos<MODE>(lane, e, ii, jj);
        if (16 * x + ii < nr && 16 * y + jj < nc) tile[pr[x][e] + 65 * pc[y]] -= (double)acc[x][y][e];
      }
}

// Schur-complement update of one 64 x 64 target tile per workgroup (the tile stays in
// LDS).  The tile's entries form groups: each entry of [e0, es) (wider than 32 in some
// direction) is one group, whose four 32 x 32 quadrants go to the four waves (their
// target positions are disjoint); the entries of [es, e1) (at most 32 x 32) form groups
// of four, one per wave, subtracted in wave order one barrier apart.  Every wave passes
// the barriers of all groups in order.  Between them each wave streams its own sequence
// of (entry, 32-column chunk) steps from registers: a step issues the loads of the next
// step -- the next chunk, or the first chunk and the target positions of the wave's next
// entry -- before the MFMAs of its own chunk, so the loads overlap the products, the
// scatters and the barriers.  The two operand register sets alternate by step (the loop
// body holds two steps, so no set is copied while its loads are in flight), and the
// target positions move to an LDS slot of the wave once they have arrived (as bytes,
// so that four workgroups fit in a compute unit's LDS).  The summation order is fixed
// by the entry list, so the result does not depend on scheduling.
template <int MODE>
__global__ __launch_bounds__(256) void k_update_waves(const UpdTile* __restrict__ tiles,
                                                      const UpdEntry* __restrict__ ents,
                                                      const int32_t* __restrict__ relmap,
                                                      double* __restrict__ arena,
                                                      const double* __restrict__ xbase,
                                                      const int32_t* __restrict__ ilim) {
  __shared__ double tile[64 * 65];
  __shared__ uint32_t maps[4][3 * 64];
  const UpdTile T = tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  uint32_t* const slot = maps[w];
  double* P = arena + T.panel;
  {
    // all sixteen loads in flight together (addresses clamped into the tile), then LDS
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = tid + 256 * u, r = idx & 63, c = idx >> 6;
      t[u] = P[(T.row0 + min(r, T.nrows - 1)) + (int64_t)(T.col0 + min(c, T.ncols - 1)) * T.ld];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = tid + 256 * u, r = idx & 63, c = idx >> 6;
      tile[r + 65 * c] = (r < T.nrows && c < T.ncols) ? t[u] : 0.0;
    }
  }
  const int GL = T.es - T.e0;                     // groups of one large entry
  const int G = GL + (T.e1 - T.es + 3) / 4;       // then groups of four small entries
  // this wave's first group at or after g with a non-empty share (G if none), in W
  auto next_work = [&](int g, WaveWork& W) __attribute__((always_inline)) -> int {
    for (; g < G; ++g) {
      int e;
      if (g < GL) {
        e = T.e0 + g; W.r0 = 32 * (w >> 1); W.c0 = 32 * (w & 1);
      } else {
        e = T.es + 4 * (g - GL) + w; W.r0 = 0; W.c0 = 0;
        if (e >= T.e1) return G;
      }
      W.E = ents[e];
      W.nr = min(32, W.E.b - W.E.a - W.r0);
      W.nc = min(32, W.E.d - W.E.c - W.c0);
      W.K = W.E.kdim >= 0 ? W.E.kdim : ilim[-1 - W.E.kdim];
      if (((W.nr - 1) | (W.nc - 1) | (W.K - 1)) >= 0) return g;   // all three positive
    }
    return G;
  };
  typename Acc<MODE>::T acc[2][2];
  // the barriers of groups [g0, g1), scattering this wave's block in group `own`
  auto groups = [&](int g0, int g1, int own, const WaveWork& W) __attribute__((always_inline)) {
    for (int g = g0; g < g1; ++g) {
      if (g < GL) {
        if (g == own) wave_scatter<MODE>(tile, acc, slot, W.nr, W.nc, lane);
        __syncthreads();
      } else {
        for (int t = 0; t < 4; ++t) {
          if (w == t && g == own) wave_scatter<MODE>(tile, acc, slot, W.nr, W.nc, lane);
          __syncthreads();
        }
      }
    }
  };
  WaveOps<MODE> o0, o1;
  WaveMaps mn;                 // target positions of the next entry, in flight
  WaveWork W, Wn;
  int gn = next_work(0, Wn);
  if (gn < G) {
    wave_load<MODE>(o0, xbase, Wn.E.x, Wn.E.ldx, Wn.E.a + Wn.r0, Wn.nr, Wn.E.c + Wn.c0, Wn.nc, 0, lane);
    wave_maps<MODE>(relmap, Wn, lane, mn);
  }
  __syncthreads();             // the tile is in LDS
  groups(0, gn, -1, Wn);
  int gw = gn, k0 = 0;
  W = Wn;
  // one step on the chunk in `cur`; returns true when the wave has no further work
  auto step = [&](WaveOps<MODE>& cur, WaveOps<MODE>& nxt) __attribute__((always_inline)) -> bool {
    const bool last = k0 + KC >= W.K;
    if (last) gn = next_work(gw + 1, Wn);
    // the loads themselves are unconditional (with no work left, the current chunk is
    // read again), so that every path issues the same loads and the waits before the
    // MFMAs count only the older ones
    {
      const bool same = !last || gn >= G;
      wave_load<MODE>(nxt, xbase, same ? W.E.x : Wn.E.x, same ? W.E.ldx : Wn.E.ldx,
                      same ? W.E.a + W.r0 : Wn.E.a + Wn.r0, same ? W.nr : Wn.nr,
                      same ? W.E.c + W.c0 : Wn.E.c + Wn.c0, same ? W.nc : Wn.nc,
                      last ? (gn < G ? 0 : k0) : k0 + KC, lane);
    }
    if (k0 == 0) {             // this entry's target positions have arrived: park them
      // tile-local positions lie in [0, 64): one byte each
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        uint32_t v = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) v |= (uint32_t)(mn.r[x][e] - T.row0) << (8 * e);
        slot[64 * x + lane] = v;
      }
      slot[128 + lane] = (uint32_t)(mn.c[0] - T.col0) | ((uint32_t)(mn.c[1] - T.col0) << 8);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[x][y][e] = 0;
    }
    const bool maps_now = last && gn < G;
    if (maps_now) wave_maps<MODE>(relmap, Wn, lane, mn);
    wave_mma<MODE>(acc, cur, (W.nr + 15) >> 4, (W.nc + 15) >> 4);
    // every load older than this step's has arrived, including those of operand blocks
    // the MFMAs skipped: stated here so that no later register reuse waits on them
    if (maps_now) wait_vmcnt<kWaveLoads<MODE> + 10>(); else wait_vmcnt<kWaveLoads<MODE>>();
    if (!last) {
      k0 += KC;
      return false;
    }
    groups(gw, gn, gw, W);
    if (gn >= G) {             // the wave is done; its last (repeated) loads are drained
      wait_vmcnt<0>();         // here, so no wait on them is merged into the loop
      return true;
    }
    W = Wn; gw = gn; k0 = 0;
    return false;
  };
  if (gn < G) {
    while (true) {
      if (step(o0, o1)) break;
      if (step(o1, o0)) break;
    }
  }
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    if (r < T.nrows && c < T.ncols) P[(T.row0 + r) + (int64_t)(T.col0 + c) * T.ld] = tile[r + 65 * c];
  }
}

template <int TM>
static void launch_gemm_tm(int mode, const GemmTask* t, int n, double* arena, const int32_t* ilim,
                           double* part, hipStream_t s) {
  const PotrfTask* np = nullptr;
  int32_t* ns = nullptr;
  switch (mode) {
    case sF64: hipLaunchKernelGGL((k_gemm_staged<sF64, TM, false>), dim3(n), dim3(Layout<TM>::NT), 0, s, t, arena, ilim, part, np, ns); break;
    case sF32: hipLaunchKernelGGL((k_gemm_staged<sF32, TM, false>), dim3(n), dim3(Layout<TM>::NT), 0, s, t, arena, ilim, part, np, ns); break;
    case sBF16x3: hipLaunchKernelGGL((k_gemm_staged<sBF16x3, TM, false>), dim3(n), dim3(Layout<TM>::NT), 0, s, t, arena, ilim, part, np, ns); break;
    default: hipLaunchKernelGGL((k_gemm_staged<sBF16, TM, false>), dim3(n), dim3(Layout<TM>::NT), 0, s, t, arena, ilim, part, np, ns); break;
  }
}

void launch_gemm_staged(int mode, int tile, const GemmTask* t, int n, double* arena,
                        const int32_t* ilim, double* part, const PotrfTask* ptasks, int32_t* status,
                        hipStream_t s) {
  if (n <= 0) return;
  if (ptasks && mode == sF64 && tile == 64)
    hipLaunchKernelGGL((k_gemm_staged<sF64, 64, true>), dim3(n), dim3(Layout<64>::NT), 0, s, t, arena, ilim,
                       part, ptasks, status);
  else if (tile == 128) launch_gemm_tm<128>(mode, t, n, arena, ilim, part, s);
  else launch_gemm_tm<64>(mode, t, n, arena, ilim, part, s);
}

void launch_gemm_reduce(int tile, const GemmTask* t, int n, double* arena, const int32_t* ilim,
                        const double* part, hipStream_t s) {
  if (n <= 0) return;
  if (tile == 128) hipLaunchKernelGGL(k_gemm_reduce<128>, dim3(n), dim3(1024), 0, s, t, arena, ilim, part);
  else hipLaunchKernelGGL(k_gemm_reduce<64>, dim3(n), dim3(1024), 0, s, t, arena, ilim, part);
}

void launch_update_waves(int mode, const UpdTile* t, int n, const UpdEntry* e, const int32_t* relmap,
                         double* arena, const double* xbase, const int32_t* ilim, hipStream_t s) {
  if (n <= 0) return;
  switch (mode) {
    case sF64: hipLaunchKernelGGL(k_update_waves<sF64>, dim3(n), dim3(256), 0, s, t, e, relmap, arena, xbase, ilim); break;
    case sF32: hipLaunchKernelGGL(k_update_waves<sF32>, dim3(n), dim3(256), 0, s, t, e, relmap, arena, xbase, ilim); break;
    default: hipLaunchKernelGGL(k_update_waves<sBF16x3>, dim3(n), dim3(256), 0, s, t, e, relmap, arena, xbase, ilim); break;
  }
}

void launch_compact_rows(int mode, const CompactTask* t, int n, const double* arena, const int32_t* ilim,
                         double* xc, float* f32, hipStream_t s) {
  if (n <= 0) return;
  if (mode == sF64) hipLaunchKernelGGL(k_compact_rows<sF64>, dim3(n), dim3(256), 0, s, t, arena, ilim, xc, f32);
  else if (mode == sF32) hipLaunchKernelGGL(k_compact_rows<sF32>, dim3(n), dim3(256), 0, s, t, arena, ilim, xc, f32);
  else hipLaunchKernelGGL(k_compact_rows<sBF16x3>, dim3(n), dim3(256), 0, s, t, arena, ilim, xc, f32);
}

}  // namespace rsc
