// gfx950 kernels of the mixed-precision form: the Schur-update, TRSM and sampling
// products with low-precision matrix-core operands and FP32 accumulation, results
// added into FP64 storage.  Operands are read from the FP64 arena and rounded in
// registers (round to nearest even):
//   kF32:    v_mfma_f32_16x16x4f32 on FP32 operands;
//   kBF16x3: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); three
//            v_mfma_f32_16x16x32_bf16 products hi*hi + hi*lo + lo*hi (about 16 bits);
//   kBF16:   one v_mfma_f32_16x16x32_bf16 product (sampling only).
// Result layout of both FP32-accumulating MFMAs: D(i,j) in lane j + 16 (i / 4),
// element i mod 4.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "tasks.h"

namespace rsc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

enum LpMode { kF32 = 1, kBF16x3 = 2, kBF16 = 3 };

__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const float f = (float)x;
  hi = (__bf16)f;
  lo = (__bf16)(f - (float)hi);
}

// acc[x][y] += A-block(x) * B-block(y)^T over k in [0, K) for one wave's 32x32 quarter.
// fa(r, k) / fb(r, k) return the FP64 operand (0 outside the valid range).
template <int MODE, class FA, class FB>
__device__ __forceinline__ void lp_block(v4f (&acc)[2][2], int K, int lane, FA fa, FB fb) {
  const int li = lane & 15, lk = lane >> 4;
  if (MODE == kF32) {
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int kk = k0 + lk;
      float av[2], bv[2];
      for (int b = 0; b < 2; ++b) {
        av[b] = (float)fa(b * 16 + li, kk);
        bv[b] = (float)fb(b * 16 + li, kk);
      }
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 32) {
      v8bf ah[2], al[2], bh[2], bl[2];
      for (int b = 0; b < 2; ++b)
        for (int e = 0; e < 8; ++e) {
          const int kk = k0 + 8 * lk + e;
          __bf16 h, l;
          split_bf16(fa(b * 16 + li, kk), h, l);
          ah[b][e] = h; al[b][e] = l;
          split_bf16(fb(b * 16 + li, kk), h, l);
          bh[b][e] = h; bl[b][e] = l;
        }
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bh[y], acc[x][y], 0, 0, 0);
          if (MODE == kBF16x3) {
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bl[y], acc[x][y], 0, 0, 0);
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], bh[y], acc[x][y], 0, 0, 0);
          }
        }
    }
  }
}

// Same tile contract as k_gemm_f64 (see tasks.h), low-precision products.
template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_lp(const GemmTask* __restrict__ tasks,
                                                 double* __restrict__ arena,
                                                 const int32_t* __restrict__ ilim) {
  const GemmTask T = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int n = T.nlim >= 0 ? min(T.n, ilim[T.nlim]) : T.n;
  const int K = T.klim >= 0 ? min(T.k, ilim[T.klim]) : T.k;
  if (T.j0 >= n) return;
  const double* A = arena + T.a;
  const double* B = arena + T.b;
  const int r0 = T.i0 + wr * 32, c0 = T.j0 + wc * 32;
  v4f acc[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) acc[x][y] = (v4f){0.f, 0.f, 0.f, 0.f};
  const bool active = (r0 < T.m) && (c0 < n);
  if (active) {
    auto fa = [&](int r, int k) -> double {
      const int i = r0 + r;
      return (i < T.m && k < K) ? A[(int64_t)i * T.ais + (int64_t)k * T.aks] : 0.0;
    };
    auto fb = [&](int r, int k) -> double {
      const int j = c0 + r;
      return (j < n && k < K) ? B[(int64_t)j * T.bjs + (int64_t)k * T.bks] : 0.0;
    };
    lp_block<MODE>(acc, K, lane, fa, fb);
  }
  __syncthreads();   // A/B may alias C (in-place triangular solve)
  if (!active) return;
  double* C = arena + T.c;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      for (int e = 0; e < 4; ++e) {
        const int i = r0 + x * 16 + 4 * (lane >> 4) + e;
        const int j = c0 + y * 16 + (lane & 15);
        if (i < T.m && j < n) {
          double* cp = C + i + (int64_t)j * T.ldc;
          const double v = T.alpha * (double)acc[x][y][e];
          const double* dp = (T.d >= 0) ? arena + T.d + i + (int64_t)j * T.ldc : cp;
          *cp = (T.beta == 0.0) ? v : v + T.beta * *dp;
        }
      }
}

// Schur-complement update tile (same contract as k_update_f64), low-precision products.
template <int MODE>
__global__ __launch_bounds__(256) void k_update_lp(const UpdTile* __restrict__ tiles,
                                                   const UpdEntry* __restrict__ ents,
                                                   const int32_t* __restrict__ relmap,
                                                   double* __restrict__ arena,
                                                   const int32_t* __restrict__ ilim) {
  __shared__ double tile[64][65];
  __shared__ int32_t rmap[64], cmap[64];
  const UpdTile T = tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
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
      v4f acc[2][2];
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = (v4f){0.f, 0.f, 0.f, 0.f};
      auto fa = [&](int r, int k) -> double {
        const int t = wr * 32 + r;
        return (t < nr && k < K) ? X[E.a + t + (int64_t)k * E.ldx] : 0.0;
      };
      auto fb = [&](int r, int k) -> double {
        const int t = wc * 32 + r;
        return (t < nc && k < K) ? X[E.c + t + (int64_t)k * E.ldx] : 0.0;
      };
      lp_block<MODE>(acc, K, lane, fa, fb);
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
          for (int e2 = 0; e2 < 4; ++e2) {
            const int pr = wr * 32 + x * 16 + 4 * (lane >> 4) + e2;
            const int pc = wc * 32 + y * 16 + (lane & 15);
            if (pr < nr && pc < nc) tile[rmap[pr]][cmap[pc]] -= (double)acc[x][y][e2];
          }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    if (r < T.nrows && c < T.ncols) P[(T.row0 + r) + (int64_t)(T.col0 + c) * T.ld] = tile[r][c];
  }
}

void launch_gemm_lp(int mode, const GemmTask* t, int n, double* arena, const int32_t* ilim, hipStream_t s) {
  if (n <= 0) return;
  if (mode == kF32) hipLaunchKernelGGL(k_gemm_lp<kF32>, dim3(n), dim3(256), 0, s, t, arena, ilim);
  else if (mode == kBF16x3) hipLaunchKernelGGL(k_gemm_lp<kBF16x3>, dim3(n), dim3(256), 0, s, t, arena, ilim);
  else hipLaunchKernelGGL(k_gemm_lp<kBF16>, dim3(n), dim3(256), 0, s, t, arena, ilim);
}

void launch_update_lp(int mode, const UpdTile* t, int n, const UpdEntry* e, const int32_t* relmap,
                      double* arena, const int32_t* ilim, hipStream_t s) {
  if (n <= 0) return;
  if (mode == kF32)
    hipLaunchKernelGGL(k_update_lp<kF32>, dim3(n), dim3(256), 0, s, t, e, relmap, arena, ilim);
  else
    hipLaunchKernelGGL(k_update_lp<kBF16x3>, dim3(n), dim3(256), 0, s, t, e, relmap, arena, ilim);
}

}  // namespace rsc
