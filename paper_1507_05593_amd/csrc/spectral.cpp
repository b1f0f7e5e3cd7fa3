// Spectral coordinates (paper Sec. 4.3): positions in three dimensions for the indices of
// a matrix, from the three lowest eigenvectors of the graph Laplacian of its pattern that
// are orthogonal to the constant vector.  Block Lanczos (the symmetric form of Arnoldi)
// with blocks of three vectors -- three coordinates may share one eigenvalue, which a
// single-vector Krylov space would not resolve -- and the constant vector kept as the
// basis' first vector; every new block is orthogonalised against all earlier basis vectors
// twice and normalised by two Cholesky-QR passes.  The coordinates are the Ritz vectors of
// the three smallest eigenvalues of the projected block-tridiagonal matrix, each signed
// so that sum_i (i + 1) y_i >= 0.
#include <cmath>
#include <vector>

#include "kernels.h"
#include "runtime.h"

namespace rsc {

#define SPCHK(x)                                                                     \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      return Error{RSC_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};  \
  } while (0)

Error spectral_coordinates(Handle& h, int32_t steps, uint64_t seed, double* xyz, double* ritz, hipStream_t s) {
  Error e = ensure_device(h);
  if (e.code) return e;
  const int64_t n = h.S.n;
  if (h.seg_first.size() != 2) return Error{RSC_ERR_INVALID_ARG, "spectral coordinates of a single system only"};
  if (steps < 1 || steps > kSpMaxSteps || 1 + 3 * (int64_t)steps > n)
    return Error{RSC_ERR_INVALID_ARG, "steps must be in [1, 30] with 1 + 3 steps <= n"};
  const int m = steps, N = 3 * m, Np = N + (N & 1), ncols = 1 + N;
  const int nchunks = (int)((n + kSpChunk - 1) / kSpChunk);
  // work space: basis Q (n x ncols), L X (n x 3), chunk partial sums, and the small blocks
  const int64_t lq = n * ncols, llx = 3 * n, lpart = (int64_t)nchunks * ncols * 3;
  const int64_t lsmall = 3 * ncols + 9 + 9 + 9 + (int64_t)N * N + (int64_t)Np * Np + N + 3;
  DevArray<double> buf;
  buf.p = static_cast<double*>(dev_alloc(sizeof(double) * (size_t)(lq + llx + lpart + lsmall)));
  if (!buf.p) return Error{RSC_ERR_OUT_OF_MEMORY, "spectral coordinates work space"};
  buf.n = lq + llx + lpart + lsmall;
  DevArray<int32_t> ib;
  ib.p = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * 8));
  if (!ib.p) return Error{RSC_ERR_OUT_OF_MEMORY, "spectral coordinates flags"};
  ib.n = 8;
  DevArray<PhiloxTask> ph;
  ph.p = static_cast<PhiloxTask*>(dev_alloc(sizeof(PhiloxTask)));
  if (!ph.p) return Error{RSC_ERR_OUT_OF_MEMORY, "spectral coordinates sample task"};
  ph.n = 1;
  double* Q = buf.p;
  double* LX = Q + lq;
  double* part = LX + llx;
  double* C = part + lpart;          // ncols x 3
  double* G = C + 3 * ncols;         // 3 x 3
  double* rinv = G + 9;
  double* racc = rinv + 9;
  double* T = racc + 9;              // N x N
  double* V = T + (int64_t)N * N;    // Np x Np
  double* ev = V + (int64_t)Np * Np; // N
  double* sums = ev + N;             // 3
  int32_t* flag = ib.p;
  int32_t* sel = ib.p + 4;
  const int64_t* rowptr = h.d_rowptr.p;
  const int32_t* colind = h.d_colind.p;

  // W = Q(:, c0 : c0 + 3) minus its components along Q(:, 0 : c0), twice
  auto reorth = [&](int c0) {
    double* W = Q + c0 * n;
    for (int pass = 0; pass < 2; ++pass) {
      launch_bdots(Q, n, c0, W, n, part, s);
      launch_bsum(part, nchunks, 3 * c0, C, c0, 0, 0, s);
      launch_bupd(Q, n, c0, C, W, n, s);
    }
  };
  // two Cholesky-QR passes on Q(:, c0 : c0 + 3); with rT >= 0 the factor R2 R1 goes to
  // the T block (rT, rT - 3) and its transpose
  auto cholqr2 = [&](int c0, int rT) {
    double* W = Q + c0 * n;
    for (int pass = 0; pass < 2; ++pass) {
      launch_bdots(W, n, 3, W, n, part, s);
      launch_bsum(part, nchunks, 9, G, 3, 0, 0, s);
      launch_chol3(G, rinv, racc, pass, rT >= 0 ? T : nullptr, N, rT, rT - 3, flag, s);
      launch_bscale(W, n, rinv, s);
    }
  };

  SPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
  launch_bcopy(nullptr, T, (int64_t)N * N, 0.0, true, s);
  launch_bcopy(nullptr, Q, n, 1.0 / std::sqrt((double)n), true, s);
  // start block: entry (i, c) of the generator under key (seed mod 2^32, (seed >> 32) XOR
  // 0xFFFFFFFF), third counter word 2
  PhiloxTask pt{};
  pt.out = 0; pt.rows = (int32_t)n; pt.cols = 3;
  pt.k0 = (uint32_t)(seed & 0xFFFFFFFFull);
  pt.k1 = (uint32_t)(((seed >> 32) & 0xFFFFFFFFull) ^ 0xFFFFFFFFull);
  pt.c2 = 2;
  SPCHK(hipMemcpyAsync(ph.p, &pt, sizeof(pt), hipMemcpyHostToDevice, s));
  SPCHK(hipStreamSynchronize(s));   // (pt is a host local)
  launch_philox(ph.p, 1, n, Q + n, false, s);
  reorth(1);
  cholqr2(1, -1);
  for (int k = 0; k < m; ++k) {
    const int cx = 1 + 3 * k;                    // this block's first basis column
    launch_lap3(rowptr, colind, n, Q + cx * n, LX, s);
    launch_bdots(Q + cx * n, n, 3, LX, n, part, s);
    launch_bsum(part, nchunks, 9, T, N, 3 * k, 3 * k, s);
    if (k + 1 == m) break;
    launch_bcopy(LX, Q + (cx + 3) * n, 3 * n, 0.0, false, s);
    reorth(cx + 3);
    cholqr2(cx + 3, 3 * (k + 1));
  }
  launch_jacobi(T, N, N, V, ev, sel, s);
  launch_ritz(Q, n, N, V, Np, sel, xyz, n, s);
  launch_bdots(nullptr, n, -1, xyz, n, part, s);
  launch_bsum(part, nchunks, 3, sums, 1, 0, 0, s);
  launch_bsign(xyz, n, sums, s);
  const hipError_t le = hipGetLastError();
  SPCHK(hipStreamSynchronize(s));   // the work space is freed on return
  SPCHK(le);
  int32_t hf[4] = {0, 0, 0, 0};
  std::vector<double> hev(N);
  SPCHK(hipMemcpyAsync(hf, ib.p, sizeof(hf), hipMemcpyDeviceToHost, s));
  SPCHK(hipMemcpyAsync(hev.data(), ev, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  int32_t hsel[3] = {0, 0, 0};
  SPCHK(hipMemcpyAsync(hsel, sel, sizeof(hsel), hipMemcpyDeviceToHost, s));
  SPCHK(hipStreamSynchronize(s));
  if (hf[0]) return Error{RSC_ERR_BREAKDOWN, "the Krylov space was exhausted (fewer steps)"};
  if (ritz)
    for (int k = 0; k < 3; ++k) ritz[k] = hev[hsel[k]];
  return Error{RSC_OK, ""};
}

}  // namespace rsc
