// Task descriptors shared by the host planner and the gfx950 kernels.
// All floating-point storage lives in one FP64 arena (offsets in elements);
// all device-side integers (ranks, status words, limits) live in one int32 arena.
#pragma once

#include <cstdint>

namespace rsc {

constexpr int kTile = 64;      // output tile edge of the MFMA kernels and POTRF block size
constexpr int kRowChunkMax = 2048;   // columns of one backward diagonal-solve chunk (LDS)

// C(i,j) = beta D(i,j) + alpha sum_k A(i,k) B(j,k) on one 64x64 output tile.
// A(i,k) = arena[a + i*ais + k*aks], B(j,k) = arena[b + j*bjs + k*bks],
// C(i,j) = arena[c + i + j*ldc].  nlim / klim >= 0 name int-arena slots holding a
// device-side limit on n / k (ranks known only on the device).
struct GemmTask {
  int64_t a, b, c;
  int64_t d;                   // beta term from D(i,j) = arena[d + i + j*ldc] (d < 0: from C)
  int32_t ais, aks, bjs, bks;
  int32_t ldc;
  int32_t m, n, k;
  int32_t i0, j0;
  int32_t nlim, klim;
  int32_t sym;                 // 1: C is symmetric; tiles on or below the diagonal only, each
                               // written with its transpose (diagonal tiles: lower half mirrored)
  int32_t kz, ks;              // kz > 1: K cut into kz chunk-aligned slices, this task computes
                               // slice ks into the partial tile at `part`; a reduce launch adds them
  int32_t potrf1;              // > 0: the tile is a panel's next diagonal block, which this
                               // workgroup then factors (POTRF task potrf1 - 1)
  int64_t part;                // scratch offset (doubles) of the partial tile, column major TM x TM
  double alpha, beta;
};

// One 64x64 target tile of a supernode panel that receives Schur-complement updates
// (Sec. 2.1, Algorithm 1): entries [e0, e1) of the entry list, applied in order.
struct UpdTile {
  int64_t panel;               // arena offset of the target panel
  int32_t ld;                  // its leading dimension
  int32_t row0, col0;          // tile origin in panel-local rows / columns
  int32_t nrows, ncols;        // valid extent (<= 64)
  int32_t e0, e1;
  int32_t es;                  // entries [e0, es) exceed 32 rows or columns, [es, e1) do not
};

// One descendant's contribution to one target tile: rows [a,b) and [c,d) of the
// gathered operand X; the target position of gathered row t is relmap[map + t]
// (panel-local row; as a column index when t < nD).  X is the compact row-major copy,
// X(t, m) at element t * ldx + m (FP64 or FP32) or t * ldx + 2 * (m / 32) * 32 + m % 32
// (BF16 high part; low part 32 further), counted from the double offset x of the
// operand's compact copy, shifted to the pair's rows.
struct UpdEntry {
  int64_t x;
  int64_t map;
  int32_t ldx;
  int32_t kdim;                // inner dimension, or -(1 + int-arena slot) of a device rank
  int32_t a, b, c, d;
};

// One 64-row block of a Schur-update operand to copy into the compact row-major form:
// rows [0, nrows) of the column-major block at arena offset src (column stride ld),
// columns k < kdim (or the device rank at slot -(1 + kdim)); zero up to kp (a multiple
// of 32), written at double offset dst of the compact buffer.
struct CompactTask {
  int64_t src, dst;
  int32_t ld, nrows, kdim, kp;
  int64_t f32;                 // offset of the block's FP32 column-major copy, or -1 for none
};

// Cholesky of one diagonal block (<= 64) of a panel plus the explicit inverse of
// that block (written column-major with ld 64 at `inv`).
struct PotrfTask {
  int64_t panel;
  int64_t inv;
  int32_t ld, nb, d0;
  int32_t sn;                  // supernode for the status word
  int32_t mode;                // 0: fail on a non-positive pivot; 1 / 2: drop dependent columns
                               // (pivot <= 1e-14 / 1e-8 times the scale)
  int32_t mrow;                // > 0: the panel is this one block over identity rows starting at
                               // row mrow, which receive M = L^{-T} (the inverse transposed)
  int64_t scale_off;           // modes 1, 2: arena offset of the scale (largest Gram diagonal)
};

// Gaussian sample of one supernode: rows x cols column-major at `out` (ld = rows).
struct PhiloxTask {
  int64_t out;
  int32_t rows, cols;
  uint32_t k0, k1;
  uint32_t c2, pad_;           // third counter word: 0 for the range-finder sample
};

// One spectral truncation problem (order l): Gram g (l x l), two l x l work
// matrices sa / sb, the Cholesky panel mpan ([G + theta I; I], ld 2l), the basis panel
// wpan ([Gram; sample], ld 2l), scalars sc[0..7], kept rank into ints[qslot].
struct TruncTask {
  int64_t g, sa, sb, mpan, wpan, sc;
  int64_t wout;                // compacted basis W (l x l, ld l)
  int32_t l, qslot;
  double tol;
};

// One 64-row piece of a column-major product: arena[out + t] = sum_m X(t, m) v[m], t < rows.
struct GemvTask {
  int64_t x;                   // X(t, m) = arena[x + t + m*ldx]
  int64_t v;                   // vector (arena offset)
  int64_t out;                 // output (arena offset)
  int32_t ldx, rows;
  int32_t kdim;                // or -(1 + slot) of a device rank
  int32_t kmax;                // bound of that device rank (the sample count)
};

}  // namespace rsc

namespace rsc {

// out[col] = sum_{t < rows(col)} X(t, col) in[idx(t)] for 16 columns [col0, col0+16);
// rows(col) = col + 1 when tri (the transposed upper-triangular inverse block),
// else rows; idx = identity when idx < 0, else the int64 gather list at idx.
// ncols < 0 names -(1 + int-arena slot) holding a device column count.
struct ColDotTask {
  int64_t x, in, idx, out;
  int32_t ldx, rows, ncols, col0;
  int32_t tri;
  int32_t r0, r1;              // rows of this task: [r0, min(r1, rows(col)))
  int32_t slot;                // >= 0: write the 16 sums to partial block `slot` instead of out
  int32_t kmax;                // ncols < 0: bound of the device rank (the sample count)
};


// Contiguous row range inside one system (segment) for chunked vector kernels.
struct Chunk {
  int64_t begin, end;
  int32_t seg, pad_;
};

}  // namespace rsc

namespace rsc {

// Arena offsets of the CG state: n-vectors and per-system scalars (doubles), and
// int-arena slots of the per-system flags.
struct PcgScalars {
  int64_t x, r, z, p, Ap;
  int64_t rz, rznew, pAp, alpha, beta, rr, bnorm, rel;
  int32_t active, iters, any, breakdown;
};

}  // namespace rsc

namespace rsc {

// One block of a factor operand to copy to FP32: rows [0, rows) of columns [0, cols) of
// the column-major block at arena offset off (column stride ld) to FP32 offset dst
// (column stride dld).
constexpr int32_t kConvRows = 4096;
struct ConvTask {
  int64_t off, dst;
  int32_t rows, cols, ld, dld;
};

// Backward diagonal solve chunk: rows [i0, i0 + 64) of z_C = M (w_C - s_C) over the
// columns t in [t0, t1) (M = (L^D)^{-T}, upper triangular, M(i, t) = arena[m + i + t*ld]).
struct RowChunk {
  int64_t m, w, s;             // s < 0: no subtraction
  int32_t ld, c, i0, t0, t1, slot;
  int32_t kind;                // 0: rows of M (w - s) over columns [t0, t1), M upper triangular;
                               // 1: rows of -W u, W = M_j U_j (c x l at m, ld c), u at w, over
                               //    columns [t0, t1) cut at the device rank
  int32_t qslot, kmax;         // kind 1: int-arena slot of the rank and its bound
  int32_t sbase, sns;          // sns > 0: s (kind 0) or u (kind 1) is the sum of column-dot
                               // partial blocks: entry t is the sum over q < sns, in order, of
                               // entry t % 16 of block sbase + (t / 16) sns + q
  int32_t pad_;
};
// One supernode of a small-supernode sweep level: both sweeps of the level run in one
// launch each, one workgroup per supernode.  M_j = (L^D_j)^{-T} (upper triangular,
// M(i, t) = F[m + i + t*ld]); the off-diagonal operand X is L^O_j (r x c) or, compressed,
// V_j (r x l) with W_j = M_j U_j (c x l, ld c) and the rank in the int arena; both column
// major.
constexpr int32_t kSweepMaxR = 2048;   // rows R_j of a small-sweep supernode (LDS)
// Interior blocks (Sec. 5.1): one step of a solve with a block's own factor for one of
// its supernodes (the supernodes of one elimination-tree level run in the same launch).
struct IntSn {
  int64_t m;                   // M_k = (L^D_k)^{-T}, upper triangular, M(i, t) at m + i + t*mld
  int64_t lo;                  // the rows of L^O_k inside the block (rh x c, ld rh)
  int64_t rows;                // offset of R_k in the row list (its first rh rows are those)
  int64_t first;               // first column (permuted index)
  int64_t a, b;                // the block's columns [a, b) (used by its root)
  int32_t c, mld, rh, root;    // root: this supernode is the block's root
};

struct SweepTask {
  int64_t m, x, u;             // u < 0: explicit L^O_j, else W_j = M_j U_j (c x l, ld c)
  int64_t first;               // first column of the supernode (permuted index)
  int64_t rows;                // offset of its rows R_j in the row list and in zr
  int32_t c, r, ld;
  int32_t qslot, kmax;         // compressed: int-arena slot of the rank and its bound
  int32_t pad_;
};

// Sum of consecutive 64-entry partial blocks s0 .. s0+ns-1 applied to a vector block:
// mode 0: dst[r] -= sum, mode 1: dst[r] = sum, for r < nrows.
struct PartApply {
  int64_t dst;
  int32_t nrows, s0, ns, mode;
};

// Scaled Newton-Schulz steps X <- (3 a_k X - a_k^3 X^3) / 2 of the spectral projector.
struct NsSchedule {
  int32_t steps;
  int32_t pad_;
  double alpha[32];
};

}  // namespace rsc
