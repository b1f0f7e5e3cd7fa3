// Host-side launchers of the gfx950 kernels (all asynchronous on the given stream).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "tasks.h"

namespace rsc {

void launch_fill(double* p, int64_t n, double v, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void launch_assemble(const double* values, const int64_t* slot, int64_t nnz, double* arena,
                     hipStream_t s);
void launch_assemble_pairs(const double* values, const int64_t* idx, const int64_t* slot, int64_t n,
                           double* arena, hipStream_t s);
void launch_scatter_const(const int64_t* slot, int64_t n, double v, double* arena, hipStream_t s);
void launch_potrf_f64(const PotrfTask* t, int n, int nbmax, double* arena, int32_t* status, hipStream_t s);
void launch_philox(const PhiloxTask* t, int n, int64_t max_work, double* arena, bool f32,
                   hipStream_t s);
// Largest Gram diagonal (the drop scale of the Cholesky step); mm[p] > 0: first add the
// shift of shifted Cholesky-QR for a sampled block of mm[p] rows.
void launch_gram_scale(const int64_t* g, const int32_t* ld, const int32_t* nn, const int32_t* mm,
                       const int64_t* out, int n, double* arena, hipStream_t s);
void launch_trunc_prep(const TruncTask* t, int n, double* arena, hipStream_t s);
void launch_trunc_power(const TruncTask* t, int n, double* arena, hipStream_t s);
// the power iteration of k_trunc_power as one launch per product over 64-row blocks
// (step it = 0..4; lmax: the largest l of the tasks), then lambda_max and theta
void launch_trunc_pmv(const TruncTask* t, int n, int lmax, int it, double* arena, hipStream_t s);
void launch_trunc_pfin(const TruncTask* t, int n, double* arena, hipStream_t s);
void launch_trunc_x0(const TruncTask* t, int n, double* arena, hipStream_t s);
void launch_trunc_p(const TruncTask* t, int n, double* arena, hipStream_t s);
void launch_trunc_compact(const TruncTask* t, int n, double* arena, int32_t* ints, hipStream_t s);
void launch_trunc_mfill(const TruncTask* t, int n, double* arena, hipStream_t s);
void launch_trunc_flags(const TruncTask* t, int n, int lmax, double* arena, hipStream_t s);
void launch_trunc_copy(const TruncTask* t, int n, int lmax, double* arena, hipStream_t s);
// the projector's Newton-Schulz steps in one workgroup per supernode with l <= kNsMaxF32
// (FP32) or kNsMaxF64 (FP64); larger supernodes are skipped
constexpr int kNsMaxF32 = 128, kNsMaxF64 = 64;
void launch_trunc_ns(const TruncTask* t, int n, bool fp32, double* arena, const NsSchedule& ns,
                     hipStream_t s);

// sweep kernels: f32 = FP32 copy of the factor operands (mixed forms), or null (arena)
void launch_gemv_n(const GemvTask* t, int n, double* arena, const float* f32, const int32_t* ilim,
                   hipStream_t s);
void launch_row_part(const RowChunk* c, int n, const double* arena, const float* f32,
                     const int32_t* ilim, double* part, hipStream_t s);
void launch_to_f32(const ConvTask* t, int n, const double* arena, float* f32, hipStream_t s);
// FP64 block copies (off -> dst, rows x cols, ld -> dld)
void launch_copy_f64(const ConvTask* t, int n, double* arena, hipStream_t s);
// interior blocks: the block solves and A's coupling products
constexpr int kIntMaxC = 1024;   // largest supernode of an interior block
void launch_interior(const IntSn* sns, int n, bool fwd, const double* arena, const float* f32,
                     const int64_t* rows, const int64_t* pull_ptr, const int64_t* pull_idx, double* w,
                     double* t, double* zr, hipStream_t s);
void launch_coupling(const int64_t* tgt, const int64_t* ptr, const int64_t* vidx, const int64_t* xidx,
                     int64_t n, const double* vals, const double* vec, double* out, bool sub, hipStream_t s);
void launch_part_apply(const PartApply* t, int n, const double* part, double* arena, hipStream_t s);
void launch_gather_rows(const int64_t* tasks, int n, const int64_t* idx, const double* src,
                        double* dst, hipStream_t s);
void launch_coldot(const ColDotTask* t, int n, double* arena, const float* f32, const int64_t* gidx,
                   const int32_t* ilim, double* part, hipStream_t s);
void launch_row_gather(const int64_t* rows, const int64_t* ptr, const int64_t* contrib,
                       int64_t nrows, const double* part, double* y, hipStream_t s);
// small-supernode sweep levels: nt threads per supernode (64 or 256), LDS vectors of
// cpad (columns), lpad (ranks) and rmax (rows) doubles
void launch_sweep_fwd(const SweepTask* t, int n, int nt, int cpad, int lpad, double* arena,
                      const float* f32, int64_t a_y, int64_t a_w, int64_t a_zr, const int32_t* ilim,
                      const int64_t* pull_ptr, const int64_t* pull_idx, hipStream_t s);
void launch_sweep_bwd(const SweepTask* t, int n, int nt, int cpad, int lpad, int rmax, double* arena,
                      const float* f32, int64_t a_w, int64_t a_zz, const int32_t* ilim,
                      const int64_t* rows_idx, hipStream_t s);
// spectral coordinates: blocks of three vectors (column-major, ld n)
constexpr int kSpChunk = 4096;               // rows per workgroup of the block inner products
constexpr int kSpGroup = 8;                  // basis columns per workgroup of the block inner products
constexpr int kSpMaxSteps = 30;              // block Lanczos steps (projected order 3 steps)
constexpr int kSpMaxN = 3 * kSpMaxSteps;
constexpr int kSpMaxCols = 1 + kSpMaxN;      // basis vectors, the constant one included
void launch_lap3(const int64_t* rowptr, const int32_t* colind, int64_t n, const double* X, double* Y,
                 hipStream_t s);
void launch_bdots(const double* Q, int64_t ldq, int ncols, const double* W, int64_t n, double* part,
                  hipStream_t s);
void launch_bsum(const double* part, int nchunks, int nout, double* out, int ld, int r0, int c0, hipStream_t s);
void launch_bupd(const double* Q, int64_t ldq, int ncols, const double* C, double* W, int64_t n, hipStream_t s);
void launch_chol3(const double* G, double* rinv, double* racc, int pass, double* T, int ldt, int r0, int c0,
                  int32_t* flag, hipStream_t s);
void launch_bscale(double* W, int64_t n, const double* rinv, hipStream_t s);
void launch_bcopy(const double* src, double* dst, int64_t len, double v, bool fill, hipStream_t s);
void launch_jacobi(const double* T, int N, int ldt, double* V, double* evals, int32_t* sel, hipStream_t s);
void launch_ritz(const double* Q, int64_t ldq, int nc, const double* V, int ldv, const int32_t* sel, double* Y,
                 int64_t n, hipStream_t s);
void launch_bsign(double* Y, int64_t n, const double* sums, hipStream_t s);
void launch_gather_perm(int64_t n, const int64_t* perm, const double* src, double* dst, hipStream_t s);
void launch_scatter_perm(int64_t n, const int64_t* perm, const double* src, double* dst, hipStream_t s);
void launch_spmv_dot(const Chunk* c, int nc, const int64_t* rowptr, const int32_t* colind,
                     const double* vals, const double* p, double* Ap, double* partial, hipStream_t s);
void launch_dot_partial(const Chunk* c, int nc, const double* a, const double* b, double* partial,
                        hipStream_t s);
void launch_resid_partial(const Chunk* c, int nc, const double* b, const double* ax,
                          double* partial, hipStream_t s);
void launch_seg_sum(const int32_t* seg_ptr, int32_t nseg, const double* partial, double* out,
                    hipStream_t s);
// per-system sum of partials, then alpha (kind 0), the convergence test (1) or beta (2)
void launch_seg_step(const int32_t* seg_ptr, int32_t nseg, const double* partial, const PcgScalars& sc,
                     double rtol, double* arena, int32_t* ints, int kind, hipStream_t s);
void launch_pcg_xr(const Chunk* c, int nc, const PcgScalars& sc, double* arena, const int32_t* ints,
                   double* partial, hipStream_t s);
void launch_pcg_p(const Chunk* c, int nc, const PcgScalars& sc, double* arena, const int32_t* ints,
                  int first, hipStream_t s);
void launch_pcg_start(int32_t nseg, const PcgScalars& sc, double* arena, int32_t* ints, hipStream_t s);
void launch_copy(int64_t n, const double* a, double* b, hipStream_t s);
void launch_grad_values(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* lam,
                        const double* x, double* g, hipStream_t s);
void launch_grad_faces(int64_t nf, const int32_t* fi, const int32_t* fj, const double* lam,
                       const double* x, double* g, hipStream_t s);
// Static device buffer for the partial sums of the allocation-free preconditioner apply
// (kApplyScratchDoubles doubles per GPU): its address on the current device.
constexpr int64_t kApplyScratchDoubles = 1 << 20;   // 8 MiB
hipError_t apply_scratch(double** out);

}  // namespace rsc

namespace rsc {
// LDS-staged MFMA kernels; mode 0 = FP64, 1 = FP32 operands, 2 = BF16 hi/lo split, 3 = BF16
// tile: output tile edge, 64 or 128 (tasks must have been cut to that edge).  ptasks (FP64,
// 64 tiles only): the launch holds tasks with potrf1 > 0, whose workgroups then factor
// their tile as the diagonal block described by ptasks[potrf1 - 1] (status as for POTRF)
void launch_gemm_staged(int mode, int tile, const GemmTask* t, int n, double* arena,
                        const int32_t* ilim, double* part, const PotrfTask* ptasks, int32_t* status,
                        hipStream_t s);
// Adds the K-slice partial tiles of split products and stores C (one workgroup per tile).
void launch_gemm_reduce(int tile, const GemmTask* t, int n, double* arena, const int32_t* ilim,
                        const double* part, hipStream_t s);
// Schur update: one workgroup per target tile (entries in tile order, es = first entry of
// at most 32 x 32); xbase = operand base (the arena in FP64 mode, else the compact copy).
void launch_update_waves(int mode, const UpdTile* t, int n, const UpdEntry* e, const int32_t* relmap,
                         double* arena, const double* xbase, const int32_t* ilim, hipStream_t s);
// Compact row-major copies (FP64, FP32 or BF16 hi/lo chunks) of Schur-update operands;
// f32 (or null): also the block's FP32 column-major copy at the arena's offsets.
void launch_compact_rows(int mode, const CompactTask* t, int n, const double* arena, const int32_t* ilim,
                         double* xc, float* f32, hipStream_t s);
}  // namespace rsc
