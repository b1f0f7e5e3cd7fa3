/*
 * rsc.h -- C ABI of the rank-structured supernodal Cholesky solver for MI355X (gfx950).
 *
 * The method (Chadwick and Bindel, "An efficient solver for sparse linear systems
 * based on rank-structured Cholesky factorization"): solve A x = b for a sparse
 * symmetric positive definite A given only as a pre-assembled matrix (Sec. 1),
 * with a symbolic phase on the host (nested-dissection ordering, elimination
 * tree, supernodes; Sec. 2.1-2.2, 3.1) and a numeric phase on the device
 * (Algorithm 1 per supernode, off-diagonal compression by Algorithm 3), the
 * resulting factor preconditioning conjugate gradients (Sec. 5.2, 6.1.1).
 *
 * Conventions for every entry point:
 *  - indices are 0-based; a function returns an rsc_status and never throws;
 *    rsc_last_error() gives a message for the calling thread's last failure;
 *  - "host" pointers are read during the call only and copied; "device" pointers
 *    are HIP device memory owned by the caller, used in stream order on the
 *    stream argument (a hipStream_t, NULL = the null stream) and must stay valid
 *    until that stream reaches the end of the call's work;
 *  - a handle owns all of its device memory (factor, plans, work space) and
 *    releases it in rsc_destroy; a handle is not thread-safe, distinct handles are
 *    independent;
 *  - the symbolic phase needs no GPU; the first numeric call initialises the
 *    current HIP device and binds the handle to it.
 */
#ifndef RSC_H
#define RSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsc_handle_s* rsc_handle;

typedef enum {
  RSC_OK = 0,
  RSC_ERR_INVALID_ARG = 1,   /* null pointer, negative size, option out of range */
  RSC_ERR_PATTERN = 2,       /* pattern not symmetric / unsorted / duplicate / diagonal missing */
  RSC_ERR_NOT_SPD = 3,       /* non-positive or non-finite pivot; supernode in rsc_stats */
  RSC_ERR_NOT_CONVERGED = 4, /* PCG reached max_iter */
  RSC_ERR_BREAKDOWN = 5,     /* PCG: p^T A p <= 0 or r^T z <= 0; or basis orthonormalisation failed */
  RSC_ERR_OUT_OF_MEMORY = 6,
  RSC_ERR_DEVICE = 7,        /* a HIP runtime call failed, or no gfx950 device */
  RSC_ERR_STATE = 8          /* e.g. rsc_pcg before a successful rsc_factor */
} rsc_status;

enum {
  RSC_FP64 = 0,        /* every product in FP64 on MFMA */
  RSC_MIXED_BF16 = 1,  /* Schur-update and TRSM products as split BF16 (hi+lo, three BF16 MFMA
                          products, FP32 accumulation), sampling products in plain BF16 with FP32
                          accumulation; POTRF, orthonormalisation, projection and PCG in FP64;
                          the preconditioner's sweeps read an FP32 copy of the factor (FP64
                          vectors and sums) */
  RSC_MIXED_FP32 = 2   /* Schur-update and TRSM products with FP32 operands and FP32 accumulation
                          on MFMA, sampling in BF16, sweeps as for RSC_MIXED_BF16; the rest FP64 */
};

typedef struct {
  int32_t leaf_max;    /* dissection stops at subgraphs of at most this many vertices (64) */
  int32_t tau_O;       /* separators with at least tau_O columns are compressed (Sec. 3.1; 32) */
  int32_t oversample;  /* p of the rank function of Sec. 5.2 (10) */
  int32_t power_iters; /* power iterations of Algorithm 3 (0): Y <- (L^O)^T (L^O Y), each product's
                          operand first conditioned by one shifted Cholesky-QR pass (the span is
                          unchanged) so that no direction kept by the truncation is lost */
  double alpha_O;      /* alpha of the rank function of Sec. 5.2, used as the sample cap (1.0) */
  uint64_t seed;       /* key of the Gaussian samples (Algorithm 3): supernode j of a system is
                          sampled from Philox4x32-10 under key (seed mod 2^32, (seed >> 32) XOR j)
                          with j counted within its own system (0) */
  int32_t precision;   /* RSC_FP64 | RSC_MIXED_BF16 | RSC_MIXED_FP32 (RSC_FP64) */
  int32_t use_graph;   /* replay the factor and PCG launch sequences as hipGraphs (1) */
  int32_t retry;       /* mixed precision: on RSC_ERR_NOT_SPD refactor with FP32 products, then
                          FP64 (the restart-with-more-accuracy policy of Sec. 5.3) (1) */
  int32_t gemm_tile;   /* output tile edge of the dense-product launches: 0 = picked per launch
                          class by the built-in autotuner (timed on the device the first time a
                          class occurs in the process), 64 or 128 = fixed (0) */
  int32_t keep_lo;     /* rank-structured factor: keep the dense L^O_j of every compressed
                          supernode for rsc_get_block (1), or hold it only while its level is
                          factored, in memory reused by the next level (0) */
  int32_t sweep_small_c; /* the preconditioner's sweeps run each elimination-tree level whose
                          supernodes all have at most this many columns (and at most 2048 rows
                          R_j) as one launch per sweep, one workgroup per supernode; the lowest
                          such levels only, up to the first level that exceeds the bound; at
                          most 1024, 0 = every level by the per-operation launches (64) */
  int32_t tau_D;       /* largest dense diagonal block (Sec. 4.1): in the rank-structured factor a
                          separator of more than tau_D columns stores L^D_j as a complete block
                          tree of depth ceil(log2(c / tau_D)) -- dense leaves of at most tau_D
                          columns, the blocks between them low rank (Sec. 4.2, Algorithms 4-6);
                          0 = every L^D_j dense; 1 is refused (0) */
  int32_t reserved0;
  double alpha_D;      /* alpha of the rank function of Sec. 5.2 for the blocks of a block tree:
                          each is sampled at min(k, ceil(alpha_D sqrt(k) log2 k) + oversample),
                          k = min(rows, cols), and kept at that rank; an indefinite pivot makes
                          rsc_factor restart with alpha_D x 1.25 (Sec. 5.3) until it succeeds or
                          every block is sampled at full rank (0.5) */
  int32_t interior;    /* interior blocks (Sec. 5.1), rank-structured factor: for each maximal
                          subtree of the elimination tree without a compressed supernode (a
                          subdomain the compressed separators cut out; columns C^B), keep only
                          the rows of its L^O_j inside C^B; the preconditioner reaches the
                          block L(R^B, C^B) = A(R^B, C^B) L(C^B, C^B)^{-T} through A's entries
                          and two triangular solves with the block's own factor per sweep
                          (eq. interiorBlockMult).  Same preconditioner; less factor memory,
                          more work per apply (0) */
  int32_t reserved2;
} rsc_options;

typedef struct {
  int32_t iters;          /* PCG iterations (one product with A each) */
  int32_t converged;      /* 1 if ||r|| / ||b|| <= rtol was reached */
  double rel_residual;    /* recursive residual ||r_k|| / ||b|| */
  double true_residual;   /* ||b - A x|| / ||b|| recomputed after the loop */
} rsc_pcg_result;

typedef struct {
  int64_t n, nnz, supernodes, levels, systems;
  int64_t factor_entries;      /* stored FP64 entries of L (diagonal triangles + dense L^O + V,U) */
  int64_t compressed;          /* supernodes stored as V U^T after the last factor */
  int64_t rank_sum, sample_sum;/* sum of kept ranks q_j and of samples l_j */
  int64_t rank_saturated;      /* supernodes with q_j == l_j < min(r_j, c_j) */
  int32_t failed_supernode;    /* -1, or the supernode whose pivot failed */
  int32_t precision_used;      /* precision of the last successful factor (after retries) */
  int32_t retries;             /* refactorisations done by the retry policy */
  int32_t reserved;
  double flops_potrf, flops_trsm, flops_update, flops_sample, flops_orth, flops_trunc;
  double bytes_factor;         /* bytes of the stored factor read by one preconditioner apply
                                  (FP32 entries after a mixed-precision factorization) */
  double t_analyze_ms;         /* host symbolic time */
  double t_factor_ms;          /* device time of the last rsc_factor (hipEvents) */
  double t_pcg_ms;             /* device time of the last rsc_pcg */
  double device_bytes;         /* device memory owned by the handle */
  int64_t gemm_tuned;          /* product launches of the current factor plan timed by the tile
                                  tuner (gemm_tile = 0) */
  int64_t gemm_tile128;        /* of those, launches that run with 128-wide tiles */
  int64_t tree_supernodes;     /* supernodes whose L^D_j is a block tree (Sec. 4), last factor */
  int64_t tree_blocks;         /* their low-rank blocks */
  int64_t tree_rank_sum;       /* the sum of those blocks' ranks */
  int64_t tree_entries;        /* stored entries of the trees: leaf triangles and V_s, U_s */
  double alpha_D_used;         /* the diagonal rank constant of the last factor */
  int32_t diag_restarts;       /* restarts of the last rsc_factor with a larger alpha_D */
  int32_t reserved1;
  int64_t interior_blocks;     /* interior blocks of the last factor (rsc_options.interior) */
  int64_t interior_dropped;    /* entries of L^O beyond the interior blocks not stored */
} rsc_stats;

/* Kernel-class timing (hipEvents around every launch of a class while enabled).  Classes
 * follow the steps of the method: Schur updates; the supernode panels' diagonal blocks,
 * in-place solves and trailing updates; the L^O product; sampling (Algorithm 3's random
 * product and power iterations); orthonormalisation of the sample; projection and kept
 * basis (V = L^O U, the basis of the projector, U_j, V_j); truncation (Gram matrix,
 * projector iterations); PCG; other (assembly, fills). */
enum { RSC_K_UPDATE = 0, RSC_K_POTRF = 1, RSC_K_TRSM = 2, RSC_K_GEMM = 3, RSC_K_EIG = 4,
       RSC_K_PCG = 5, RSC_K_OTHER = 6, RSC_K_LO = 7, RSC_K_SAMPLE = 8, RSC_K_ORTH = 9,
       RSC_K_BASIS = 10, RSC_K_CLASSES = 11 };
/* Flops are counted two ways.  Algorithmic: the work of the method's own steps per
 * supernode from the symbolic plan -- POTRF c^3/3, off-diagonal solve r c^2, Schur updates
 * (SYRK lower half + GEMM) per descendant pair, sampling 2 r c l per product with L^O,
 * orthonormalisation 2 c l^2, Gram matrix 2 r l^2, eigen-truncation 9 l^3 (a symmetric
 * eigensolver's count), kept basis 2 (r + c) l q -- each step's total split over the
 * launches that carry it in proportion to their tile work; explicit inverses, extra
 * orthonormalisation passes and padding earn nothing.  Tile: what the launched tiles
 * execute (2 m n k per tile, ragged edges exact). */
enum { RSC_ARITH_F64 = 0, RSC_ARITH_F32 = 1, RSC_ARITH_BF16 = 2, RSC_ARITHS = 3 };
typedef struct {
  int64_t launches[RSC_K_CLASSES];
  double ms[RSC_K_CLASSES];
  double flops[RSC_K_CLASSES];        /* algorithmic flops of the timed launches */
  double tile_flops[RSC_K_CLASSES];   /* executed tile flops of the timed launches */
  double flops_arith[RSC_K_CLASSES][RSC_ARITHS];  /* algorithmic flops by MFMA arithmetic */
} rsc_profile;

/* Fill *opt with the defaults listed beside each field. */
void rsc_default_options(rsc_options* opt);

/* Symbolic phase (host only, no GPU needed; Sec. 2.1, 2.2, 3.1).
 * n: order of A; rowptr: host int64[n+1]; colind: host int32[rowptr[n]] -- the full
 * symmetric pattern (both triangles), rows sorted, no duplicates, every diagonal
 * entry present.  opt may be NULL (defaults).  On success *out is a new handle.
 * Errors: RSC_ERR_INVALID_ARG, RSC_ERR_PATTERN, RSC_ERR_OUT_OF_MEMORY. */
rsc_status rsc_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind,
                       const rsc_options* opt, rsc_handle* out);

/* rsc_analyze with positions of the indices (Sec. 4.1, 4.3): xyz is host memory,
 * double[3 n] (x, y, z of original index i at 3i .. 3i+2; a two-dimensional problem
 * passes z = 0), borrowed for the call.  With opt->tau_D > 0 the columns of every
 * separator of more than tau_D columns are reordered by the recursive split of their
 * positions along the longest side of each piece's bounding box (a stable sort, the
 * first of equal sides, first half m / 2) into the leaves of its block tree; the
 * supernode's pattern is unchanged.  Positions may come from the mesh or from
 * rsc_spectral_coordinates.  Errors as rsc_analyze, and RSC_ERR_INVALID_ARG for a
 * null xyz or a non-finite position. */
rsc_status rsc_analyze_coords(int64_t n, const int64_t* rowptr, const int32_t* colind,
                              const double* xyz, const rsc_options* opt, rsc_handle* out);

/* Symbolic phase for `count` independent systems factored together: the systems
 * form one block-diagonal matrix (system i's unknowns follow system i-1's), so
 * every elimination-tree level of every system is processed by the same launches;
 * rsc_pcg then runs one independent CG per system.  n, rowptr, colind: host arrays
 * of `count` entries, each as in rsc_analyze.  Values and vectors passed later are
 * the systems' arrays concatenated in order.  Each system is dissected, sampled
 * and solved exactly as it would be alone. */
rsc_status rsc_analyze_batch(int32_t count, const int64_t* n, const int64_t* const* rowptr,
                             const int32_t* const* colind, const rsc_options* opt, rsc_handle* out);

/* Numeric factorization on the device (Algorithm 1 for every supernode, level by
 * level; with tol > 0, Algorithm 3 plus spectral truncation at tol for separators
 * with at least tau_O columns).  values: device double[nnz] aligned with colind;
 * only entries with col <= row are read (the values are taken as symmetric).
 * tol: 0 for the exact factor, else the relative singular-value cut-off (0 < tol < 1).
 * Returns RSC_ERR_NOT_SPD (with stats.failed_supernode) when a pivot is not positive.
 * Synchronises the stream before returning (it reads the status word). */
rsc_status rsc_factor(rsc_handle h, const double* values, double tol, void* stream);

/* Preconditioned CG (Sec. 5.2, 6.1.1) with the factor as preconditioner: x0 = 0,
 * stop when ||r_k|| / ||b|| <= rtol or after max_iter iterations.  b, x: device
 * double[n].  out: host array of `systems` results (one per system of a batch).
 * Returns RSC_ERR_NOT_CONVERGED if some system did not converge (x still holds the
 * last iterate), RSC_ERR_BREAKDOWN on a non-positive curvature or r^T z. */
rsc_status rsc_pcg(rsc_handle h, const double* b, double* x, double rtol, int32_t max_iter,
                   void* stream, rsc_pcg_result* out);

/* z = P^T L^{-T} L^{-1} P r: the two triangular solves of Sec. 1 with the stored
 * (exact or rank-structured) factor.  r, z: device double[n], may not alias. */
rsc_status rsc_apply_preconditioner(rsc_handle h, const double* r, double* z, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same z as
 * rsc_apply_preconditioner, with the same kernels, launched directly on `stream` (no
 * graph of the library's own, so a caller may capture it) and with the partial sums of
 * the sweeps in a static device buffer of RSC_APPLY_SCRATCH_BYTES per GPU instead of
 * memory of the handle; it calls no allocator.  Needs a handle that rsc_factor factored
 * (rsc_factor builds the sweep plan): RSC_ERR_STATE otherwise; RSC_ERR_INVALID_ARG when
 * the plan's partial sums exceed the buffer (the message gives both sizes).  The buffer
 * needs no clearing (every sweep stage writes each block it reads first) and keeps the
 * last call's contents.  All calls on one GPU share it: calls that overlap in time on
 * one GPU (other streams, other threads) race; calls in one stream's order do not.
 * r, z: device double[n], may not alias. */
#define RSC_APPLY_SCRATCH_BYTES (8u << 20)
rsc_status rsc_apply_preconditioner_noalloc(rsc_handle h, const double* r, double* z, void* stream);

/* Spectral coordinates (Sec. 4.3): a position in three dimensions for every index of the
 * handle's matrix (one system only), for reordering when the problem supplies none: the
 * three lowest eigenvectors orthogonal to the constant vector of the graph Laplacian of
 * the pattern (-1 per stored off-diagonal entry, the row's count of them on the
 * diagonal), approximated by block Lanczos iteration (the symmetric form of Arnoldi) with
 * blocks of three vectors over `steps` blocks, every block orthogonalised against all
 * earlier ones; the Ritz vectors of the three smallest Ritz values, each signed so that
 * sum_i (i + 1) y_i >= 0.  The start block is entry (i, c) of the Philox4x32-10 Gaussian
 * stream under key (seed mod 2^32, (seed >> 32) XOR 0xFFFFFFFF) with third counter word 2.
 * xyz: device double[3 n], coordinate c of index i (caller's order) at xyz[i + c n].
 * ritz: optional host double[3], the Ritz values (ascending).  steps in [1, 30] with
 * 1 + 3 steps <= n.  Allocates its work space (n x (1 + 3 steps) doubles and small blocks)
 * for the call and synchronises the stream before returning.
 * Errors: RSC_ERR_INVALID_ARG (null xyz, a batch handle, steps out of range),
 * RSC_ERR_BREAKDOWN (the Krylov space was exhausted: fewer steps), RSC_ERR_OUT_OF_MEMORY,
 * RSC_ERR_DEVICE. */
rsc_status rsc_spectral_coordinates(rsc_handle h, int32_t steps, uint64_t seed, double* xyz, double* ritz,
                                    void* stream);

/* Adjoint of the solve with respect to the matrix values (not in the paper):
 * g[p] = -lambda[row(p)] * x[col(p)] for every stored entry p (CSR order).
 * lambda, x: device double[n]; g: device double[nnz]. */
rsc_status rsc_grad_values(rsc_handle h, const double* lambda, const double* x, double* g,
                           void* stream);

/* Gradient with respect to face coefficients of a two-point-flux operator (not in
 * the paper): g[f] = -(lambda[i]-lambda[j])(x[i]-x[j]) for a face between unknowns
 * i = face_i[f] and j = face_j[f] >= 0, and -lambda[i] x[i] when face_j[f] < 0
 * (a boundary face).  All arrays are device memory; nfaces >= 0. */
rsc_status rsc_grad_faces(int64_t nfaces, const int32_t* face_i, const int32_t* face_j,
                          const double* lambda, const double* x, double* g, void* stream);

/* ---- inspection (host copies; valid after rsc_analyze unless noted) ---- */
rsc_status rsc_get_sizes(rsc_handle h, int64_t* n, int64_t* nnz, int64_t* supernodes,
                         int64_t* levels, int64_t* systems);
/* perm: host int64[n], new index -> old index. */
rsc_status rsc_get_permutation(rsc_handle h, int64_t* perm);
/* first: int64[M+1] column boundaries; parent, level, kind (0 leaf, 1 separator): int32[M]. */
rsc_status rsc_get_supernodes(rsc_handle h, int64_t* first, int32_t* parent, int32_t* level,
                              int32_t* kind);
/* depth: int32[M], the depth d of each supernode's diagonal block tree (Sec. 4.1; 0 for a
 * dense L^D_j): 2^d leaves from halving its c columns (first half m / 2), used by the
 * rank-structured factor. */
rsc_status rsc_get_tree_depths(rsc_handle h, int32_t* depth);
/* rowptr: int64[M+1]; rows: int64[rowptr[M]]: the sorted off-diagonal rows R_j. */
rsc_status rsc_get_rowsets(rsc_handle h, int64_t* rowptr, int64_t* rows);
/* After rsc_factor: samples l_j and kept ranks q_j (0 for uncompressed), int32[M]. */
rsc_status rsc_get_ranks(rsc_handle h, int32_t* ell, int32_t* q);
/* After rsc_factor: copy one supernode's blocks to host, column-major:
 * LD (c x c, lower triangle valid), LO (r x c: the dense off-diagonal block
 * U^O_j (L^D_j)^{-T}; for a compressed supernode the block as computed before
 * compression, available only with rsc_options.keep_lo -- RSC_ERR_STATE otherwise --
 * the factor itself uses V_j, U_j; for a supernode of an interior block (rsc_options.
 * interior) only its rows inside the block are stored: the others are returned as 0),
 * V (r x q), U (c x q).  The factor keeps U_j as W_j = (L^D_j)^{-T} U_j, the form its
 * sweeps apply; U is rebuilt here on the host as (L^D_j)^T W_j (O(c^2 q) host work).
 * Any pointer may be NULL. */
rsc_status rsc_get_block(rsc_handle h, int64_t j, double* LD, double* LO, double* V, double* U);
rsc_status rsc_get_stats(rsc_handle h, rsc_stats* out);
rsc_status rsc_profile_enable(rsc_handle h, int32_t on);   /* also resets the counters */
rsc_status rsc_get_profile(rsc_handle h, rsc_profile* out);
/* The same timings per kernel (and precision mode) rather than per class: entry k in
 * [0, RSC_KERNELS) gives the kernel's name (static string), its launch count, the
 * summed hipEvent time of those launches in ms (events on the launch stream, so
 * each interval is one launch), their algorithmic flops and their executed tile flops
 * (both as for rsc_profile; launches whose extents depend on the kept ranks are counted
 * at the ranks of the factorisation that ran).  Any output may be NULL.  Errors:
 * RSC_ERR_INVALID_ARG for a null handle or k out of range. */
#define RSC_KERNELS 42
rsc_status rsc_get_kernel_profile(rsc_handle h, int32_t k, const char** name, int64_t* launches,
                                  double* ms, double* flops, double* tile_flops);

/* Device memory.  Every device allocation of the library (factor arena, task lists, work
 * buffers) is made by alloc(bytes, stream, ctx) and returned by release(ptr, stream, ctx)
 * (stream is always NULL: the memory outlives any one stream's work; it is released
 * by rsc_destroy after the handle's work is complete).  For callers that manage device
 * memory themselves, e.g. a caching allocator.  alloc returns NULL when it cannot
 * satisfy the request (the calling function then fails with RSC_ERR_OUT_OF_MEMORY).
 * Both NULL restores hipMalloc / hipFree.  Process wide; it may only change while no
 * handle exists.  Errors: RSC_ERR_INVALID_ARG (one callback without the other),
 * RSC_ERR_STATE (handles exist). */
rsc_status rsc_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                             void (*release)(void* ptr, void* stream, void* ctx), void* ctx);

const char* rsc_status_string(rsc_status s);
const char* rsc_last_error(void);
/* Releases the handle and all its device memory (after synchronising its device). */
void rsc_destroy(rsc_handle h);

#ifdef __cplusplus
}
#endif
#endif /* RSC_H */
