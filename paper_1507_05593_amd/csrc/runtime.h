// Device runtime of the solver: memory plan, launch plans, executor, factor and PCG drivers.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <array>
#include <memory>
#include <string>
#include <vector>

#include "../../include/rsc.h"
#include "symbolic.h"
#include "tasks.h"

namespace rsc {

struct Error {
  rsc_status code;
  std::string msg;
};

// One launch of the executor.
enum CmdType : int32_t {
  kCmdFill, kCmdFillInts, kCmdAssemble, kCmdIdent, kCmdUpdate, kCmdPotrf, kCmdGemm,
  kCmdPhilox, kCmdGramScale, kCmdTruncPrep, kCmdTruncPower, kCmdTruncX0, kCmdTruncP, kCmdTruncCompact,
  kCmdGemvN, kCmdColDot, kCmdRowPart, kCmdPartApply, kCmdRowGather, kCmdGatherPerm, kCmdScatterPerm,
  kCmdGatherRows, kCmdCompact, kCmdGemmReduce, kCmdTruncMfill, kCmdTruncFlags, kCmdTruncCopy,
  kCmdToF32, kCmdTruncNs, kCmdAssembleLevel, kCmdSweepFwd, kCmdSweepBwd, kCmdCopy, kCmdInterior,
  kCmdCoupling,
};

// Kernel identity of a command for the per-kernel profile (index into kernel_name()).
int32_t kernel_id(int32_t type, int64_t a, int64_t b, bool post = false);
const char* kernel_name(int32_t k);

struct Cmd {
  int32_t type;
  int32_t klass;        // RSC_K_* profiling class
  int64_t off;          // offset into the task array of this type (or arena offset)
  int64_t count;        // number of tasks (or elements)
  int64_t a, b;         // command-specific
  double v;             // command-specific
  double flops;         // executed tile flops of the launch (profiling)
  double mflops = 0;    // algorithmic flops of the method credited to the launch
  int32_t mkind = 0;    // with dyn: 1 = Schur update (recount from the pairs' ranks),
                        // 2 = algorithmic = executed (recount), 0 = keep mflops
  int64_t alt_off = -1; // product launch: 128-tile task list awaiting the tile tuner
  int64_t alt_count = 0;
  bool dyn = false;     // inner or column extents read from device ranks: the profile
                        // recounts the flops from the tasks once the ranks are known
  int32_t lds_l = 0, lds_r = 0;   // small-supernode sweep launch: LDS doubles for ranks, rows
  bool post = false;    // product launch whose tasks include next diagonal blocks to factor
};

// Device memory of the library: the caller's allocator when one is set (rsc_set_allocator),
// else hipMalloc / hipFree.  dev_alloc returns nullptr on failure.
void* dev_alloc(size_t bytes);
void dev_free(void* p);
// Replaces the allocator; false while any handle holds device memory.
bool set_allocator(void* (*alloc)(size_t, void*, void*), void (*release)(void*, void*, void*), void* ctx);
// Live handles (an allocator may only change while there are none).
void handle_count(int delta);

template <class T>
struct DevArray {
  T* p = nullptr;
  int64_t n = 0;
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  DevArray& operator=(const DevArray&) = delete;
  ~DevArray() { reset(); }
  void reset() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
};

// Per-supernode storage of the compressed form and its work space (arena offsets).
struct CompSlot {
  int32_t ell = 0;
  // Vj: V_j (r x l); Uj: the kept basis as W_j = M_j U_j (c x l), the form the sweeps apply
  int64_t omega = -1, ypanel = -1, ydinv = -1, V = -1, Vj = -1, Uj = -1, gscale = -1, tvq = -1,
          u = -1;
  int64_t tmp = -1;                  // c x l work block of the implicit products
  int64_t zpanel = -1, zdinv = -1;   // power iterations: [Gram; L^O Y] panel ((l + r) x l) and its inverses
  // truncation work space (l x l blocks, panels with ld 2l)
  int64_t G = -1, Sa = -1, Sb = -1, Mpan = -1, Mdinv = -1, Wpan = -1, Wdinv = -1, Om2 = -1,
          sc = -1;
  int32_t qslot = -1;
};

// One block of a supernode's diagonal block tree (Sec. 4.1-4.2), in-order label s.  A leaf
// (height 0) is the dense diagonal block on columns [ca, cb) (= [ra, rb)) of C_j; an
// internal block is L(R_s, C_s) ~ V_s U_s^T with C_s = [ca, cb) its left subtree's
// columns and R_s = [ra, rb) its right subtree's (offsets relative to C_j).  Arena
// offsets of its work space in the level pool of the rank-structured layout.
struct TreeNode {
  int32_t s = 0, ht = 0;
  int32_t ca = 0, cb = 0, ra = 0, rb = 0;
  int32_t ell = 0;                   // samples (= kept rank) of an internal block
  int64_t dinv = -1;                 // 64 x 64 inverse blocks: the leaf's panel steps, or
                                     // the orthonormalisation panel's
  int64_t omega = -1, tmp = -1, ypanel = -1, W = -1, V = -1, X = -1, gscale = -1;
  int64_t zpanel = -1, zdinv = -1;   // power iterations
};

// A launch plan (command list + task arrays) for one factor mode.
struct FactorPlan {
  bool compressed = false;
  double alpha_D = 0;                // the diagonal rank constant the block trees were planned with
  int32_t tuned = 0, tuned128 = 0;   // product launches tried by the tile tuner / set to 128
  int32_t precision = RSC_FP64;
  double tol = 0;
  std::vector<Cmd> cmds;
  std::vector<GemmTask> gemm;
  std::vector<UpdTile> tiles;
  std::vector<UpdEntry> ents;
  std::vector<double> ent_lower;      // per entry: its (row, col) pairs on or below the diagonal
  std::vector<CompactTask> compact;
  int64_t xc_size = 0;                // compact operand copies (doubles)
  int64_t split_size = 0;             // partial tiles of the largest split-K product (doubles)
  std::vector<PotrfTask> potrf;
  std::vector<PhiloxTask> philox;
  std::vector<TruncTask> trunc;
  std::vector<int64_t> gs_g, gs_out;
  std::vector<int32_t> gs_ld, gs_n, gs_m;   // gs_m > 0: shifted Cholesky-QR pass over gs_m rows
  std::vector<ConvTask> conv;         // FP32 copy of the sweeps' operands (mixed forms)
  std::vector<ConvTask> copy;         // interior blocks: L^O_k's rows inside the block, pool -> factor
  DevArray<GemmTask> d_gemm;
  DevArray<UpdTile> d_tiles;
  DevArray<UpdEntry> d_ents;
  DevArray<CompactTask> d_compact;
  DevArray<double> d_xc;              // compact row-major Schur-update operands
  DevArray<double> d_split;           // K-slice partial tiles (reused by every split product)
  DevArray<PotrfTask> d_potrf;
  DevArray<PhiloxTask> d_philox;
  DevArray<TruncTask> d_trunc;
  DevArray<int64_t> d_gs_g, d_gs_out;
  DevArray<int32_t> d_gs_ld, d_gs_n, d_gs_m;
  DevArray<ConvTask> d_conv;
  DevArray<ConvTask> d_copy;
  hipGraphExec_t graph = nullptr;
  double flops[6] = {0, 0, 0, 0, 0, 0};  // potrf, trsm, update, sample, orth, trunc
};

struct SolvePlan {
  bool compressed = false;
  std::vector<Cmd> fwd_bwd;           // commands of one preconditioner apply (y -> zz)
  std::vector<GemvTask> gemv;
  std::vector<ColDotTask> coldot;
  std::vector<RowChunk> rchunks;
  std::vector<PartApply> papply;
  int64_t part_slots = 0;             // 64-entry partial blocks (reused level by level)
  std::vector<int64_t> rg_rows, rg_ptr, rg_contrib;  // row-gather CSR (all levels)
  std::vector<int64_t> gath;          // (begin, count) pairs of z gathers over R_j
  int32_t small_levels = 0;           // levels 0 .. small_levels-1 run as small-supernode steps
  std::vector<SweepTask> sweep;       // their supernodes, level by level
  std::vector<int64_t> pull_ptr, pull_idx;   // per row (n + 1): zr slots of the contributions
                                             // it pulls inside those levels
  DevArray<GemvTask> d_gemv;
  DevArray<ColDotTask> d_coldot;
  DevArray<RowChunk> d_rchunks;
  DevArray<PartApply> d_papply;
  DevArray<double> d_part;
  DevArray<int64_t> d_rg_rows, d_rg_ptr, d_rg_contrib, d_gath;
  DevArray<SweepTask> d_sweep;
  // interior blocks (Sec. 5.1): the block solves and A's coupling products of each level
  std::vector<IntSn> isns;
  std::vector<int64_t> cp_tgt, cp_ptr, cp_vidx, cp_xidx;
  std::vector<int64_t> ipull_ptr, ipull_idx;   // per column (n + 1): zr slots of the in-block
                                               // products it pulls in the blocks' forward solve
  DevArray<IntSn> d_isns;
  DevArray<int64_t> d_cp_tgt, d_cp_ptr, d_cp_vidx, d_cp_xidx, d_ipull_ptr, d_ipull_idx;
  DevArray<int64_t> d_pull_ptr, d_pull_idx;
  hipGraphExec_t graph_a = nullptr, graph_b = nullptr, graph_apply = nullptr;
  double bytes = 0;                   // factor bytes read by one apply
  double v_rtol = -1;                 // rtol baked into graph_a
  int32_t f32_mode = -1;              // factor operand copy the graphs were captured with
  bool f32_tasks = false;             // the tasks address M_j in the FP32 copy's compact blocks
};

struct Handle {
  rsc_options opt;
  Symbolic S;
  std::vector<int64_t> rowptr;        // original CSR (systems concatenated)
  std::vector<int32_t> colind;
  std::vector<int64_t> seg_first;     // systems + 1
  double t_analyze_ms = 0;

  // layout (host, computed at analyze)
  // (all offsets are arena offsets)
  std::vector<int64_t> panel_off;     // [L^D_j; M_j], 2c x c
  std::vector<int32_t> panel_ld;      // 2c
  std::vector<int64_t> dinv_off;      // 64 x 64 inverse blocks of the panel steps (level pool)
  std::vector<int64_t> uo_off;        // U^O_j (r x c, ld r) in the level pool, or -1
  std::vector<int64_t> lo_off;        // L^O_j (r x c, ld r) of the current factor's layout
  std::vector<int64_t> lo_off_exact, lo_off_comp;   // ... of the exact / rank-structured layout
  std::vector<std::array<int64_t, 2>> lev_uo;       // per level: its U^O range of the pool
  std::vector<int64_t> asm_slot;      // per stored entry: panel slot (rows in C_j) or -1
  std::vector<int64_t> asmo_idx, asmo_slot, asmo_ptr;   // entries of rows R_j: value index and
                                                        // pool-relative slot, by level (asmo_ptr)
  // level pool: offsets relative to its start (set_layout adds the layout's start)
  int64_t pool_base_exact = 0, pool_base_comp = 0;
  std::vector<int64_t> uo_rel, dinv_rel;
  std::vector<std::array<int64_t, 2>> lev_uo_rel;
  std::vector<CompSlot> comp_rel;     // the work-space fields of comp, pool-relative
  // diagonal block trees (rank-structured layout): per supernode its blocks in order
  // (empty: dense L^D_j), planned for the rank constant tree_alpha
  std::vector<std::vector<TreeNode>> tree;
  double tree_alpha = 0;
  std::vector<int64_t> lev_pool_comp;  // per level: its rank-structured pool end before the trees
  int64_t pool_comp_plain = 0;         // the largest of those
  int32_t diag_restarts = 0;           // refactorizations with a larger alpha_D (Sec. 5.3)
  // interior blocks (Sec. 5.1, rank-structured layout with rsc_options.interior): per
  // supernode the root of its block (-1: not in one), the rows of R_j inside the block
  // (r_j otherwise) and the arena offset of those rows of L^O_j kept by the factor
  std::vector<int32_t> iroot;
  std::vector<int32_t> r_in;
  std::vector<int64_t> lo_in;
  std::vector<int64_t> ident_slot;
  std::vector<int32_t> compressible;  // separator with c >= tau_O and r > 0
  std::vector<int32_t> sn_local;      // supernode index within its own system (sample key)

  // device
  bool dev_ready = false;
  int device = -1;
  hipStream_t cap_stream = nullptr;   // private stream used for graph capture only
  int64_t arena_size = 0, ints_size = 0;    // arena_size: the allocated arena's length
  int64_t arena_size_exact = 0, arena_size_comp = 0;   // length each layout needs
  int64_t panels_size = 0;
  int64_t f32_end_exact = 0, f32_end_comp = 0;          // end of the sweeps' operands per layout
  // FP32 copy (mixed forms): offsets [a_lo, f32_end) mirror the arena (L^O_j, V_j, W_j);
  // below a_lo, m32_size floats hold each M_j compact (c x c, ld c) at m32_off[j]
  int64_t a_lo = 0, m32_size = 0;
  std::vector<int64_t> m32_off;
  int64_t a_pool = 0;
  DevArray<double> arena;
  DevArray<float> arena32;            // FP32 copy of the sweeps' factor operands (mixed forms):
                                      // element k holds FP32 offset a_lo - m32_size + k
  bool f32_valid = false;             // the last factorization was mixed: the sweeps read arena32
  DevArray<int32_t> ints;
  DevArray<int64_t> d_asm_slot, d_ident_slot, d_perm, d_rows, d_rowptr, d_asmo_idx, d_asmo_slot;
  DevArray<int32_t> d_colind, d_relmap;
  DevArray<Chunk> d_chunks;
  DevArray<int32_t> d_seg_chunk_ptr;
  int32_t nchunks = 0;
  // arena regions
  int64_t a_values = 0, a_panels = 0;
  int64_t a_x, a_r, a_z, a_p, a_Ap, a_y, a_w, a_s, a_zz, a_b, a_zr, a_partial, a_seg;
  int64_t a_t = 0;                    // interior blocks' solve vector (n)
  PcgScalars sc{};
  int32_t i_status = 0, i_ranks = 0;
  std::vector<CompSlot> comp;         // per supernode (compressible ones only)
  bool comp_ready = false;

  std::unique_ptr<FactorPlan> fplans[3];  // per precision
  FactorPlan* fplan = nullptr;          // plan of the last factor
  std::unique_ptr<SolvePlan> splan;
  bool factored = false;
  double tol = 0;
  int32_t failed_supernode = -1;
  int32_t precision_used = RSC_FP64;
  int32_t retries = 0;
  double t_factor_ms = 0, t_pcg_ms = 0;

  // profiling
  bool profiling = false;
  rsc_profile prof{};
  int64_t kprof_launches[RSC_KERNELS] = {};
  double kprof_ms[RSC_KERNELS] = {};
  double kprof_flops[RSC_KERNELS] = {};
  double kprof_tile_flops[RSC_KERNELS] = {};
};

// analyze-phase layout (no device work)
void plan_layout(Handle& h);
// the pool offsets (and L^O offsets) of the exact (false) or rank-structured layout
void set_layout(Handle& h, bool compressed);
// the diagonal block trees' work space for the rank constant alpha_D (sets
// arena_size_comp); whether every internal block is then sampled at full rank
void plan_trees(Handle& h, double alpha_D);
bool trees_exact(const Handle& h);
// device set-up (first numeric call)
Error ensure_device(Handle& h);
void drop_graphs(Handle& h);
Error ensure_arena(Handle& h, int64_t len);
Error factor(Handle& h, const double* values, double tol, hipStream_t stream);
Error pcg(Handle& h, const double* b, double* x, double rtol, int32_t max_iter, hipStream_t stream,
          rsc_pcg_result* out);
Error apply_preconditioner(Handle& h, const double* r, double* z, hipStream_t stream);
Error apply_preconditioner_noalloc(Handle& h, const double* r, double* z, hipStream_t stream);
Error grad_values(Handle& h, const double* lam, const double* x, double* g, hipStream_t stream);
Error spectral_coordinates(Handle& h, int32_t steps, uint64_t seed, double* xyz, double* ritz, hipStream_t s);
void release_device(Handle& h);

int32_t sample_count(int32_t r, int32_t c, double alpha, int32_t p);

}  // namespace rsc
