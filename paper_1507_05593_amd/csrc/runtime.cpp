// Device runtime: memory plan, launch plans (factor and solve), executor with
// hipGraph replay, the factor driver and the PCG driver.
//
// Storage (one FP64 arena per handle):
//   panel j: column-major 2 c_j x c_j, ld = 2 c_j; rows [0, c) hold L^D_j, rows [c, 2c)
//   start as the identity and end as M_j = (L^D_j)^{-T} (the same blocked factorisation
//   step), the explicit inverse that the sweeps and the implicit products use.
//   L^O_j (r_j x c_j, ld r_j, rows R_j in order) has a block of its own; a compressed
//   supernode holds V_j (r x l_j) and W_j = M_j U_j (c x l_j, the kept basis U_j in the
//   form the sweeps apply) instead (the first q_j columns are the kept basis).  The Schur update U^O_j and the range finder's work space live in a
//   level pool that every elimination-tree level reuses.
#include "runtime.h"

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>

#include "kernels.h"

namespace rsc {

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      return Error{RSC_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};  \
  } while (0)

static const Error kOk{RSC_OK, ""};
// Sign iteration of the spectral projector: the odd cubic f(y) = (3y - y^3)/2 applied to
// a_k X.  On an eigenvalue interval [l, u] the scale a_k = sqrt(3 / (u^2 + u l + l^2)) makes
// f(a_k l) = f(a_k u) (the equioscillating, minimax choice), so small eigenvalues grow
// by about 2.6 per step instead of 1.5; u = 1 + 0.01 keeps an eigenvalue that rounding
// lifts slightly above 1 from crossing the cubic's zero at sqrt(3).  From l >= 0.6 on the
// plain step (a = 1) converges to +-1.  Starting from |x0| >= 1e-5 (an eigenvalue 2e-5
// relative from the cut-off), 18 steps bring every eigenvalue to +-1 within FP64
// rounding -- an eigenvalue left at 1 - 1e-7 would leave a direction of size 5e-8 in the
// projector, which the basis step's relative pivot threshold 1e-14 could keep.
static NsSchedule ns_schedule() {
  NsSchedule s{};
  double l = 1e-5;
  const double u = 1.01;
  auto f = [](double y) { return 0.5 * (3.0 * y - y * y * y); };
  while (1.0 - l > 1e-12 && s.steps < 30) {
    double a = 1.0, nl;
    if (l < 0.6) {
      a = std::sqrt(3.0 / (u * u + u * l + l * l));
      nl = std::min(f(a * l), f(a * u));
    } else {
      nl = f(l);
    }
    s.alpha[s.steps++] = a;
    l = nl;
  }
  if (s.steps % 2) s.alpha[s.steps++] = 1.0;   // the iterate ends in the buffer it started in
  return s;
}
static const NsSchedule kNs = ns_schedule();
static constexpr int32_t kOuter = 256;   // outer block width of the panel factorisation
// levels whose largest sample count exceeds this run the truncation's power iteration as
// row-block launches (one workgroup per supernode streams l^2 entries per product)
static constexpr int32_t kPowerRowsMin = 256;

int32_t sample_count(int32_t r, int32_t c, double alpha, int32_t p) {
  const int32_t k = std::min(r, c);
  if (k <= 0) return 0;
  const double v = std::ceil(alpha * std::sqrt((double)k) * std::log2((double)k)) + p;
  return (int32_t)std::min<double>(k, v);
}

static int64_t align64(int64_t x) { return (x + 63) & ~int64_t(63); }

// ------------------------------------------------------------------ layout

void plan_layout(Handle& h) {
  Symbolic& S = h.S;
  const int64_t M = S.M();
  h.panel_off.assign(M, 0);
  h.panel_ld.assign(M, 0);
  h.compressible.assign(M, 0);
  int64_t poff = 0;
  for (int64_t j = 0; j < M; ++j) {
    const int64_t c = S.c(j), r = S.r(j);
    h.panel_ld[j] = (int32_t)(2 * c);
    h.panel_off[j] = poff;
    poff += align64(2 * c * c);
    h.compressible[j] = (S.kind[j] == kSeparator && c >= h.opt.tau_O && r > 0) ? 1 : 0;
  }
  // Systems of a batch are dissected one after another, so each owns a contiguous
  // range of supernodes; the Gaussian sample is keyed by the index within that range
  // so that a system draws the same sample batched or alone.
  h.sn_local.assign(M, 0);
  {
    int64_t s = 0, base = 0;
    for (int64_t j = 0; j < M; ++j) {
      const int64_t v = S.perm[S.first[j]];
      if (v >= h.seg_first[s + 1]) {
        while (v >= h.seg_first[s + 1]) ++s;
        base = j;
      }
      h.sn_local[j] = (int32_t)(j - base);
    }
  }
  // Interior blocks (Sec. 5.1): the maximal subtrees of the elimination tree holding no
  // compressible supernode (the subdomains that the compressed separators cut out; a
  // subtree's supernodes are consecutive, its root last).  With rsc_options.interior the
  // rank-structured factor keeps of each of their L^O_j only the rows inside the block.
  h.iroot.assign(M, -1);
  h.r_in.assign(M, 0);
  h.lo_in.assign(M, -1);
  for (int64_t j = 0; j < M; ++j) h.r_in[j] = S.r(j);
  const bool ib = h.opt.interior != 0;
  if (ib) {
    std::vector<char> clean(M, 0), kids_ok(M, 1);
    std::vector<int64_t> size(M, 1);
    for (int64_t j = 0; j < M; ++j) {   // children come before their parent
      clean[j] = kids_ok[j] && !h.compressible[j] && S.c(j) <= kIntMaxC;
      if (S.parent[j] >= 0) {
        if (!clean[j]) kids_ok[S.parent[j]] = 0;
        size[S.parent[j]] += size[j];
      }
    }
    for (int64_t b = 0; b < M; ++b) {
      if (!clean[b] || (S.parent[b] >= 0 && clean[S.parent[b]])) continue;
      const int64_t end = S.first[b + 1];
      for (int64_t k = b - size[b] + 1; k <= b; ++k) {
        h.iroot[k] = (int32_t)b;
        const int64_t* rb = S.rows.data() + S.rows_ptr[k];
        h.r_in[k] = (int32_t)(std::lower_bound(rb, rb + S.r(k), end) - rb);
      }
    }
  }
  auto interior = [&](int64_t j) { return ib && h.iroot[j] >= 0 && S.r(j) > 0; };
  const int64_t n = S.n, nnz = S.nnz;
  const int32_t nseg = (int32_t)h.seg_first.size() - 1;
  // arena regions: values, PCG vectors, then the factor's persistent blocks, then the
  // level pool
  int64_t a = 0;
  h.a_values = a; a += align64(nnz);
  h.a_x = a; a += align64(n);
  h.a_r = a; a += align64(n);
  h.a_z = a; a += align64(n);
  h.a_p = a; a += align64(n);
  h.a_Ap = a; a += align64(n);
  h.a_y = a; a += align64(n);
  h.a_w = a; a += align64(n);
  h.a_s = a; a += align64(n);
  h.a_zz = a; a += align64(n);
  h.a_b = a; a += align64(n);
  h.a_t = a; a += align64(n);
  h.a_zr = a; a += align64(std::max<int64_t>((int64_t)S.rows.size(), 1));
  // chunks of <= 256 rows inside one system
  int32_t nch = 0;
  for (int32_t s = 0; s < nseg; ++s) nch += (int32_t)((h.seg_first[s + 1] - h.seg_first[s] + 255) / 256);
  h.nchunks = nch;
  h.a_partial = a; a += align64(std::max(nch, 1));
  h.a_seg = a; a += align64(10 * (int64_t)nseg);
  h.sc.x = h.a_x; h.sc.r = h.a_r; h.sc.z = h.a_z; h.sc.p = h.a_p; h.sc.Ap = h.a_Ap;
  h.sc.rz = h.a_seg; h.sc.rznew = h.a_seg + nseg; h.sc.pAp = h.a_seg + 2 * nseg;
  h.sc.alpha = h.a_seg + 3 * nseg; h.sc.beta = h.a_seg + 4 * nseg; h.sc.rr = h.a_seg + 5 * nseg;
  h.sc.bnorm = h.a_seg + 6 * nseg; h.sc.rel = h.a_seg + 7 * nseg;
  // panels [L^D_j; M_j], 2c x c (ld 2c)
  h.a_panels = a; a += poff;
  h.panels_size = poff;
  for (int64_t j = 0; j < M; ++j) h.panel_off[j] += h.a_panels;
  // the FP32 copy's compact M_j blocks sit just below a_lo in its own offsets
  h.a_lo = a;
  h.m32_off.assign(M, 0);
  {
    int64_t m32 = 0;
    for (int64_t j = 0; j < M; ++j) { h.m32_off[j] = m32; m32 += align64((int64_t)S.c(j) * S.c(j)); }
    h.m32_size = m32;
    for (int64_t j = 0; j < M; ++j) h.m32_off[j] += h.a_lo - m32;
  }
  // dense L^O_j of the supernodes never compressed
  h.lo_off_exact.assign(M, -1);
  h.lo_off_comp.assign(M, -1);
  for (int64_t j = 0; j < M; ++j)
    if (S.r(j) > 0 && !h.compressible[j] && !interior(j)) {
      h.lo_off_exact[j] = h.lo_off_comp[j] = a;
      a += align64((int64_t)S.c(j) * S.r(j));
    }
  // Region X.  Exact factor: the dense L^O_j of the compressible supernodes.  Rank-
  // structured factor: their V_j, W_j = M_j U_j (slot Uj) and the sweeps' two small
  // vectors (and L^O_j when it is kept for inspection).
  const int64_t aX = a;
  int64_t ax = aX;
  for (int64_t j = 0; j < M; ++j)
    if (h.compressible[j] || interior(j)) { h.lo_off_exact[j] = ax; ax += align64((int64_t)S.c(j) * S.r(j)); }
  h.comp.assign(M, CompSlot());
  int32_t islot = 0;
  h.i_status = islot; islot += 4;
  h.i_ranks = islot; islot += (int32_t)M;
  int64_t ac = aX;
  for (int64_t j = 0; j < M; ++j) {
    if (!h.compressible[j]) continue;
    CompSlot& C = h.comp[j];
    const int32_t c = S.c(j), r = S.r(j);
    C.ell = std::min<int32_t>(sample_count(r, c, h.opt.alpha_O, h.opt.oversample), 2048);
    const int64_t l = C.ell;
    C.Vj = ac; ac += align64(r * l);
    C.Uj = ac; ac += align64(c * l);
    C.tvq = ac; ac += align64(l);
    C.u = ac; ac += align64(l);
    if (h.opt.keep_lo) { h.lo_off_comp[j] = ac; ac += align64((int64_t)c * r); }
    C.qslot = h.i_ranks + (int32_t)j;
  }
  // interior blocks: the rows of L^O_j inside the block (r_in x c, ld r_in)
  for (int64_t j = 0; j < M; ++j)
    if (interior(j) && h.r_in[j] > 0) { h.lo_in[j] = ac; ac += align64((int64_t)h.r_in[j] * S.c(j)); }
  h.f32_end_exact = ax;
  h.f32_end_comp = ac;
  // Level pool: per elimination-tree level, U^O_j of its supernodes (assembled and
  // updated there, dead once L^O_j is formed), the 64 x 64 inverse blocks of their panel
  // steps, and with compression the range finder's work space.  The levels run one after
  // another, so each reuses the pool from its start.  The pool follows region X of the
  // factor's own layout (the exact layout's dense L^O_j or the compressed one's V_j, U_j),
  // so its offsets are kept relative to its start and made absolute by set_layout.
  h.pool_base_exact = align64(ax);
  h.pool_base_comp = align64(ac);
  h.uo_rel.assign(M, -1);
  h.dinv_rel.assign(M, 0);
  h.lev_uo_rel.assign(S.nlevels, {0, 0});
  h.comp_rel = h.comp;
  int64_t pool_exact = 0, pool_comp = 0;
  h.lev_pool_comp.assign(S.nlevels, 0);
  for (int32_t L = 0; L < S.nlevels; ++L) {
    int64_t p = 0;
    for (int32_t j : S.by_level[L])
      if (S.r(j) > 0) { h.uo_rel[j] = p; p += align64((int64_t)S.c(j) * S.r(j)); }
    h.lev_uo_rel[L] = {0, p};
    for (int32_t j : S.by_level[L]) { h.dinv_rel[j] = p; p += ((S.c(j) + 63) / 64) * 4096; }
    pool_exact = std::max(pool_exact, p);
    for (int32_t j : S.by_level[L]) {
      if (!h.compressible[j]) continue;
      CompSlot& C = h.comp_rel[j];
      const int64_t c = S.c(j), r = S.r(j), l = C.ell;
      C.omega = p; p += align64(r * l);
      C.tmp = p; p += align64(c * l);
      C.ypanel = p; p += align64((l + c) * l);
      C.ydinv = p; p += ((l + 63) / 64) * 4096;
      C.V = p; p += align64(r * l);
      C.gscale = p; p += 64;
      C.G = p; p += align64(l * l);
      C.Sa = p; p += align64(l * l);
      C.Sb = p; p += align64(l * l);
      C.Om2 = p; p += align64(l * l);
      C.Mpan = p; p += align64(2 * l * l);
      C.Mdinv = p; p += ((l + 63) / 64) * 4096;
      C.Wpan = p; p += align64(2 * l * l);
      C.Wdinv = p; p += ((l + 63) / 64) * 4096;
      C.sc = p; p += 128;   // scalars [0, 64), power-iteration partial sums [64, 128)
      if (h.opt.power_iters > 0) {
        C.zpanel = p; p += align64((l + r) * l);
        C.zdinv = p; p += ((l + 63) / 64) * 4096;
      }
    }
    // interior blocks: the whole L^O_j of the level's interior supernodes, held only while
    // the level is factored (its rows beyond the block feed the Schur updates' compact
    // copies, then die)
    for (int32_t j : S.by_level[L])
      if (interior(j)) { h.lo_off_comp[j] = h.pool_base_comp + p; p += align64((int64_t)S.c(j) * S.r(j)); }
    h.lev_pool_comp[L] = p;
    pool_comp = std::max(pool_comp, p);
  }
  h.arena_size_exact = align64(h.pool_base_exact + pool_exact);
  h.pool_comp_plain = pool_comp;
  plan_trees(h, h.opt.alpha_D);
  h.lo_off = h.lo_off_exact;
  h.a_pool = -1;
  set_layout(h, false);
  // PCG int slots
  h.sc.active = islot; islot += nseg;
  h.sc.iters = islot; islot += nseg;
  h.sc.any = islot++;
  h.sc.breakdown = islot++;
  h.ints_size = islot;

  // assembly: entry (i, col) with col <= i goes to the lower position of the permuted
  // pair in the supernode owning the column -- its panel (rows in C_j, at the start of
  // a factorization) or its U^O_j in the pool (rows in R_j, at the start of its level;
  // offsets relative to the pool)
  h.asm_slot.assign(nnz, -1);
  std::vector<std::vector<std::pair<int64_t, int64_t>>> lev_ent(S.nlevels);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = h.rowptr[i]; p < h.rowptr[i + 1]; ++p) {
      const int64_t col = h.colind[p];
      if (col > i) continue;
      const int64_t ni = S.iperm[i], nc = S.iperm[col];
      const int64_t lo = std::min(ni, nc), hi = std::max(ni, nc);
      const int64_t j = S.owner[lo];
      const int64_t t = lo - S.first[j];
      if (hi < S.first[j + 1]) {
        h.asm_slot[p] = h.panel_off[j] + t * h.panel_ld[j] + (hi - S.first[j]);
      } else {
        const int64_t* b = S.rows.data() + S.rows_ptr[j];
        const int64_t* e = S.rows.data() + S.rows_ptr[j + 1];
        const int64_t f = std::lower_bound(b, e, hi) - b;
        lev_ent[S.level[j]].push_back({p, h.uo_rel[j] + t * S.r(j) + f});
      }
    }
  }
  h.asmo_idx.clear();
  h.asmo_slot.clear();
  h.asmo_ptr.assign(1, 0);
  for (int32_t L = 0; L < S.nlevels; ++L) {
    for (auto& e : lev_ent[L]) { h.asmo_idx.push_back(e.first); h.asmo_slot.push_back(e.second); }
    h.asmo_ptr.push_back((int64_t)h.asmo_idx.size());
  }
  h.ident_slot.clear();
  for (int64_t j = 0; j < M; ++j) {
    const int64_t c = S.c(j);
    for (int64_t t = 0; t < c; ++t) h.ident_slot.push_back(h.panel_off[j] + t * h.panel_ld[j] + (c + t));
  }
}

// Diagonal block trees (Sec. 4.1-4.2): a supernode with tree depth d > 0 splits its c
// columns into 2^d leaves by halving (first half m / 2); the blocks are numbered in order
// (leaves odd, the root 2^d).  Each level's trees take work space after that level's
// rank-structured pool: a leaf its panel steps' inverse blocks; an internal block its
// sample, the intermediate of its products, the orthonormalisation panel [Gram; Y], the
// kept W = M_{s1} U_s, V_s and X = M_{s2}^T V_s.
void plan_trees(Handle& h, double alpha_D) {
  const Symbolic& S = h.S;
  h.tree.assign(S.M(), {});
  h.tree_alpha = alpha_D;
  const int64_t base = h.pool_base_comp;
  int64_t pool = h.pool_comp_plain;
  for (int32_t L = 0; L < S.nlevels; ++L) {
    int64_t p = h.lev_pool_comp[L];
    for (int32_t j : S.by_level[L]) {
      const int32_t d = S.depth[j];
      if (d == 0) continue;
      const int32_t c = S.c(j), nleaf = 1 << d;
      std::vector<int32_t> bnd;
      std::function<void(int32_t, int32_t, int32_t)> split = [&](int32_t lo, int32_t m, int32_t dep) {
        if (dep == 0) { bnd.push_back(lo); return; }
        split(lo, m / 2, dep - 1);
        split(lo + m / 2, m - m / 2, dep - 1);
      };
      split(0, c, d);
      bnd.push_back(c);
      std::vector<TreeNode>& T = h.tree[j];
      T.resize(2 * nleaf - 1);
      for (int32_t s = 1; s < 2 * nleaf; ++s) {
        TreeNode& t = T[s - 1];
        t.s = s;
        t.ht = __builtin_ctz(s);
        auto span = [&](int32_t u, int32_t hu, int32_t& a, int32_t& b) {
          const int32_t f = (u - ((1 << hu) - 1)) / 2;
          a = bnd[f]; b = bnd[f + (1 << hu)];
        };
        if (t.ht == 0) {
          span(s, 0, t.ca, t.cb);
          t.ra = t.ca; t.rb = t.cb;
          t.dinv = base + p; p += ((t.cb - t.ca + 63) / 64) * 4096;
          continue;
        }
        span(s - (1 << (t.ht - 1)), t.ht - 1, t.ca, t.cb);
        span(s + (1 << (t.ht - 1)), t.ht - 1, t.ra, t.rb);
        const int64_t nc = t.cb - t.ca, nr = t.rb - t.ra;
        t.ell = std::min<int32_t>(sample_count((int32_t)nr, (int32_t)nc, alpha_D, h.opt.oversample), 2048);
        const int64_t l = t.ell;
        t.omega = base + p; p += align64(nr * l);
        t.tmp = base + p; p += align64(std::max(nc, nr) * l);
        t.ypanel = base + p; p += align64((l + nc) * l);
        t.dinv = base + p; p += ((l + 63) / 64) * 4096;
        t.W = base + p; p += align64(nc * l);
        t.V = base + p; p += align64(nr * l);
        t.X = base + p; p += align64(nr * l);
        t.gscale = base + p; p += 64;
        if (h.opt.power_iters > 0) {
          t.zpanel = base + p; p += align64((l + nr) * l);
          t.zdinv = base + p; p += ((l + 63) / 64) * 4096;
        }
      }
    }
    pool = std::max(pool, p);
  }
  h.arena_size_comp = align64(h.pool_base_comp + pool);
}

bool trees_exact(const Handle& h) {
  for (const auto& T : h.tree)
    for (const TreeNode& t : T)
      if (t.ht > 0 && t.ell < std::min(t.cb - t.ca, t.rb - t.ra)) return false;
  return true;
}

// Pool offsets of one layout (exact or compressed factor): the pool-relative tables plus
// that layout's pool start.
void set_layout(Handle& h, bool compressed) {
  const int64_t base = compressed ? h.pool_base_comp : h.pool_base_exact;
  h.lo_off = compressed ? h.lo_off_comp : h.lo_off_exact;
  if (h.a_pool == base) return;
  h.a_pool = base;
  const int64_t M = h.S.M();
  h.uo_off.assign(M, -1);
  h.dinv_off.assign(M, 0);
  for (int64_t j = 0; j < M; ++j) {
    if (h.uo_rel[j] >= 0) h.uo_off[j] = base + h.uo_rel[j];
    h.dinv_off[j] = base + h.dinv_rel[j];
  }
  h.lev_uo.assign(h.lev_uo_rel.size(), {0, 0});
  for (size_t L = 0; L < h.lev_uo_rel.size(); ++L)
    h.lev_uo[L] = {base + h.lev_uo_rel[L][0], base + h.lev_uo_rel[L][1]};
  for (int64_t j = 0; j < M; ++j) {
    if (!h.compressible[j]) continue;
    const CompSlot& R = h.comp_rel[j];
    CompSlot& C = h.comp[j];
    auto abs = [&](int64_t x) { return x >= 0 ? base + x : x; };
    C.omega = abs(R.omega); C.tmp = abs(R.tmp); C.ypanel = abs(R.ypanel); C.ydinv = abs(R.ydinv);
    C.V = abs(R.V); C.gscale = abs(R.gscale); C.G = abs(R.G); C.Sa = abs(R.Sa); C.Sb = abs(R.Sb);
    C.Om2 = abs(R.Om2); C.Mpan = abs(R.Mpan); C.Mdinv = abs(R.Mdinv); C.Wpan = abs(R.Wpan);
    C.Wdinv = abs(R.Wdinv); C.sc = abs(R.sc); C.zpanel = abs(R.zpanel); C.zdinv = abs(R.zdinv);
  }
}

// ------------------------------------------------------------------ device set-up

namespace {
void* (*g_alloc)(size_t, void*, void*) = nullptr;
void (*g_release)(void*, void*, void*) = nullptr;
void* g_alloc_ctx = nullptr;
std::atomic<int> g_live_handles{0};
std::mutex g_alloc_mu;
}  // namespace

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (g_alloc) return g_alloc(bytes, nullptr, g_alloc_ctx);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void dev_free(void* p) {
  if (!p) return;
  if (g_release) {
    // hipFree waits for the device; a caller's allocator may hand the block out at once
    (void)hipDeviceSynchronize();
    g_release(p, nullptr, g_alloc_ctx);
  } else {
    (void)hipFree(p);
  }
}

bool set_allocator(void* (*alloc)(size_t, void*, void*), void (*release)(void*, void*, void*), void* ctx) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (alloc == g_alloc && release == g_release && (alloc == nullptr || ctx == g_alloc_ctx))
    return true;                                   // no change
  if (g_live_handles.load() != 0) return false;
  g_alloc = alloc;
  g_release = release;
  g_alloc_ctx = alloc ? ctx : nullptr;
  return true;
}

void handle_count(int delta) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_live_handles += delta;
}

template <class T>
static Error upload(DevArray<T>& d, const std::vector<T>& v) {
  d.reset();
  d.n = (int64_t)v.size();
  if (v.empty()) return kOk;
  d.p = static_cast<T*>(dev_alloc(sizeof(T) * v.size()));
  if (!d.p) return Error{RSC_ERR_OUT_OF_MEMORY, "device array of " + std::to_string(sizeof(T) * v.size()) + " bytes"};
  HIPCHK(hipMemcpy(d.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return kOk;
}

Error ensure_device(Handle& h) {
  if (h.dev_ready) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != h.device) return Error{RSC_ERR_STATE, "handle is bound to another device"};
    return kOk;
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return Error{RSC_ERR_DEVICE, std::string("this library is built for gfx950, found ") + prop.gcnArchName};
  h.device = dev;
  h.ints.p = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (size_t)h.ints_size));
  if (!h.ints.p) return Error{RSC_ERR_OUT_OF_MEMORY, "int arena"};
  h.ints.n = h.ints_size;
  HIPCHK(hipMemset(h.ints.p, 0, sizeof(int32_t) * (size_t)h.ints_size));
  Error r;
  if ((r = upload(h.d_asm_slot, h.asm_slot)).code) return r;
  if ((r = upload(h.d_asmo_idx, h.asmo_idx)).code) return r;
  if ((r = upload(h.d_asmo_slot, h.asmo_slot)).code) return r;
  if ((r = upload(h.d_ident_slot, h.ident_slot)).code) return r;
  if ((r = upload(h.d_perm, h.S.perm)).code) return r;
  if ((r = upload(h.d_rows, h.S.rows)).code) return r;
  if ((r = upload(h.d_rowptr, h.rowptr)).code) return r;
  if ((r = upload(h.d_colind, h.colind)).code) return r;
  if ((r = upload(h.d_relmap, h.S.relmap)).code) return r;
  std::vector<Chunk> ch;
  std::vector<int32_t> segp(1, 0);
  const int32_t nseg = (int32_t)h.seg_first.size() - 1;
  for (int32_t s = 0; s < nseg; ++s) {
    for (int64_t b = h.seg_first[s]; b < h.seg_first[s + 1]; b += 256)
      ch.push_back(Chunk{b, std::min(b + 256, h.seg_first[s + 1]), s, 0});
    segp.push_back((int32_t)ch.size());
  }
  if ((r = upload(h.d_chunks, ch)).code) return r;
  if ((r = upload(h.d_seg_chunk_ptr, segp)).code) return r;
  HIPCHK(hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking));
  h.dev_ready = true;
  return kOk;
}

// Destroys every captured graph of the handle (they hold device pointers of the arena
// and its FP32 copy); plans keep their task lists and are captured again when next run.
void drop_graphs(Handle& h) {
  if (h.dev_ready) (void)hipDeviceSynchronize();
  for (auto& fp : h.fplans)
    if (fp && fp->graph) { (void)hipGraphExecDestroy(fp->graph); fp->graph = nullptr; }
  if (h.splan) {
    if (h.splan->graph_a) (void)hipGraphExecDestroy(h.splan->graph_a);
    if (h.splan->graph_b) (void)hipGraphExecDestroy(h.splan->graph_b);
    if (h.splan->graph_apply) (void)hipGraphExecDestroy(h.splan->graph_apply);
    h.splan->graph_a = h.splan->graph_b = h.splan->graph_apply = nullptr;
  }
}

// The arena at least `len` doubles long (the layout of the factor about to run).
Error ensure_arena(Handle& h, int64_t len) {
  if (h.arena.p && h.arena.n >= len) return kOk;
  drop_graphs(h);
  h.arena.reset();
  h.arena.p = static_cast<double*>(dev_alloc(sizeof(double) * (size_t)len));
  h.arena.n = h.arena.p ? len : 0;
  h.arena_size = h.arena.n;
  if (!h.arena.p) return Error{RSC_ERR_OUT_OF_MEMORY, "arena of " + std::to_string(8 * len) + " bytes"};
  return kOk;
}

void release_device(Handle& h) {
  if (h.dev_ready) (void)hipDeviceSynchronize();
  for (auto& fp : h.fplans)
    if (fp && fp->graph) (void)hipGraphExecDestroy(fp->graph);
  if (h.splan) {
    if (h.splan->graph_a) (void)hipGraphExecDestroy(h.splan->graph_a);
    if (h.splan->graph_b) (void)hipGraphExecDestroy(h.splan->graph_b);
    if (h.splan->graph_apply) (void)hipGraphExecDestroy(h.splan->graph_apply);
  }
  for (auto& fp : h.fplans) fp.reset();
  h.fplan = nullptr;
  h.splan.reset();
  if (h.cap_stream) (void)hipStreamDestroy(h.cap_stream);
  h.cap_stream = nullptr;
  h.dev_ready = false;
}

// ------------------------------------------------------------------ factor plan

namespace {

struct PanelDesc {
  int64_t off;
  int32_t ld, n, m_below;
  bool ident;
  int64_t dinv;
  int32_t sn, mode;
  int64_t scale_off;
  int32_t lp_lo = 0, lp_hi = 0;   // rows [lp_lo, lp_hi) use the low-precision products
  bool skip_mid = false;          // ... or are not touched at all
  bool tail_lp = false;           // rows from lp_hi on (the inverse being formed) use lp_tri
};

// Merges a GEMM command's 64 x 64 output tiles (tasks [off, end) of the list, in the
// order the builder cut them) into 128 x 128 tiles: tasks of one product share every
// field but the tile origin and, for a triangular right operand, k; four neighbours
// (origins relative to the product's first tile) become one task whose k is the
// largest of theirs.  Returns the new task count.  Blocks the 64 cut skipped (strictly
// above the diagonal of a symmetric product) may be computed inside a merged tile;
// those entries are never read.
static int64_t retile128(std::vector<GemmTask>& g, int64_t off) {
  struct Key {
    GemmTask t;
    bool same(const GemmTask& u) const {
      return u.a == t.a && u.b == t.b && u.c == t.c && u.d == t.d && u.ais == t.ais &&
             u.aks == t.aks && u.bjs == t.bjs && u.bks == t.bks && u.ldc == t.ldc && u.m == t.m &&
             u.n == t.n && u.nlim == t.nlim && u.klim == t.klim && u.alpha == t.alpha &&
             u.beta == t.beta;
    }
  };
  std::vector<GemmTask> out;
  std::vector<std::pair<int64_t, int64_t>> org;           // per product: origin (i0, j0)
  std::vector<size_t> prod_first;                         // first output index of each product
  std::map<std::tuple<size_t, int32_t, int32_t>, size_t> slot;
  std::vector<Key> prods;
  const int64_t end = (int64_t)g.size();
  for (int64_t i = off; i < end; ++i) {
    const GemmTask& u = g[i];
    size_t pi = prods.size();
    for (size_t q = prods.size(); q-- > 0;) {
      if (prods[q].same(u)) { pi = q; break; }
    }
    if (pi == prods.size()) {
      prods.push_back(Key{u});
      int64_t i0 = u.i0, j0 = u.j0;
      for (int64_t v = i; v < end; ++v)            // the product's smallest origins
        if (Key{u}.same(g[v])) { i0 = std::min<int64_t>(i0, g[v].i0); j0 = std::min<int64_t>(j0, g[v].j0); }
      org.push_back({i0, j0});
    }
    const int32_t bi = (int32_t)((u.i0 - org[pi].first) / 128), bj = (int32_t)((u.j0 - org[pi].second) / 128);
    auto key = std::make_tuple(pi, bi, bj);
    auto it = slot.find(key);
    if (it == slot.end()) {
      GemmTask t = u;
      t.i0 = (int32_t)(org[pi].first + 128 * bi);
      t.j0 = (int32_t)(org[pi].second + 128 * bj);
      slot[key] = out.size();
      out.push_back(t);
    } else {
      GemmTask& t = out[it->second];
      t.k = std::max(t.k, u.k);
    }
  }
  g.resize(off);
  g.insert(g.end(), out.begin(), out.end());
  return (int64_t)out.size();
}

constexpr int kCholQRPasses = 2;

struct Builder {
  Handle& h;
  FactorPlan& P;
  int32_t lp_update = 0;   // 0: FP64 MFMA; else the low-precision mode of launch_gemm_staged
  int32_t lp_sample = 0;
  int32_t lp_eig = 0;      // products of the spectral truncation (projector iterations)
  int32_t lp_tri = 0;      // the rows of a panel that form the inverse of its diagonal block
  bool next_post = false;  // the next cmd() is a product launch carrying diagonal blocks
  int32_t ctx = -1;        // >= 0: profiling class of every launch emitted (a compression stage)
  std::vector<int64_t> xc_off;   // compact copy of supernode j's update operand (doubles), or -1
  std::vector<int32_t> xc_kp;    // its row length: kept columns rounded up to 32
  Builder(Handle& hh, FactorPlan& pp) : h(hh), P(pp) {
    if (P.precision == RSC_MIXED_BF16) { lp_update = 2; lp_sample = 3; lp_eig = 1; lp_tri = 1; }
    if (P.precision == RSC_MIXED_FP32) { lp_update = 1; lp_sample = 3; lp_eig = 1; lp_tri = 1; }
    const Symbolic& S = h.S;
    xc_off.assign(S.M(), -1);
    xc_kp.assign(S.M(), 0);
    // r x kp FP64 values (r * kp doubles), or FP32 values or BF16 pairs (r * kp / 2)
    int64_t off = 0;
    for (int64_t j = 0; j < S.M(); ++j) {
      if (S.r(j) == 0) continue;
      const int32_t kmax = (P.compressed && h.compressible[j]) ? h.comp[j].ell : S.c(j);
      xc_kp[j] = (kmax + 31) / 32 * 32;
      xc_off[j] = off;
      off += ((int64_t)S.r(j) * xc_row(j) + 31) / 32 * 32;
    }
    P.xc_size = off;
  }

  // doubles per row of supernode j's compact operand copy
  int64_t xc_row(int64_t j) const { return lp_update == 0 ? xc_kp[j] : xc_kp[j] / 2; }

  void cmd(int32_t type, int32_t klass, int64_t off, int64_t count, double flops, int64_t a = 0,
           int64_t b = 0, double v = 0) {
    const bool post = next_post;          // tasks with next diagonal blocks: no split, no 128 copy
    next_post = false;
    if (count <= 0) return;
    int64_t alt_off = -1, alt_count = 0;
    // split K: a 64-tile product with fewer tiles than two per compute unit and a long
    // K gets kz slices per tile (each at least 256 of K, at most 2048 workgroups in all)
    // whose partial tiles a reduce launch adds
    int32_t kz = 1;
    int64_t red_off = -1;
    if (type == kCmdGemm) {
      // the command's 64-tile tasks are the last ones pushed; with a fixed tile option
      // they are cut to it, else a 128-tile copy is kept for the tile tuner
      b = 64;
      if (off + count == (int64_t)P.gemm.size()) {
        int64_t last_col = 0;
        int32_t kmax = 0;
        for (int64_t i = off; i < off + count; ++i) {
          if (P.gemm[i].n - P.gemm[i].j0 <= kTile) ++last_col;
          kmax = std::max(kmax, P.gemm[i].k);
        }
        // products mostly one 64-column tile wide (the in-place triangular solves)
        // would leave half of every 128 tile idle; launches under 16 tiles would leave
        // most of the chip idle with a quarter as many workgroups
        const bool narrow = 2 * last_col > count;
        if (!post && h.opt.gemm_tile != 128 && count < 512)
          kz = (int32_t)std::min<int64_t>({8, (2048 + count - 1) / count, std::max(1, kmax / 256)});
        if (h.opt.gemm_tile == 128) {
          count = retile128(P.gemm, off);
          b = 128;
        } else if (kz > 1) {
          red_off = off;
          std::vector<GemmTask> sl;
          sl.reserve((size_t)(count * kz));
          for (int64_t i = 0; i < count; ++i) {
            GemmTask& t = P.gemm[off + i];
            t.kz = kz;
            t.part = i * kz * 4096;
            for (int32_t q = 0; q < kz; ++q) {
              GemmTask u = t;
              u.ks = q;
              u.part = t.part + (int64_t)q * 4096;
              sl.push_back(u);
            }
          }
          off = (int64_t)P.gemm.size();
          P.gemm.insert(P.gemm.end(), sl.begin(), sl.end());
          count *= kz;
          P.split_size = std::max(P.split_size, count * 4096);
        } else if (!post && h.opt.gemm_tile == 0 && !narrow && count >= 16) {
          alt_off = (int64_t)P.gemm.size();
          P.gemm.insert(P.gemm.end(), P.gemm.begin() + off, P.gemm.begin() + off + count);
          alt_count = retile128(P.gemm, alt_off);
        }
      }
    }
    Cmd c;
    c.type = type; c.klass = ctx >= 0 ? ctx : klass; c.off = off; c.count = count; c.a = a; c.b = b; c.v = v;
    c.flops = flops;
    c.alt_off = alt_off; c.alt_count = alt_count;
    c.post = post;
    if (type == kCmdGemm)
      for (int64_t i = off; i < off + count && !c.dyn; ++i) c.dyn = (P.gemm[i].nlim >= 0 || P.gemm[i].klim >= 0);
    P.cmds.push_back(c);
    if (red_off >= 0) {
      Cmd r = c;
      r.type = kCmdGemmReduce; r.off = red_off; r.count = count / kz; r.flops = 0; r.dyn = false;
      P.cmds.push_back(r);
    }
  }

  // Algorithmic flops of one step of the method, `total`, split over the commands
  // emitted since command index c0 in proportion to their tile work.
  void credit(size_t c0, double total) {
    double ex = 0;
    for (size_t i = c0; i < P.cmds.size(); ++i) ex += P.cmds[i].flops;
    if (ex <= 0) return;
    for (size_t i = c0; i < P.cmds.size(); ++i) P.cmds[i].mflops += total * P.cmds[i].flops / ex;
  }

  // Tiles of C(i, j) for i in [ib, m), j in [jb, n); lower: skip tiles lying strictly
  // above the diagonal.
  double tiles(GemmTask t, int32_t ib, int32_t jb, bool lower, std::vector<GemmTask>* out = nullptr) {
    double fl = 0;
    std::vector<GemmTask>& dst = out ? *out : P.gemm;
    for (int32_t j0 = jb; j0 < t.n; j0 += kTile)
      for (int32_t i0 = ib; i0 < t.m; i0 += kTile) {
        if (lower && i0 + kTile - 1 < j0) continue;
        t.i0 = i0; t.j0 = j0;
        dst.push_back(t);
        fl += 2.0 * std::min(kTile, t.m - i0) * std::min(kTile, t.n - j0) * (double)t.k;
      }
    return fl;
  }

  static GemmTask gt(int64_t a, int32_t ais, int32_t aks, int64_t b, int32_t bjs, int32_t bks,
                     int64_t c, int32_t ldc, int32_t m, int32_t n, int32_t k, double alpha,
                     double beta) {
    GemmTask t{};
    t.a = a; t.ais = ais; t.aks = aks; t.b = b; t.bjs = bjs; t.bks = bks; t.c = c; t.ldc = ldc;
    t.m = m; t.n = n; t.k = k; t.alpha = alpha; t.beta = beta; t.nlim = -1; t.klim = -1; t.d = -1;
    t.sym = 0; t.kz = 1; t.ks = 0; t.part = 0;
    return t;
  }

  // Symmetric product: the tiles on or below the diagonal, each written with its mirror
  // image.  The beta term must come from a separate D (the mirror writes would overwrite
  // C before it is read); otherwise the full product is emitted.
  double sym_tiles(GemmTask t) {
    if (t.beta != 0.0 && t.d < 0) return tiles(t, 0, 0, false);
    t.sym = 1;
    return tiles(t, 0, 0, true);
  }

  // Blocked right-looking factorisation of tall panels [diag n x n; m_below rows;
  // optional identity rows], 64 columns per step: diagonal Cholesky + inverse, the
  // rows below times the inverse (in place), then the trailing update.
  static PotrfTask potrf_task(const PanelDesc& p, int32_t d0) {
    PotrfTask t{};
    t.panel = p.off; t.inv = p.dinv + (int64_t)(d0 / kTile) * 4096; t.ld = p.ld;
    t.nb = std::min(kTile, p.n - d0); t.d0 = d0; t.sn = p.sn; t.mode = p.mode;
    t.scale_off = p.scale_off;
    t.mrow = one_block(p) ? p.n : 0;
    return t;
  }
  // a panel of one 64-column block over identity rows only: POTRF stores M itself
  static bool one_block(const PanelDesc& p) { return p.ident && p.m_below == 0 && p.n <= kTile; }

  // Inside an outer block the next step's diagonal block is last updated by one tile of
  // this step's in-block trailing launch; that tile's workgroup factors it right after
  // storing it (GemmTask::potrf1), so only the first step of each outer block has a POTRF
  // launch of its own.  (The wide outer launches keep the plain kernel: the fused one
  // holds twice the LDS, which would cost them a third of their workgroups per CU.)
  void panel_steps(const std::vector<PanelDesc>& pan) {
    int32_t maxn = 0;
    for (auto& p : pan) maxn = std::max(maxn, p.n);
    const bool fuse = h.opt.gemm_tile != 128;   // (a fixed 128 edge merges the tiles)
    std::vector<char> fused(pan.size(), 0);     // panel's POTRF of this step already placed
    for (int32_t d0 = 0; d0 < maxn; d0 += kTile) {
      // blocks of at most 32 columns in a launch of the 32-edge kernel (when there are
      // enough of them to fill the chip several times), the rest after
      int64_t nsmall = 0;
      for (size_t pi = 0; pi < pan.size(); ++pi)
        if (pan[pi].n > d0 && !fused[pi] && std::min(kTile, pan[pi].n - d0) <= 32) ++nsmall;
      const bool split = nsmall >= 1024;
      for (int edge : {32, 64}) {
        if (edge == 32 && !split) continue;
        const int64_t q0 = (int64_t)P.potrf.size();
        double fl = 0;
        for (size_t pi = 0; pi < pan.size(); ++pi) {
          const PanelDesc& p = pan[pi];
          if (p.n <= d0 || fused[pi]) continue;
          const int32_t nb = std::min(kTile, p.n - d0);
          if (split && (nb <= 32) != (edge == 32)) continue;
          P.potrf.push_back(potrf_task(p, d0));
          fl += std::pow((double)nb, 3) / 3.0;
        }
        int32_t nbmax = 0;
        for (int64_t q = q0; q < (int64_t)P.potrf.size(); ++q) nbmax = std::max(nbmax, P.potrf[q].nb);
        cmd(kCmdPotrf, RSC_K_POTRF, q0, (int64_t)P.potrf.size() - q0, fl, nbmax <= 32 ? 32 : 64);
      }
      std::fill(fused.begin(), fused.end(), 0);
      // rows below the diagonal block times its inverse, then the trailing update in two
      // levels: each 64-column step updates the columns of its kOuter-wide block, and the
      // block's last step adds the whole block (K = kOuter) to the columns right of it,
      // so the wide trailing matrix is read and written once per kOuter columns;
      // rows inside [lp_lo, lp_hi) go to the low-precision launch
      const int32_t dend = (d0 / kOuter + 1) * kOuter;   // end of this step's outer block
      for (int phase = 0; phase < 3; ++phase) {
        if (phase == 2 && d0 + kTile != dend) continue;
        std::vector<GemmTask> hi_t, lo_t, tl_t;
        double fh = 0, flo = 0, ftl = 0;
        for (size_t pi = 0; pi < pan.size(); ++pi) {
          const PanelDesc& p = pan[pi];
          if (p.n <= d0) continue;
          const size_t h0 = hi_t.size();
          const int32_t nb = std::min(kTile, p.n - d0);
          if (phase == 0 && one_block(p)) continue;
          if (phase >= 1 && p.n <= d0 + nb) continue;
          if (phase == 1 && d0 + nb >= dend) continue;      // no columns left in the block
          const int32_t R0 = (phase == 2) ? dend : d0 + nb;
          const int32_t R1 = p.n + p.m_below + (p.ident ? std::min(p.n, d0 + nb) : 0);
          const int64_t colb = p.off + (int64_t)d0 * p.ld;
          const int64_t colo = p.off + (int64_t)(dend - kOuter) * p.ld;
          GemmTask t = (phase == 0)
              ? gt(colb, 1, p.ld, p.dinv + (int64_t)(d0 / kTile) * 4096, 1, kTile, colb, p.ld, R1, nb, nb, 1.0, 0.0)
              : (phase == 1)
              ? gt(colb, 1, p.ld, colb, 1, p.ld, p.off, p.ld, R1, std::min(p.n, dend), nb, -1.0, 1.0)
              : gt(colo, 1, p.ld, colo, 1, p.ld, p.off, p.ld, R1, p.n, kOuter, -1.0, 1.0);
          const int32_t jb = (phase == 0) ? 0 : (phase == 1) ? d0 + nb : dend;
          const bool lower = (phase >= 1);
          const bool use_lp = ((lp_update || p.skip_mid) && p.lp_hi > p.lp_lo) || (p.tail_lp && lp_tri);
          // segments [R0, lp_lo), [lp_lo, lp_hi), [lp_hi, R1)
          int32_t cuts[4] = {R0, use_lp ? std::max(R0, p.lp_lo) : R1, use_lp ? std::max(R0, p.lp_hi) : R1, R1};
          for (int sgm = 0; sgm < 3; ++sgm) {
            const int32_t lo = cuts[sgm], hi = std::min(cuts[sgm + 1], R1);
            if (hi <= lo) continue;
            GemmTask ts = t;
            ts.m = hi;
            if (sgm == 1 && p.skip_mid) continue;
            if (sgm == 1) flo += tiles(ts, lo, jb, lower, &lo_t);
            else if (sgm == 2 && p.tail_lp && lp_tri) ftl += tiles(ts, lo, jb, lower, &tl_t);
            else fh += tiles(ts, lo, jb, lower, &hi_t);
          }
          const int32_t nd = d0 + kTile;   // the next step's diagonal block
          if (fuse && phase == 1 && p.n > nd && nd < dend)
            for (size_t q = h0; q < hi_t.size(); ++q)
              if (hi_t[q].i0 == nd && hi_t[q].j0 == nd) {
                hi_t[q].potrf1 = (int32_t)P.potrf.size() + 1;
                P.potrf.push_back(potrf_task(p, nd));
                fh += std::pow((double)P.potrf.back().nb, 3) / 3.0;
                fused[pi] = 1;
                break;
              }
        }
        // the diagonal blocks' workgroups first: they have the factorization still to do
        std::stable_partition(hi_t.begin(), hi_t.end(), [](const GemmTask& t) { return t.potrf1 > 0; });
        const bool post = !hi_t.empty() && hi_t.front().potrf1 > 0;
        const int klass = phase == 0 ? RSC_K_TRSM : RSC_K_GEMM;
        int64_t g0 = (int64_t)P.gemm.size();
        P.gemm.insert(P.gemm.end(), hi_t.begin(), hi_t.end());
        next_post = post;
        cmd(kCmdGemm, klass, g0, (int64_t)hi_t.size(), fh, 0);
        g0 = (int64_t)P.gemm.size();
        P.gemm.insert(P.gemm.end(), lo_t.begin(), lo_t.end());
        cmd(kCmdGemm, klass, g0, (int64_t)lo_t.size(), flo, lp_update);
        g0 = (int64_t)P.gemm.size();
        P.gemm.insert(P.gemm.end(), tl_t.begin(), tl_t.end());
        cmd(kCmdGemm, klass, g0, (int64_t)tl_t.size(), ftl, lp_tri);
      }
    }
  }

  // L^O_j = U^O_j (L^D_j)^{-T} = U^O_j M_j with the upper-triangular M_j = (L^D_j)^{-T}
  // that the panel factorisation left in the panel's last c rows; column block j0 of
  // the product only needs rows k < j0 + 64 of M.  U^O_j comes from the level pool.
  void offdiag_solve(const std::vector<int32_t>& level) {
    const Symbolic& S = h.S;
    const int64_t g0 = (int64_t)P.gemm.size();
    const size_t c0 = P.cmds.size();
    double fl = 0, mfl = 0;
    for (int32_t j : level) {
      const int32_t c = S.c(j), r = S.r(j), ld = h.panel_ld[j];
      if (r == 0) continue;
      // a compressed supernode's L^O_j is only reached through the implicit products
      // of Algorithm 2 (formed here only when kept for inspection, and not credited)
      const bool implicit = P.compressed && h.compressible[j];
      if (implicit && !h.opt.keep_lo) continue;
      const int64_t pan = h.panel_off[j];
      if (!implicit) mfl += (double)r * c * c;
      GemmTask t = gt(h.uo_off[j], 1, r, pan + c, ld, 1, h.lo_off[j], r, r, c, c, 1.0, 0.0);
      for (int32_t j0 = 0; j0 < c; j0 += kTile)
        for (int32_t i0 = 0; i0 < r; i0 += kTile) {
          GemmTask u = t;
          u.i0 = i0; u.j0 = j0; u.k = std::min(c, j0 + kTile);
          P.gemm.push_back(u);
          fl += 2.0 * std::min(kTile, r - i0) * std::min(kTile, c - j0) * (double)u.k;
        }
    }
    cmd(kCmdGemm, RSC_K_LO, g0, (int64_t)P.gemm.size() - g0, fl, lp_update);
    credit(c0, mfl);
  }

  // Schur-complement updates of every supernode of one level (Algorithm 1, the
  // descendant loop), as target tiles with ordered contribution lists.
  void updates(const std::vector<int32_t>& level) {
    const Symbolic& S = h.S;
    struct TileW { UpdTile t; double work; std::vector<UpdEntry> e; std::vector<double> ke, lw; };
    std::vector<TileW> all;
    for (int32_t j : level) {
      const int32_t c = S.c(j), r = S.r(j);
      // row tiles: 64-row blocks of C_j (in the panel), then of R_j (U^O_j in the pool);
      // no tile straddles the two
      const int32_t nIc = (c + kTile - 1) / kTile, nJ = nIc;
      const int32_t nI = nIc + (r + kTile - 1) / kTile;
      auto tile_of = [&](int32_t x) { return x < c ? x / kTile : nIc + (x - c) / kTile; };
      std::vector<std::vector<UpdEntry>> ents((size_t)nI * nJ);
      std::vector<std::vector<double>> kes((size_t)nI * nJ);   // planning inner dimension
      std::vector<std::vector<double>> lws((size_t)nI * nJ);   // pairs on or below the diagonal
      std::vector<double> work((size_t)nI * nJ, 0.0);
      for (int64_t q = S.pair_ptr[j]; q < S.pair_ptr[j + 1]; ++q) {
        const Pair& pr = S.pairs[q];
        const int32_t k = pr.k;
        UpdEntry base{};
        double kest;
        if (P.compressed && h.compressible[k]) {
          base.kdim = -(1 + h.comp[k].qslot);
          kest = h.comp[k].ell;
        } else {
          base.kdim = S.c(k);
          kest = S.c(k);
        }
        // the compact copy of V_k or L^O_k, shifted to the pair's rows (ldx in the copy's
        // element type)
        base.x = xc_off[k] + (int64_t)pr.p0 * xc_row(k);
        base.ldx = (lp_update == 2 ? 2 : 1) * xc_kp[k];
        base.map = pr.map_off;
        const int32_t* rm = S.relmap.data() + pr.map_off;
        // runs of gathered rows per 64-row tile (relmap is increasing)
        std::vector<std::array<int32_t, 3>> rr, cc;
        for (int32_t t = 0; t < pr.nrows;) {
          const int32_t I = tile_of(rm[t]);
          int32_t u = t;
          while (u < pr.nrows && tile_of(rm[u]) == I) ++u;
          rr.push_back({I, t, u});
          t = u;
        }
        for (int32_t t = 0; t < pr.nD;) {
          const int32_t J = rm[t] / kTile;
          int32_t u = t;
          while (u < pr.nD && rm[u] / kTile == J) ++u;
          cc.push_back({J, t, u});
          t = u;
        }
        for (auto& R : rr)
          for (auto& Cc : cc) {
            if (R[0] < Cc[0]) continue;   // tile strictly above the diagonal
            UpdEntry e = base;
            e.a = R[1]; e.b = R[2]; e.c = Cc[1]; e.d = Cc[2];
            const size_t id = (size_t)R[0] * nJ + Cc[0];
            // SYRK lower half in a diagonal tile (gathered row t >= column s), else all
            double lw = (double)(e.b - e.a) * (e.d - e.c);
            if (R[0] == Cc[0]) {
              lw = 0;
              for (int32_t s2 = e.c; s2 < e.d; ++s2) lw += std::max(0, e.b - std::max(e.a, s2));
            }
            ents[id].push_back(e);
            kes[id].push_back(kest);
            lws[id].push_back(lw);
            work[id] += 2.0 * (e.b - e.a) * (e.d - e.c) * kest;
          }
      }
      for (int32_t I = 0; I < nI; ++I)
        for (int32_t J = 0; J < nJ; ++J) {
          const size_t id = (size_t)I * nJ + J;
          if (ents[id].empty()) continue;
          TileW tw;
          if (I < nIc) {       // target rows in C_j: the panel
            tw.t.panel = h.panel_off[j];
            tw.t.ld = h.panel_ld[j];
            tw.t.row0 = I * kTile;
            tw.t.nrows = std::min(kTile, c - I * kTile);
          } else {             // rows of R_j: U^O_j, addressed so that row c is its first row
            tw.t.panel = h.uo_off[j] - c;
            tw.t.ld = r;
            tw.t.row0 = c + (I - nIc) * kTile;
            tw.t.nrows = std::min(kTile, c + r - tw.t.row0);
          }
          tw.t.col0 = J * kTile;
          tw.t.ncols = std::min(kTile, c - J * kTile);
          tw.work = work[id];
          tw.e = std::move(ents[id]);
          tw.ke = std::move(kes[id]);
          tw.lw = std::move(lws[id]);
          all.push_back(std::move(tw));
        }
    }
    if (all.empty()) return;
    // heaviest tiles first: the long ones start early and the tail is short
    std::stable_sort(all.begin(), all.end(), [](const TileW& x, const TileW& y) { return x.work > y.work; });
    // within a tile: entries wider than 32 first (list order), then the others by
    // decreasing inner dimension, so that the four entries taken together are alike
    const int64_t t0 = (int64_t)P.tiles.size();
    double fl = 0, mfl = 0;
    bool dyn = false;
    for (auto& tw : all) {
      std::vector<int32_t> idx(tw.e.size());
      for (size_t q = 0; q < idx.size(); ++q) idx[q] = (int32_t)q;
      auto big = [&](int32_t q) { return tw.e[q].b - tw.e[q].a > 32 || tw.e[q].d - tw.e[q].c > 32; };
      std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
        const bool bx = big(x), by = big(y);
        if (bx != by) return bx;
        return !bx && tw.ke[x] > tw.ke[y];
      });
      tw.t.e0 = (int32_t)P.ents.size();
      tw.t.es = tw.t.e0;
      for (int32_t q : idx) {
        const UpdEntry& e = tw.e[q];
        if (big(q)) ++tw.t.es;
        fl += 2.0 * (e.b - e.a) * (e.d - e.c) * tw.ke[q];
        mfl += 2.0 * tw.lw[q] * tw.ke[q];
        dyn |= (e.kdim < 0);
        P.ents.push_back(e);
        P.ent_lower.push_back(tw.lw[q]);
      }
      tw.t.e1 = (int32_t)P.ents.size();
      P.tiles.push_back(tw.t);
    }
    cmd(kCmdUpdate, RSC_K_UPDATE, t0, (int64_t)P.tiles.size() - t0, fl, lp_update);
    P.cmds.back().dyn = dyn;
    P.cmds.back().mflops = mfl;
    P.cmds.back().mkind = 1;
  }

  // Compact row-major copies of the Schur-update operands of a level once they are
  // final: L^O_j of the supernodes kept explicit, V_j of the compressed.
  void compact_operands(const std::vector<int32_t>& level, bool compressed_ones) {
    const Symbolic& S = h.S;
    const int64_t c0 = (int64_t)P.compact.size();
    for (int32_t j : level) {
      const int32_t r = S.r(j);
      if (r == 0 || xc_off[j] < 0) continue;
      const bool comp = P.compressed && h.compressible[j];
      if (comp != compressed_ones) continue;
      for (int32_t r0 = 0; r0 < r; r0 += kTile) {
        CompactTask t{};
        t.src = (comp ? h.comp[j].Vj : h.lo_off[j]) + r0;
        t.dst = xc_off[j] + (int64_t)r0 * xc_row(j);
        t.ld = r;
        t.nrows = std::min(kTile, r - r0);
        t.kdim = comp ? -(1 + h.comp[j].qslot) : S.c(j);
        t.kp = xc_kp[j];
        // (an interior supernode's L^O_j sits in the level pool: the factor's FP32 copy
        // takes only its rows inside the block, from their own storage)
        t.f32 = in_block(j) ? -1 : t.src;
        P.compact.push_back(t);
      }
    }
    cmd(kCmdCompact, RSC_K_UPDATE, c0, (int64_t)P.compact.size() - c0, 0.0, lp_update);
  }

  // the rows of each interior supernode's L^O_j inside its block, from the level pool to
  // the factor's own storage
  bool in_block(int64_t j) const { return P.compressed && h.opt.interior && h.iroot[j] >= 0 && h.S.r(j) > 0; }
  void interior_copy(const std::vector<int32_t>& level) {
    const Symbolic& S = h.S;
    const int64_t c0 = (int64_t)P.copy.size();
    for (int32_t j : level) {
      if (!in_block(j) || h.r_in[j] == 0) continue;
      const int32_t c = S.c(j), r = S.r(j), ri = h.r_in[j];
      for (int32_t j0 = 0; j0 < c; j0 += 64)
        for (int32_t i0 = 0; i0 < ri; i0 += kConvRows)
          P.copy.push_back(ConvTask{h.lo_off[j] + i0 + (int64_t)j0 * r, h.lo_in[j] + i0 + (int64_t)j0 * ri,
                                    std::min(kConvRows, ri - i0), std::min(64, c - j0), r, ri});
    }
    cmd(kCmdCopy, RSC_K_OTHER, c0, (int64_t)P.copy.size() - c0, 0.0, 0);
  }

  // FP32 copy (mixed forms) of the factor operands the two sweeps of the preconditioner
  // read: the inverse diagonal blocks M_j as compact c x c blocks, W_j at its arena
  // offsets (L^O_j and V_j are copied by k_compact_rows along with their compact copies);
  // blocks of at most 64 columns and kConvRows rows.
  void f32_copy() {
    const Symbolic& S = h.S;
    const int64_t c0 = (int64_t)P.conv.size();
    // upper: only rows above the column block's end (M_j is upper triangular)
    auto add = [&](int64_t off, int32_t ld, int64_t dst, int32_t dld, int32_t rows, int32_t cols, bool upper) {
      for (int32_t j0 = 0; j0 < cols; j0 += 64) {
        const int32_t rr = upper ? std::min(rows, j0 + 64) : rows;
        for (int32_t i0 = 0; i0 < rr; i0 += kConvRows)
          P.conv.push_back(ConvTask{off + i0 + (int64_t)j0 * ld, dst + i0 + (int64_t)j0 * dld,
                                    std::min(kConvRows, rr - i0), std::min(64, cols - j0), ld, dld});
      }
    };
    for (int64_t j = 0; j < S.M(); ++j) {
      const int32_t c = S.c(j), r = S.r(j);
      add(h.panel_off[j] + c, h.panel_ld[j], h.m32_off[j], c, c, c, true);
      if (r == 0) continue;
      if (P.compressed && h.compressible[j]) add(h.comp[j].Uj, c, h.comp[j].Uj, c, c, h.comp[j].ell, false);
      if (in_block(j) && h.r_in[j] > 0) add(h.lo_in[j], h.r_in[j], h.lo_in[j], h.r_in[j], h.r_in[j], c, false);
    }
    cmd(kCmdToF32, RSC_K_OTHER, c0, (int64_t)P.conv.size() - c0, 0.0, 0);
  }

  // One Cholesky-QR pass over the sample panels of a level (Y: rows [l, l + c) of the
  // panel [Gram; Y], or with zp the power iteration's Z = L^O Y, rows [l, l + r) of its
  // panel): Gram = Y^T Y (lower tiles), the drop scale (and with shifted, the shift of
  // shifted Cholesky-QR), then the blocked panel factorisation, which leaves Y R^{-1}.
  // One Cholesky-QR pass over panels [Gram (l x l); Y (m x l)] (ld l + m): the Gram
  // matrix Y^T Y, its diagonal scaling (and shift), then the panel factorisation whose
  // rows below turn Y into Y R^{-1} (dependent columns dropped).
  struct QRPanel { int64_t pnl; int32_t l, m; int64_t dinv; int32_t sn; int64_t sc; };
  void cholqr(const std::vector<QRPanel>& qs, bool shifted) {
    const int64_t g0 = (int64_t)P.gemm.size();
    double fl = 0;
    const int64_t s0 = (int64_t)P.gs_g.size();
    std::vector<PanelDesc> pan;
    for (const QRPanel& q : qs) {
      const int32_t l = q.l, m = q.m, ld = l + m;
      fl += tiles(gt(q.pnl + l, ld, 1, q.pnl + l, ld, 1, q.pnl, ld, l, l, m, 1.0, 0.0), 0, 0, true);
      P.gs_g.push_back(q.pnl); P.gs_ld.push_back(ld); P.gs_n.push_back(l); P.gs_out.push_back(q.sc);
      P.gs_m.push_back(shifted ? m : 0);
      pan.push_back(PanelDesc{q.pnl, ld, l, m, false, q.dinv, q.sn, 1, q.sc});
    }
    cmd(kCmdGemm, RSC_K_GEMM, g0, (int64_t)P.gemm.size() - g0, fl);
    cmd(kCmdGramScale, RSC_K_OTHER, s0, (int64_t)P.gs_g.size() - s0, 0);
    panel_steps(pan);
  }
  void cholqr_pass(const std::vector<int32_t>& js, bool zp, bool shifted) {
    const Symbolic& S = h.S;
    std::vector<QRPanel> qs;
    for (int32_t j : js) {
      const CompSlot& C = h.comp[j];
      qs.push_back(QRPanel{zp ? C.zpanel : C.ypanel, C.ell, zp ? S.r(j) : S.c(j), zp ? C.zdinv : C.ydinv,
                           j, zp ? C.gscale + 1 : C.gscale});
    }
    cholqr(qs, shifted);
  }

  // Algorithm 2 on the device.  Its descendant terms, summed over k, are the rows R_j of
  // the Schur update: the update launch accumulates them once per supernode into U^O_j
  // (level pool) instead of re-forming them for every product, so
  //   L^O_j G = U^O_j ((L^D_j)^{-T} G) = U^O_j (M_j G)   and   (L^O_j)^T G = M_j^T (U^O_j^T G),
  // with M_j = (L^D_j)^{-T} the inverse the panel factorisation leaves in rows [c, 2c) of
  // the panel.  L^O_j (r x c) and the r c^2 solve that forms it are never needed.
  // A product's operands: src (rows x l, column-major, ld) -> dst; the launch mode `mode`.
  struct Blk { int64_t off; int32_t ld; };
  // dst = M_j src (c x l): M_j upper triangular, row tile i0 needs k >= i0 (operands shifted)
  double emit_M(const std::vector<int32_t>& js, const std::function<Blk(int32_t)>& src,
                const std::function<Blk(int32_t)>& dst, int mode) {
    const Symbolic& S = h.S;
    const int64_t g0 = (int64_t)P.gemm.size();
    double fl = 0;
    for (int32_t j : js) {
      const int32_t c = S.c(j), l = h.comp[j].ell, ldp = h.panel_ld[j];
      const Blk s = src(j), d = dst(j);
      const int64_t Mp = h.panel_off[j] + c;      // M(i, k) at Mp + i + k ldp
      for (int32_t j0 = 0; j0 < l; j0 += kTile)
        for (int32_t i0 = 0; i0 < c; i0 += kTile) {
          GemmTask t = gt(Mp + (int64_t)i0 * ldp, 1, ldp, s.off + i0, s.ld, 1, d.off, d.ld, c, l, c - i0, 1.0, 0.0);
          t.i0 = i0; t.j0 = j0;
          P.gemm.push_back(t);
          fl += 2.0 * std::min(kTile, c - i0) * std::min(kTile, l - j0) * (double)(c - i0);
        }
    }
    cmd(kCmdGemm, RSC_K_GEMM, g0, (int64_t)P.gemm.size() - g0, fl, mode);
    return fl;
  }
  // dst = M_j^T src (c x l): M_j^T lower triangular, row tile i0 needs k < i0 + 64
  double emit_MT(const std::vector<int32_t>& js, const std::function<Blk(int32_t)>& src,
                 const std::function<Blk(int32_t)>& dst, int mode) {
    const Symbolic& S = h.S;
    const int64_t g0 = (int64_t)P.gemm.size();
    double fl = 0;
    for (int32_t j : js) {
      const int32_t c = S.c(j), l = h.comp[j].ell, ldp = h.panel_ld[j];
      const Blk s = src(j), d = dst(j);
      const int64_t Mp = h.panel_off[j] + c;      // M^T(i, k) = M(k, i) at Mp + k + i ldp
      for (int32_t j0 = 0; j0 < l; j0 += kTile)
        for (int32_t i0 = 0; i0 < c; i0 += kTile) {
          GemmTask t = gt(Mp, ldp, 1, s.off, s.ld, 1, d.off, d.ld, c, l, std::min(c, i0 + kTile), 1.0, 0.0);
          t.i0 = i0; t.j0 = j0;
          P.gemm.push_back(t);
          fl += 2.0 * std::min(kTile, c - i0) * std::min(kTile, l - j0) * (double)t.k;
        }
    }
    cmd(kCmdGemm, RSC_K_GEMM, g0, (int64_t)P.gemm.size() - g0, fl, mode);
    return fl;
  }
  // dst = U^O_j src (r x l, src c x l) or, with trans, dst = (U^O_j)^T src (c x l, src r x l)
  double emit_UO(const std::vector<int32_t>& js, bool trans, const std::function<Blk(int32_t)>& src,
                 const std::function<Blk(int32_t)>& dst, int mode) {
    const Symbolic& S = h.S;
    const int64_t g0 = (int64_t)P.gemm.size();
    double fl = 0;
    for (int32_t j : js) {
      const int32_t c = S.c(j), r = S.r(j), l = h.comp[j].ell;
      const Blk s = src(j), d = dst(j);
      const int64_t uo = h.uo_off[j];             // U^O(i, k) at uo + i + k r
      fl += trans ? tiles(gt(uo, r, 1, s.off, s.ld, 1, d.off, d.ld, c, l, r, 1.0, 0.0), 0, 0, false)
                  : tiles(gt(uo, 1, r, s.off, s.ld, 1, d.off, d.ld, r, l, c, 1.0, 0.0), 0, 0, false);
    }
    cmd(kCmdGemm, RSC_K_GEMM, g0, (int64_t)P.gemm.size() - g0, fl, mode);
    return fl;
  }

  // Algorithm 3 for every compressible supernode of a level, its products with L^O_j
  // formed implicitly (Algorithm 2, above), followed by the spectral truncation.
  void compression(const std::vector<int32_t>& level, double tol) {
    const Symbolic& S = h.S;
    std::vector<int32_t> js;
    for (int32_t j : level)
      if (h.compressible[j]) js.push_back(j);
    if (js.empty()) return;
    ctx = RSC_K_SAMPLE;
    // algorithmic work of the steps (summed over the level's compressible supernodes)
    double m_prod = 0, m_orth = 0, m_gram = 0, m_eig = 0, m_diag = 0;
    for (int32_t j : js) {
      const double c = S.c(j), r = S.r(j), l = h.comp[j].ell;
      m_prod += 2.0 * r * c * l;       // one product with L^O_j or its transpose
      m_diag += c * c * l;             // Algorithm 2's diagonal solve of a c x l operand
      m_orth += 2.0 * c * l * l;       // orthonormalisation of the c x l sample
      m_gram += 2.0 * r * l * l;       // Gram matrix of V
      m_eig += 9.0 * l * l * l;        // symmetric eigen-decomposition of the l x l Gram matrix
    }
    size_t cs = P.cmds.size();
    // 1. Gaussian samples
    const int64_t ph0 = (int64_t)P.philox.size();
    int64_t maxw = 0;
    for (int32_t j : js) {
      const CompSlot& C = h.comp[j];
      PhiloxTask t{};
      t.out = C.omega; t.rows = S.r(j); t.cols = C.ell;
      t.k0 = (uint32_t)(h.opt.seed & 0xFFFFFFFFull);
      t.k1 = (uint32_t)(((h.opt.seed >> 32) & 0xFFFFFFFFull) ^ (uint64_t)(uint32_t)h.sn_local[j]);
      P.philox.push_back(t);
      maxw = std::max<int64_t>(maxw, (int64_t)S.r(j) * ((C.ell + 3) / 4));
    }
    // the mixed forms round the sample to BF16 in the product: the transform runs in FP32
    cmd(kCmdPhilox, RSC_K_OTHER, ph0, (int64_t)P.philox.size() - ph0, 0, maxw, lp_sample ? 1 : 0);
    // 2. Y = (L^O_j)^T Omega = M_j^T (U^O_j^T Omega) into rows [l, l + c) of the
    //    orthonormalisation panel (the intermediate in the c x l work block `tmp`)
    auto omega = [&](int32_t j) { return Blk{h.comp[j].omega, S.r(j)}; };
    auto tmpb = [&](int32_t j) { return Blk{h.comp[j].tmp, S.c(j)}; };
    auto ybl = [&](int32_t j) { return Blk{h.comp[j].ypanel + h.comp[j].ell, h.comp[j].ell + S.c(j)}; };
    auto zbl = [&](int32_t j) { return Blk{h.comp[j].zpanel + h.comp[j].ell, h.comp[j].ell + S.r(j)}; };
    auto vbl = [&](int32_t j) { return Blk{h.comp[j].V, S.r(j)}; };
    emit_UO(js, true, omega, tmpb, lp_sample);
    credit(cs, m_prod);
    cs = P.cmds.size();
    emit_MT(js, tmpb, ybl, lp_update);
    credit(cs, m_diag);
    int64_t g0;
    double fl;
    // 3. power iterations Y = (L^O)^T (L^O Y).  Each product is preceded by one shifted
    //    Cholesky-QR pass over its operand: the span is unchanged (a right factor), but the
    //    operand's spread of singular values no longer compounds over the iterations, so
    //    no direction that the final orthonormalisation would keep sinks below rounding.
    for (int it = 0; it < h.opt.power_iters; ++it) {
      cholqr_pass(js, false, true);
      cs = P.cmds.size();
      emit_M(js, ybl, tmpb, 0);                // Z = L^O Y = U^O (M Y)
      credit(cs, m_diag);
      cs = P.cmds.size();
      emit_UO(js, false, tmpb, zbl, 0);
      credit(cs, m_prod);
      cholqr_pass(js, true, true);
      cs = P.cmds.size();
      emit_UO(js, true, zbl, tmpb, 0);         // Y = (L^O)^T Z = M^T (U^O^T Z)
      credit(cs, m_prod);
      cs = P.cmds.size();
      emit_MT(js, tmpb, ybl, 0);
      credit(cs, m_diag);
    }
    ctx = RSC_K_ORTH;
    // 4. orthonormalisation by Cholesky-QR passes, dependent columns dropped.  Two plain
    //    passes (the first leaves a condition number below ~1e7, the second restores
    //    orthogonality) lose the directions of Y below ~1e-7 of its largest, i.e. singular
    //    values of L^O_j below ~1e-6 sigma_1: harmless for tol >= 1e-5.  Below that the first
    //    pass is shifted (shifted Cholesky-QR3: three passes), which keeps every direction
    //    above the rounding of Y.
    const bool accurate = tol < 1e-5;
    cs = P.cmds.size();
    for (int pass = 0; pass < (accurate ? 3 : 2); ++pass) cholqr_pass(js, false, accurate && pass == 0);
    credit(cs, m_orth);
    ctx = RSC_K_BASIS;
    // 5. V = L^O_j U (FP32 MFMA in the mixed forms, like the other basis products: its
    //    rounding, ~1e-7 of |V|, is far below the truncation threshold tol^2 lambda_max)
    cs = P.cmds.size();
    emit_M(js, ybl, tmpb, lp_eig);             // V = L^O U = U^O (M U)
    credit(cs, m_diag);
    cs = P.cmds.size();
    emit_UO(js, false, tmpb, vbl, lp_eig);
    credit(cs, m_prod);
    ctx = RSC_K_EIG;
    // 6. Gram G = V^T V (full)
    cs = P.cmds.size();
    g0 = (int64_t)P.gemm.size(); fl = 0;
    for (int32_t j : js) {
      const CompSlot& C = h.comp[j];
      const int32_t r = S.r(j), l = C.ell;
      fl += sym_tiles(gt(C.V, r, 1, C.V, r, 1, C.G, l, l, l, r, 1.0, 0.0));
    }
    cmd(kCmdGemm, RSC_K_GEMM, g0, (int64_t)P.gemm.size() - g0, fl);
    credit(cs, m_gram);
    cs = P.cmds.size();   // the eigen-truncation's launches, up to the kept basis
    // 7. spectral projector onto lambda > tol^2 lambda_max (see the truncation kernels)
    const int64_t t0 = (int64_t)P.trunc.size();
    for (int32_t j : js) {
      const CompSlot& C = h.comp[j];
      TruncTask t{};
      t.g = C.G; t.sa = C.Sa; t.sb = C.Sb; t.mpan = C.Mpan; t.wpan = C.Wpan; t.sc = C.sc;
      t.wout = C.Om2;
      t.l = C.ell; t.qslot = C.qslot; t.tol = tol;
      P.trunc.push_back(t);
    }
    const int64_t nt = (int64_t)P.trunc.size() - t0;
    auto sq_gemm = [&](bool a_to_b, double alpha, double beta, int64_t dsel) {
      // C = alpha X Y^T (+ beta D) on every problem's l x l blocks; X = Y symmetric
      const int64_t gg = (int64_t)P.gemm.size();
      double f = 0;
      for (int32_t j : js) {
        const CompSlot& C = h.comp[j];
        const int32_t l = C.ell;
        const int64_t src = a_to_b ? C.Sa : C.Sb, dst = a_to_b ? C.Sb : C.Sa;
        GemmTask t = gt(src, 1, l, src, 1, l, dst, l, l, l, l, alpha, beta);
        (void)dsel;
        f += sym_tiles(t);
      }
      // FP64: (G / tr G)^32 would underflow FP32 when lambda_max is a small share of tr G
      cmd(kCmdGemm, RSC_K_EIG, gg, (int64_t)P.gemm.size() - gg, f);
    };
    cmd(kCmdTruncPrep, RSC_K_EIG, t0, nt, 0);          // sa = G / tr G
    for (int k = 0; k < 5; ++k) sq_gemm(k % 2 == 0, 1.0, 0.0, -1);   // sb = (G / tr G)^32
    {
      // lambda_max, theta: one workgroup per supernode, or for large l each product of
      // the power iteration as its own launch over 64-row blocks
      int32_t lmax = 0;
      for (int32_t j : js) lmax = std::max(lmax, h.comp[j].ell);
      if (lmax > kPowerRowsMin) {
        for (int32_t it = 0; it <= 5; ++it) cmd(kCmdTruncPower, RSC_K_EIG, t0, nt, 0, lmax, it);
      } else {
        cmd(kCmdTruncPower, RSC_K_EIG, t0, nt, 0);
      }
    }
    cmd(kCmdTruncMfill, RSC_K_EIG, t0, nt, 0);         // [G + theta I; I]
    {
      std::vector<PanelDesc> pan;
      for (int32_t j : js) {
        const CompSlot& C = h.comp[j];
        pan.push_back(PanelDesc{C.Mpan, 2 * C.ell, C.ell, 0, true, C.Mdinv, j, 1, C.sc + 3});
      }
      panel_steps(pan);                                 // rows [l, 2l) become L^{-T}
    }
    // H = (G + theta I)^{-1} = L^{-T} L^{-1} into sb
    g0 = (int64_t)P.gemm.size(); fl = 0;
    for (int32_t j : js) {
      const CompSlot& C = h.comp[j];
      const int32_t l = C.ell;
      fl += sym_tiles(gt(C.Mpan + l, 1, 2 * l, C.Mpan + l, 1, 2 * l, C.Sb, l, l, l, l, 1.0, 0.0));
    }
    cmd(kCmdGemm, RSC_K_EIG, g0, (int64_t)P.gemm.size() - g0, fl);
    cmd(kCmdTruncX0, RSC_K_EIG, t0, nt, 0);            // sa = I - 2 theta H
    // a level whose supernodes all have l <= nsmax runs every step in one workgroup per
    // supernode (k_trunc_ns); any other level, all of it by product launches (whose count
    // does not depend on how many supernodes they hold, so splitting a level would only
    // add the in-LDS launch to them)
    int32_t nsmax = lp_eig ? kNsMaxF32 : kNsMaxF64;
    {
      int32_t lmax = 0;
      double f = 0;
      for (int32_t j : js) {
        lmax = std::max(lmax, h.comp[j].ell);
        f += 2.0 * kNs.steps * std::pow((double)h.comp[j].ell, 3);
      }
      if (lmax <= nsmax) cmd(kCmdTruncNs, RSC_K_EIG, t0, nt, f, lp_eig ? 1 : 0);
      else nsmax = 0;
    }
    for (int it = 0; nsmax == 0 && it < kNs.steps; ++it) {
      const double a = kNs.alpha[it];
      // sb = X X ; X_new = 1.5 X - 0.5 X sb (into sb via the D operand, then swap roles).
      // The right operands are passed transposed (B(j, k) = Y(k, j)) so that the products
      // are X X and X (X X): with X X^T in their place the iteration doubles the
      // antisymmetric part of its rounding error on every step.
      g0 = (int64_t)P.gemm.size(); fl = 0;
      const bool even = (it % 2 == 0);
      for (int32_t j : js) {
        const CompSlot& C = h.comp[j];
        const int32_t l = C.ell;
        if (l <= nsmax) continue;
        const int64_t X = even ? C.Sa : C.Sb;
        fl += sym_tiles(gt(X, 1, l, X, l, 1, C.Om2, l, l, l, l, 1.0, 0.0));
      }
      cmd(kCmdGemm, RSC_K_EIG, g0, (int64_t)P.gemm.size() - g0, fl, lp_eig);
      g0 = (int64_t)P.gemm.size(); fl = 0;
      for (int32_t j : js) {
        const CompSlot& C = h.comp[j];
        const int32_t l = C.ell;
        if (l <= nsmax) continue;
        const int64_t X = even ? C.Sa : C.Sb, Xn = even ? C.Sb : C.Sa;
        GemmTask t = gt(X, 1, l, C.Om2, l, 1, Xn, l, l, l, l, -0.5 * a * a * a, 1.5 * a);
        t.d = X;
        fl += sym_tiles(t);
      }
      cmd(kCmdGemm, RSC_K_EIG, g0, (int64_t)P.gemm.size() - g0, fl, lp_eig);
    }
    // (kNs.steps is even: the iterate ends in sa)
    cmd(kCmdTruncP, RSC_K_EIG, t0, nt, 0);             // sa = P
    ctx = RSC_K_BASIS;
    // 8. basis of range(P): W = orth(P Omega2) over all l columns; the columns the
    //    orthonormalisation keeps are compacted to the front of Om2, their count is q_j
    {
      const int64_t ph0 = (int64_t)P.philox.size();
      int64_t maxw2 = 0;
      for (int32_t j : js) {
        const CompSlot& C = h.comp[j];
        PhiloxTask t{};
        t.out = C.Om2; t.rows = C.ell; t.cols = C.ell; t.c2 = 1;
        t.k0 = (uint32_t)(h.opt.seed & 0xFFFFFFFFull);
        t.k1 = (uint32_t)(((h.opt.seed >> 32) & 0xFFFFFFFFull) ^ (uint64_t)(uint32_t)h.sn_local[j]);
        P.philox.push_back(t);
        maxw2 = std::max<int64_t>(maxw2, (int64_t)C.ell * ((C.ell + 3) / 4));
      }
      cmd(kCmdPhilox, RSC_K_OTHER, ph0, (int64_t)P.philox.size() - ph0, 0, maxw2, lp_eig ? 1 : 0);
      g0 = (int64_t)P.gemm.size(); fl = 0;
      for (int32_t j : js) {
        const CompSlot& C = h.comp[j];
        const int32_t l = C.ell;
        fl += tiles(gt(C.Sa, 1, l, C.Om2, l, 1, C.Wpan + l, 2 * l, l, l, l, 1.0, 0.0), 0, 0, false);
      }
      cmd(kCmdGemm, RSC_K_EIG, g0, (int64_t)P.gemm.size() - g0, fl, lp_eig);
      for (int pass = 0; pass < kCholQRPasses; ++pass) {
        g0 = (int64_t)P.gemm.size(); fl = 0;
        const int64_t s0 = (int64_t)P.gs_g.size();
        std::vector<PanelDesc> pan;
        for (int32_t j : js) {
          const CompSlot& C = h.comp[j];
          const int32_t l = C.ell;
          fl += tiles(gt(C.Wpan + l, 2 * l, 1, C.Wpan + l, 2 * l, 1, C.Wpan, 2 * l, l, l, l, 1.0, 0.0), 0, 0, true);
          P.gs_g.push_back(C.Wpan); P.gs_ld.push_back(2 * l); P.gs_n.push_back(l); P.gs_out.push_back(C.sc + 4);
          P.gs_m.push_back(0);
          // drop mode 2 (relative pivot 1e-8) when the projector came from FP32
          // products: its rounding leaves ~1e-6 in the directions it annihilates
          pan.push_back(PanelDesc{C.Wpan, 2 * l, l, l, false, C.Wdinv, j, lp_eig ? 2 : 1, C.sc + 4});
        }
        cmd(kCmdGemm, RSC_K_EIG, g0, (int64_t)P.gemm.size() - g0, fl);
        cmd(kCmdGramScale, RSC_K_OTHER, s0, (int64_t)P.gs_g.size() - s0, 0);
        panel_steps(pan);
      }
      int32_t lmax = 0;
      for (int32_t j : js) lmax = std::max(lmax, h.comp[j].ell);
      cmd(kCmdTruncFlags, RSC_K_EIG, t0, nt, 0, lmax);
      cmd(kCmdTruncCompact, RSC_K_EIG, t0, nt, 0);
      cmd(kCmdTruncCopy, RSC_K_EIG, t0, nt, 0, lmax);
    }
    credit(cs, m_eig);
    // 9. the kept basis U_j = U Z and V_j = V Z (Z: the projector's basis, columns beyond
    //    the device rank q_j skipped).  U_j is stored as W_j = M_j U_j = (M U) Z, from the
    //    product M U that step 5 left in tmp: the sweeps apply (L^D_j)^{-1} and U_j^T in
    //    one product, W_j^T y = U_j^T (L^D_j)^{-1} y.
    g0 = (int64_t)P.gemm.size(); fl = 0;
    for (int32_t j : js) {
      const CompSlot& C = h.comp[j];
      const int32_t c = S.c(j), r = S.r(j), l = C.ell;
      GemmTask t = gt(C.tmp, 1, c, C.Om2, l, 1, C.Uj, c, c, l, l, 1.0, 0.0);
      t.nlim = C.qslot;
      fl += tiles(t, 0, 0, false);
      GemmTask t2 = gt(C.V, 1, r, C.Om2, l, 1, C.Vj, r, r, l, l, 1.0, 0.0);
      t2.nlim = C.qslot;
      fl += tiles(t2, 0, 0, false);
    }
    cs = P.cmds.size();
    cmd(kCmdGemm, RSC_K_GEMM, g0, (int64_t)P.gemm.size() - g0, fl, lp_eig);
    // the kept basis U Z_q, V Z_q: algorithmic = executed (exact extents, at the ranks)
    for (size_t i = cs; i < P.cmds.size(); ++i) { P.cmds[i].mflops = P.cmds[i].flops; P.cmds[i].mkind = 2; }
    ctx = -1;
  }

  // Sec. 4.2 for the block-tree supernodes of one level: every block of each tree in
  // order, right-looking on the dense Schur block that the level's Schur update left in
  // the panel (A(C_j, C_j) minus every descendant's term: the first terms of Algorithms
  // 5 and 6, subtracted once for all blocks):
  //  * leaf (Algorithm 6): the panel factorisation of its diagonal block alone, the rows
  //    below it untouched, its inverse into its rows of M_j (which start as I);
  //  * internal block s: Algorithm 3 on L(R_s, C_s) = S(R_s, C_s) M_{s1}, M_{s1} the left
  //    subtree's (finished) part of M_j = (L^D_j)^{-T} -- Algorithm 4 as a product with
  //    that explicit inverse -- at the fixed rank l_s (no truncation); then S(R_s, R_s) -= V_s V_s^T (every later block's term from block s,
  //    Algorithms 5 and 6's loop over earlier blocks) and V_s U_s^T written over
  //    S(R_s, C_s), so that the panel holds the block tree's L^D_j;
  //  * once both subtrees of block t are done, M_j's coupling block
  //    M(C_t, R_t) = -(M_{t1} U_t) (M_{t2}^T V_t)^T (the inverse of the 2 x 2 block
  //    triangle), bottom-up, so that M_{s1} is whole before block s needs it.
  // The supernodes of one tree depth run in the same launches.
  void diag_trees(const std::vector<int32_t>& js) {
    const Symbolic& S = h.S;
    std::map<int32_t, std::vector<int32_t>> by_d;
    for (int32_t j : js) by_d[S.depth[j]].push_back(j);
    const size_t c_first = P.cmds.size();
    for (auto& kv : by_d) {
      const int32_t d = kv.first;
      const std::vector<int32_t>& g = kv.second;
      auto node = [&](int32_t j, int32_t s) -> const TreeNode& { return h.tree[j][s - 1]; };
      // tasks of dst = M(a:a+n, a:a+n) src or its transpose times src (n x l operands)
      auto tri = [&](int32_t j, bool trans, int32_t a, int32_t n, int32_t l, int64_t src, int32_t sld,
                     int64_t dst, int32_t dld) {
        const int32_t ldp = h.panel_ld[j];
        const int64_t M0 = h.panel_off[j] + S.c(j) + a + (int64_t)a * ldp;
        double f = 0;
        for (int32_t j0 = 0; j0 < l; j0 += kTile)
          for (int32_t i0 = 0; i0 < n; i0 += kTile) {
            GemmTask t = trans ? gt(M0, ldp, 1, src, sld, 1, dst, dld, n, l, std::min(n, i0 + kTile), 1.0, 0.0)
                               : gt(M0 + (int64_t)i0 * ldp, 1, ldp, src + i0, sld, 1, dst, dld, n, l, n - i0, 1.0, 0.0);
            t.i0 = i0; t.j0 = j0;
            P.gemm.push_back(t);
            f += 2.0 * std::min(kTile, n - i0) * std::min(kTile, l - j0) * (double)t.k;
          }
        return f;
      };
      auto launch = [&](int mode, const std::function<double(int32_t)>& push) {
        const int64_t g0 = (int64_t)P.gemm.size();
        double f = 0;
        for (int32_t j : g) f += push(j);
        cmd(kCmdGemm, RSC_K_GEMM, g0, (int64_t)P.gemm.size() - g0, f, mode);
      };
      auto SRC = [&](int32_t j, const TreeNode& n) {   // S(R_s, C_s) in the panel (ld 2c)
        return h.panel_off[j] + n.ra + (int64_t)n.ca * h.panel_ld[j];
      };
      auto assemble = [&](int32_t t) {
        ctx = RSC_K_TRSM;
        launch(lp_eig, [&](int32_t j) {          // X = M(R, R)^T V
          const TreeNode& n = node(j, t);
          const int32_t nr = n.rb - n.ra;
          return tri(j, true, n.ra, nr, n.ell, n.V, nr, n.X, nr);
        });
        launch(lp_eig, [&](int32_t j) {          // M(C, R) = -W X^T
          const TreeNode& n = node(j, t);
          const int32_t nc = n.cb - n.ca, nr = n.rb - n.ra, ldp = h.panel_ld[j];
          return tiles(gt(n.W, 1, nc, n.X, 1, nr, h.panel_off[j] + S.c(j) + n.ca + (int64_t)n.ra * ldp,
                          ldp, nc, nr, n.ell, -1.0, 0.0), 0, 0, false);
        });
        ctx = -1;
      };
      auto qr = [&](bool z, bool shifted) {
        std::vector<QRPanel> qs;
        for (int32_t j : g) {
          // (one tree's blocks run one after another, so they share the scale slot)
          const TreeNode& n = node(j, cur_s);
          qs.push_back(z ? QRPanel{n.zpanel, n.ell, n.rb - n.ra, n.zdinv, j, n.gscale + 1}
                         : QRPanel{n.ypanel, n.ell, n.cb - n.ca, n.dinv, j, n.gscale});
        }
        cholqr(qs, shifted);
      };
      const int32_t nb = (2 << d) - 1;
      for (int32_t s = 1; s <= nb; ++s) {
        cur_s = s;
        const int32_t ht = __builtin_ctz(s);
        if (ht == 0) {
          std::vector<PanelDesc> pan;
          for (int32_t j : g) {
            const TreeNode& n = node(j, s);
            const int32_t nn = n.cb - n.ca, c = S.c(j), ld = h.panel_ld[j];
            PanelDesc p{h.panel_off[j] + n.ca + (int64_t)n.ca * ld, ld, nn, c - nn, true, n.dinv, j, 0, 0};
            p.lp_lo = nn; p.lp_hi = c; p.skip_mid = true;   // [diagonal block; rows below (untouched); I]
            pan.push_back(p);
          }
          panel_steps(pan);
          continue;
        }
        for (int32_t hh = 1; hh < ht; ++hh) assemble(s - (1 << hh));
        // sample Omega (|R_s| x l), key of supernode j, third counter word 4 + s
        ctx = RSC_K_SAMPLE;
        const int64_t ph0 = (int64_t)P.philox.size();
        int64_t maxw = 0;
        for (int32_t j : g) {
          const TreeNode& n = node(j, s);
          PhiloxTask t{};
          t.out = n.omega; t.rows = n.rb - n.ra; t.cols = n.ell; t.c2 = 4 + (uint32_t)s;
          t.k0 = (uint32_t)(h.opt.seed & 0xFFFFFFFFull);
          t.k1 = (uint32_t)(((h.opt.seed >> 32) & 0xFFFFFFFFull) ^ (uint64_t)(uint32_t)h.sn_local[j]);
          P.philox.push_back(t);
          maxw = std::max<int64_t>(maxw, (int64_t)t.rows * ((t.cols + 3) / 4));
        }
        cmd(kCmdPhilox, RSC_K_OTHER, ph0, (int64_t)P.philox.size() - ph0, 0, maxw, lp_sample ? 1 : 0);
        // Y = L(R, C)^T Omega = M_{s1}^T (S(R, C)^T Omega) into rows [l, l + |C|) of the panel
        launch(lp_sample, [&](int32_t j) {
          const TreeNode& n = node(j, s);
          const int32_t nc = n.cb - n.ca, nr = n.rb - n.ra, ld = h.panel_ld[j];
          return tiles(gt(SRC(j, n), ld, 1, n.omega, nr, 1, n.tmp, nc, nc, n.ell, nr, 1.0, 0.0), 0, 0, false);
        });
        launch(lp_update, [&](int32_t j) {
          const TreeNode& n = node(j, s);
          const int32_t nc = n.cb - n.ca;
          return tri(j, true, n.ca, nc, n.ell, n.tmp, nc, n.ypanel + n.ell, n.ell + nc);
        });
        for (int it = 0; it < h.opt.power_iters; ++it) {
          qr(false, true);
          launch(0, [&](int32_t j) {             // Z = L(R, C) Y = S(R, C) (M_{s1} Y)
            const TreeNode& n = node(j, s);
            const int32_t nc = n.cb - n.ca;
            return tri(j, false, n.ca, nc, n.ell, n.ypanel + n.ell, n.ell + nc, n.tmp, nc);
          });
          launch(0, [&](int32_t j) {
            const TreeNode& n = node(j, s);
            const int32_t nc = n.cb - n.ca, nr = n.rb - n.ra, ld = h.panel_ld[j];
            return tiles(gt(SRC(j, n), 1, ld, n.tmp, nc, 1, n.zpanel + n.ell, n.ell + nr, nr, n.ell, nc, 1.0, 0.0),
                         0, 0, false);
          });
          qr(true, true);
          launch(0, [&](int32_t j) {             // Y = M_{s1}^T (S(R, C)^T Z)
            const TreeNode& n = node(j, s);
            const int32_t nc = n.cb - n.ca, nr = n.rb - n.ra, ld = h.panel_ld[j];
            return tiles(gt(SRC(j, n), ld, 1, n.zpanel + n.ell, n.ell + nr, 1, n.tmp, nc, nc, n.ell, nr, 1.0, 0.0),
                         0, 0, false);
          });
          launch(0, [&](int32_t j) {
            const TreeNode& n = node(j, s);
            const int32_t nc = n.cb - n.ca;
            return tri(j, true, n.ca, nc, n.ell, n.tmp, nc, n.ypanel + n.ell, n.ell + nc);
          });
        }
        // U = orth(Y): as for the off-diagonal blocks, two plain Cholesky-QR passes (the
        // directions of Y below ~1e-7 of its largest are lost: far below the error of a
        // fixed-rank block) for tol >= 1e-5, else shifted Cholesky-QR3, which keeps every
        // direction above the rounding of Y
        ctx = RSC_K_ORTH;
        const bool accurate = P.tol < 1e-5;
        for (int pass = 0; pass < (accurate ? 3 : 2); ++pass) qr(false, accurate && pass == 0);
        // W = M_{s1} U, V = S(R, C) W = L(R, C) U
        ctx = RSC_K_BASIS;
        launch(lp_eig, [&](int32_t j) {
          const TreeNode& n = node(j, s);
          const int32_t nc = n.cb - n.ca;
          return tri(j, false, n.ca, nc, n.ell, n.ypanel + n.ell, n.ell + nc, n.W, nc);
        });
        launch(lp_eig, [&](int32_t j) {
          const TreeNode& n = node(j, s);
          const int32_t nc = n.cb - n.ca, nr = n.rb - n.ra, ld = h.panel_ld[j];
          return tiles(gt(SRC(j, n), 1, ld, n.W, nc, 1, n.V, nr, nr, n.ell, nc, 1.0, 0.0), 0, 0, false);
        });
        // S(R, R) -= V V^T (tiles on or below the diagonal); L(R, C) = V U^T over S(R, C)
        ctx = RSC_K_UPDATE;
        launch(lp_update, [&](int32_t j) {
          const TreeNode& n = node(j, s);
          const int32_t nr = n.rb - n.ra, ld = h.panel_ld[j];
          return tiles(gt(n.V, 1, nr, n.V, 1, nr, h.panel_off[j] + n.ra + (int64_t)n.ra * ld, ld, nr, nr,
                          n.ell, -1.0, 1.0), 0, 0, true);
        });
        ctx = RSC_K_BASIS;
        launch(lp_eig, [&](int32_t j) {
          const TreeNode& n = node(j, s);
          const int32_t nc = n.cb - n.ca, nr = n.rb - n.ra, ld = h.panel_ld[j];
          return tiles(gt(n.V, 1, nr, n.ypanel + n.ell, 1, n.ell + nc, SRC(j, n), ld, nr, nc, n.ell, 1.0, 0.0),
                       0, 0, false);
        });
        ctx = -1;
      }
      for (int32_t hh = 1; hh <= d; ++hh) assemble((2 << d) - (1 << hh));
    }
    // algorithmic = executed for the trees' launches (exact extents, fixed ranks)
    for (size_t i = c_first; i < P.cmds.size(); ++i) P.cmds[i].mflops = P.cmds[i].flops;
  }
  int32_t cur_s = 0;   // the tree block being emitted
};

template <class T>
Error upload_plan(DevArray<T>& d, const std::vector<T>& v) { return upload(d, v); }

}  // namespace

// Tile tuner.  Every product launch that kept a 128-tile alternative is run with
// both task lists on the handle's own arena (one warm-up and one hipEvent-timed launch
// each, on the handle's private stream) and keeps the faster; the 64 list stays unless
// 128 is at least 3 % faster.  The arena holds scratch at this point -- the
// factorisation writes every region it reads before reading it -- and the device ranks
// are set to their largest value so that rank-limited products run at full width.
static Error tune_tiles(Handle& h, FactorPlan& P, hipStream_t caller) {
  bool any = false;
  for (const Cmd& c : P.cmds) any |= (c.alt_off >= 0);
  if (!any) return kOk;
  hipStream_t s = h.cap_stream;
  {
    // the tuner overwrites the arena and the device ranks: work the caller queued
    // before this factorization (a preconditioner apply, a PCG) must be done first
    hipEvent_t done;
    HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(done, caller));
    HIPCHK(hipStreamWaitEvent(s, done, 0));
    (void)hipEventDestroy(done);
  }
  double* A = h.arena.p;
  int32_t* I = h.ints.p;
  launch_fill_i32(I + h.i_ranks, h.S.M(), INT_MAX, s);
  hipEvent_t ev[4];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  Error err = kOk;
  for (Cmd& c : P.cmds) {
    if (c.alt_off < 0) continue;
    const int mode = (int)c.a;
    launch_gemm_staged(mode, 64, P.d_gemm.p + c.off, (int)c.count, A, I, nullptr, nullptr, nullptr, s);
    HIPCHK(hipEventRecord(ev[0], s));
    launch_gemm_staged(mode, 64, P.d_gemm.p + c.off, (int)c.count, A, I, nullptr, nullptr, nullptr, s);
    HIPCHK(hipEventRecord(ev[1], s));
    launch_gemm_staged(mode, 128, P.d_gemm.p + c.alt_off, (int)c.alt_count, A, I, nullptr, nullptr, nullptr, s);
    HIPCHK(hipEventRecord(ev[2], s));
    launch_gemm_staged(mode, 128, P.d_gemm.p + c.alt_off, (int)c.alt_count, A, I, nullptr, nullptr, nullptr, s);
    HIPCHK(hipEventRecord(ev[3], s));
    HIPCHK(hipEventSynchronize(ev[3]));
    float t64 = 0, t128 = 0;
    HIPCHK(hipEventElapsedTime(&t64, ev[0], ev[1]));
    HIPCHK(hipEventElapsedTime(&t128, ev[2], ev[3]));
    if (t128 < 0.97f * t64) {
      c.off = c.alt_off;
      c.count = c.alt_count;
      c.b = 128;
      ++P.tuned128;
    }
    ++P.tuned;
    c.alt_off = -1;
  }
  launch_fill_i32(I + h.i_ranks, h.S.M(), 0, s);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  for (auto& e : ev) (void)hipEventDestroy(e);
  return err;
}

static Error build_factor_plan(Handle& h, bool compressed, double tol, int32_t precision,
                               hipStream_t stream) {
  auto P = std::make_unique<FactorPlan>();
  P->compressed = compressed;
  P->precision = precision;
  P->tol = tol;
  Builder B(h, *P);
  const Symbolic& S = h.S;
  B.cmd(kCmdFill, RSC_K_OTHER, h.a_panels, h.panels_size, 0, 0, 0, 0.0);
  B.cmd(kCmdFillInts, RSC_K_OTHER, h.i_status, 2, 0, 0, 0, (double)INT_MAX);
  B.cmd(kCmdAssemble, RSC_K_OTHER, 0, S.nnz, 0);
  B.cmd(kCmdIdent, RSC_K_OTHER, 0, (int64_t)h.ident_slot.size(), 0);
  if (compressed) B.cmd(kCmdFillInts, RSC_K_OTHER, h.i_ranks, S.M(), 0, 0, 0, 0.0);
  for (int32_t L = 0; L < S.nlevels; ++L) {
    const auto& lev = S.by_level[L];
    // the level's U^O blocks in the pool: zero, then A(R_j, C_j)
    B.cmd(kCmdFill, RSC_K_OTHER, h.lev_uo[L][0], h.lev_uo[L][1] - h.lev_uo[L][0], 0, 0, 0, 0.0);
    B.cmd(kCmdAssembleLevel, RSC_K_OTHER, h.asmo_ptr[L], h.asmo_ptr[L + 1] - h.asmo_ptr[L], 0);
    B.updates(lev);
    std::vector<PanelDesc> pan;
    std::vector<int32_t> trees;   // rank-structured factor: L^D_j as a block tree (Sec. 4)
    double m_potrf = 0;
    for (int32_t j : lev) {
      if (compressed && S.depth[j] > 0) { trees.push_back(j); continue; }
      // [L^D_j; I]: the Cholesky factor and, in the rows below, M_j
      pan.push_back(PanelDesc{h.panel_off[j], h.panel_ld[j], S.c(j), 0, true, h.dinv_off[j], j, 0, 0});
      m_potrf += std::pow((double)S.c(j), 3) / 3.0;
    }
    const size_t cp = P->cmds.size();
    B.panel_steps(pan);
    B.credit(cp, m_potrf);
    if (!trees.empty()) B.diag_trees(trees);
    B.offdiag_solve(lev);
    B.compact_operands(lev, false);
    if (compressed && h.opt.interior) B.interior_copy(lev);
    if (compressed) {
      B.compression(lev, tol);
      B.compact_operands(lev, true);
    }
  }
  if (precision != RSC_FP64) B.f32_copy();
  // algorithmic flop counts of the method (per supernode, from the symbolic plan)
  P->alpha_D = h.tree_alpha;
  for (int64_t j = 0; j < S.M(); ++j) {
    const double c = S.c(j), r = S.r(j);
    if (compressed && S.depth[j] > 0) {
      // block tree: leaves' Cholesky, and per internal block its two products with
      // S(R, C), the products with M_{s1}, Cholesky-QR, the Schur update and M's coupling
      for (const TreeNode& t : h.tree[j]) {
        const double nc = t.cb - t.ca, nr = t.rb - t.ra, l = t.ell;
        if (t.ht == 0) { P->flops[0] += nc * nc * nc / 3.0; continue; }
        P->flops[3] += 4.0 * nr * nc * l + 2.0 * nc * nc * l;
        P->flops[4] += 2.0 * nc * l * l;
        P->flops[2] += nr * nr * l + nr * nr * l + 2.0 * nc * nr * l;
      }
    } else {
      P->flops[0] += c * c * c / 3.0;
    }
    if (!(compressed && h.compressible[j])) P->flops[1] += r * c * c;
    if (compressed && h.compressible[j]) {
      const double l = h.comp[j].ell;
      // the products with U^O_j and Algorithm 2's diagonal solves (c^2 l each)
      P->flops[3] += (4.0 * r * c * l + 2.0 * c * c * l) * (1 + h.opt.power_iters);
      P->flops[4] += 2.0 * c * l * l;
      P->flops[5] += 2.0 * r * l * l + 9.0 * l * l * l;   // + the kept basis, at the ranks (stats)
    }
  }
  Error e;
  if ((e = upload(P->d_gemm, P->gemm)).code) return e;
  if ((e = upload(P->d_tiles, P->tiles)).code) return e;
  if ((e = upload(P->d_ents, P->ents)).code) return e;
  if ((e = upload(P->d_compact, P->compact)).code) return e;
  if (P->xc_size > 0) {
    P->d_xc.p = static_cast<double*>(dev_alloc(sizeof(double) * P->xc_size));
    if (!P->d_xc.p) return Error{RSC_ERR_OUT_OF_MEMORY, "compact operand copies"};
    P->d_xc.n = P->xc_size;
  }
  if (P->split_size > 0) {
    P->d_split.p = static_cast<double*>(dev_alloc(sizeof(double) * P->split_size));
    if (!P->d_split.p) return Error{RSC_ERR_OUT_OF_MEMORY, "split-K scratch"};
    P->d_split.n = P->split_size;
  }
  if ((e = upload(P->d_potrf, P->potrf)).code) return e;
  if ((e = upload(P->d_philox, P->philox)).code) return e;
  if ((e = upload(P->d_trunc, P->trunc)).code) return e;
  if ((e = upload(P->d_gs_g, P->gs_g)).code) return e;
  if ((e = upload(P->d_gs_out, P->gs_out)).code) return e;
  if ((e = upload(P->d_gs_ld, P->gs_ld)).code) return e;
  if ((e = upload(P->d_gs_n, P->gs_n)).code) return e;
  if ((e = upload(P->d_gs_m, P->gs_m)).code) return e;
  if ((e = upload(P->d_conv, P->conv)).code) return e;
  if ((e = upload(P->d_copy, P->copy)).code) return e;
  // FP32 copy of the sweeps' operands: the compact M_j, dense L^O and region X of this layout
  const int64_t n32 = h.m32_size + (compressed ? h.f32_end_comp : h.f32_end_exact) - h.a_lo;
  if (!P->conv.empty() && h.arena32.n < n32) {
    drop_graphs(h);
    h.arena32.reset();
    h.arena32.p = static_cast<float*>(dev_alloc(sizeof(float) * (size_t)n32));
    h.arena32.n = h.arena32.p ? n32 : 0;
    if (!h.arena32.p) return Error{RSC_ERR_OUT_OF_MEMORY, "FP32 copy of the factor operands"};
  }
  if ((e = tune_tiles(h, *P, stream)).code) return e;
  auto& slot = h.fplans[precision];
  if (slot && slot->graph) (void)hipGraphExecDestroy(slot->graph);
  slot = std::move(P);
  return kOk;
}

// ------------------------------------------------------------------ executor

struct EventPair {
  hipEvent_t a, b;
  int32_t klass, kid, arith;   // arith: RSC_ARITH_* of the launch's MFMA work, -1 none
  double flops, mflops;        // executed tile flops, algorithmic flops
  const Cmd* cmd;
  const FactorPlan* plan;
};

// MFMA arithmetic of a command (RSC_ARITH_*), or -1 when it has no MFMA work.
static int32_t cmd_arith(const Cmd& c) {
  switch (c.type) {
    case kCmdGemm: case kCmdUpdate: {
      const int m = (int)(c.a & 3);
      return m == 0 ? RSC_ARITH_F64 : m == 1 ? RSC_ARITH_F32 : RSC_ARITH_BF16;
    }
    case kCmdPotrf: return RSC_ARITH_F64;
    case kCmdTruncNs: return c.a != 0 ? RSC_ARITH_F32 : RSC_ARITH_F64;
    default: return -1;
  }
}

// Flops of a launch whose extents come from device ranks, from its tasks and the
// ranks as they stand (I: host copy of the int arena): executed tile flops, and in *mfl
// the algorithmic flops of a Schur update (the entries' pairs on or below the diagonal).
static double recount_flops(const Cmd& c, const FactorPlan& P, const std::vector<int32_t>& I,
                            double* mfl) {
  double fl = 0;
  *mfl = 0;
  if (c.type == kCmdUpdate) {
    for (int64_t t = c.off; t < c.off + c.count; ++t)
      for (int32_t i = P.tiles[t].e0; i < P.tiles[t].e1; ++i) {
        const UpdEntry& e = P.ents[i];
        const double K = e.kdim >= 0 ? e.kdim : I[-1 - e.kdim];
        fl += 2.0 * (e.b - e.a) * (e.d - e.c) * K;
        *mfl += 2.0 * P.ent_lower[i] * K;
      }
  } else if (c.type == kCmdGemm) {
    const int32_t T = (int32_t)c.b;
    for (int64_t i = c.off; i < c.off + c.count; ++i) {
      const GemmTask& t = P.gemm[i];
      const int32_t n = t.nlim >= 0 ? std::min(t.n, I[t.nlim]) : t.n;
      int32_t K = t.klim >= 0 ? std::min(t.k, I[t.klim]) : t.k;
      if (t.kz > 1) {                    // this task's K slice
        const int32_t per = ((K + t.kz - 1) / t.kz + 31) / 32 * 32;
        const int32_t kb = std::min(K, t.ks * per);
        K = std::min(K, kb + per) - kb;
      }
      fl += 2.0 * std::min(T, t.m - t.i0) * std::max(0, std::min(T, n - t.j0)) * (double)K;
    }
  }
  return fl;
}

static const char* const kKernelNames[RSC_KERNELS] = {  // index = kernel_id()
    "gemm_staged_f64", "gemm_staged_f32", "gemm_staged_bf16x3", "gemm_staged_bf16",
    "update_waves_f64", "update_waves_f32", "update_waves_bf16x3", "update_waves_bf16",
    "potrf_f64", "philox", "gram_scale", "trunc_prep", "trunc_power", "trunc_x0", "trunc_p",
    "trunc_compact", "assemble", "fill", "row_gather", "coldot", "row_part", "gemv_n",
    "gather", "part_apply", "other", "gemm_staged128_f64", "gemm_staged128_f32",
    "gemm_staged128_bf16x3", "gemm_staged128_bf16", "compact_rows", "gemm_reduce", "trunc_mfill",
    "trunc_flags", "trunc_copy", "to_f32", "trunc_ns", "sweep_fwd", "sweep_bwd", "gemm_potrf_f64",
    "copy_f64", "interior_solve", "coupling"};

int32_t kernel_id(int32_t type, int64_t a, int64_t b, bool post) {
  switch (type) {
    case kCmdGemm: return post ? 38 : (int32_t)((b == 128 ? 25 : 0) + (a & 3));
    case kCmdUpdate: return (int32_t)(4 + (a & 3));
    case kCmdCompact: return 29;
    case kCmdGemmReduce: return 30;
    case kCmdTruncMfill: return 31;
    case kCmdTruncFlags: return 32;
    case kCmdTruncCopy: return 33;
    case kCmdToF32: return 34;
    case kCmdTruncNs: return 35;
    case kCmdSweepFwd: return 36;
    case kCmdSweepBwd: return 37;
    case kCmdCopy: return 39;
    case kCmdInterior: return 40;
    case kCmdCoupling: return 41;
    case kCmdPotrf: return 8;
    case kCmdPhilox: return 9;
    case kCmdGramScale: return 10;
    case kCmdTruncPrep: return 11;
    case kCmdTruncPower: return 12;
    case kCmdTruncX0: return 13;
    case kCmdTruncP: return 14;
    case kCmdTruncCompact: return 15;
    case kCmdAssemble: case kCmdIdent: case kCmdAssembleLevel: return 16;
    case kCmdFill: case kCmdFillInts: return 17;
    case kCmdColDot: return 19;
    case kCmdRowPart: return 20;
    case kCmdGemvN: return 21;
    case kCmdRowGather: return 18;
    case kCmdGatherRows: case kCmdGatherPerm: case kCmdScatterPerm: return 22;
    case kCmdPartApply: return 23;
    default: return 24;
  }
}

const char* kernel_name(int32_t k) { return (k >= 0 && k < RSC_KERNELS) ? kKernelNames[k] : ""; }

// The FP32 copy addressed by FP32 offsets: element a_lo - m32_size + k of the result is
// element k of the copy (no offset below that is ever used with it).
static float* f32_base(Handle& h) {
  return reinterpret_cast<float*>(reinterpret_cast<uintptr_t>(h.arena32.p) -
                                  sizeof(float) * (uintptr_t)(h.a_lo - h.m32_size));
}

static void launch_cmd(Handle& h, const Cmd& c, const FactorPlan* P, const SolvePlan* Q,
                       hipStream_t s, double* part_buf = nullptr) {
  double* A = h.arena.p;
  // partial-sum blocks of the sweeps: the solve plan's own, or a caller's buffer
  double* QP = part_buf ? part_buf : (Q ? Q->d_part.p : nullptr);
  int32_t* I = h.ints.p;
  const float* F32 = h.f32_valid ? f32_base(h) : nullptr;   // factor operands of the sweeps
  switch (c.type) {
    case kCmdFill: launch_fill(A + c.off, c.count, c.v, s); break;
    case kCmdFillInts: launch_fill_i32(I + c.off, c.count, (int32_t)c.v, s); break;
    case kCmdAssemble: launch_assemble(A + h.a_values, h.d_asm_slot.p, c.count, A, s); break;
    case kCmdAssembleLevel:
      launch_assemble_pairs(A + h.a_values, h.d_asmo_idx.p + c.off, h.d_asmo_slot.p + c.off, c.count,
                            A + h.a_pool, s);
      break;
    case kCmdIdent: launch_scatter_const(h.d_ident_slot.p, c.count, 1.0, A, s); break;
    case kCmdUpdate:
      launch_update_waves((int)c.a, P->d_tiles.p + c.off, (int)c.count, P->d_ents.p, h.d_relmap.p, A,
                          P->d_xc.p, I, s);
      break;
    case kCmdCompact:
      launch_compact_rows((int)c.a, P->d_compact.p + c.off, (int)c.count, A, I, P->d_xc.p,
                          P->precision != RSC_FP64 ? f32_base(h) : nullptr, s);
      break;
    case kCmdPotrf: launch_potrf_f64(P->d_potrf.p + c.off, (int)c.count, (int)c.a, A, I + h.i_status, s); break;
    case kCmdGemm:
      launch_gemm_staged((int)c.a, (int)c.b, P->d_gemm.p + c.off, (int)c.count, A, I, P->d_split.p,
                         c.post ? P->d_potrf.p : nullptr, I + h.i_status, s);
      break;
    case kCmdGemmReduce: launch_gemm_reduce((int)c.b, P->d_gemm.p + c.off, (int)c.count, A, I, P->d_split.p, s); break;
    case kCmdPhilox: launch_philox(P->d_philox.p + c.off, (int)c.count, c.a, A, c.b != 0, s); break;
    case kCmdGramScale:
      launch_gram_scale(P->d_gs_g.p + c.off, P->d_gs_ld.p + c.off, P->d_gs_n.p + c.off,
                        P->d_gs_m.p + c.off, P->d_gs_out.p + c.off, (int)c.count, A, s);
      break;
    case kCmdTruncPrep: launch_trunc_prep(P->d_trunc.p + c.off, (int)c.count, A, s); break;
    case kCmdTruncPower:
      if (c.a == 0) launch_trunc_power(P->d_trunc.p + c.off, (int)c.count, A, s);
      else if (c.b < 5) launch_trunc_pmv(P->d_trunc.p + c.off, (int)c.count, (int)c.a, (int)c.b, A, s);
      else launch_trunc_pfin(P->d_trunc.p + c.off, (int)c.count, A, s);
      break;
    case kCmdTruncX0: launch_trunc_x0(P->d_trunc.p + c.off, (int)c.count, A, s); break;
    case kCmdTruncP: launch_trunc_p(P->d_trunc.p + c.off, (int)c.count, A, s); break;
    case kCmdTruncCompact: launch_trunc_compact(P->d_trunc.p + c.off, (int)c.count, A, I, s); break;
    case kCmdTruncMfill: launch_trunc_mfill(P->d_trunc.p + c.off, (int)c.count, A, s); break;
    case kCmdTruncFlags: launch_trunc_flags(P->d_trunc.p + c.off, (int)c.count, (int)c.a, A, s); break;
    case kCmdTruncCopy: launch_trunc_copy(P->d_trunc.p + c.off, (int)c.count, (int)c.a, A, s); break;
    case kCmdGemvN: launch_gemv_n(Q->d_gemv.p + c.off, (int)c.count, A, F32, I, s); break;
    case kCmdColDot: launch_coldot(Q->d_coldot.p + c.off, (int)c.count, A, F32, h.d_rows.p, I, QP, s); break;
    case kCmdRowPart: launch_row_part(Q->d_rchunks.p + c.off, (int)c.count, A, F32, I, QP, s); break;
    case kCmdToF32: launch_to_f32(P->d_conv.p + c.off, (int)c.count, A, f32_base(h), s); break;
    case kCmdTruncNs:
      launch_trunc_ns(P->d_trunc.p + c.off, (int)c.count, c.a != 0, A, kNs, s);
      break;
    case kCmdPartApply: launch_part_apply(Q->d_papply.p + c.off, (int)c.count, QP, A, s); break;
    case kCmdSweepFwd:
      launch_sweep_fwd(Q->d_sweep.p + c.off, (int)c.count, (int)c.a, (int)c.b, c.lds_l, A, F32, h.a_y,
                       h.a_w, h.a_zr, I, Q->d_pull_ptr.p, Q->d_pull_idx.p, s);
      break;
    case kCmdSweepBwd:
      launch_sweep_bwd(Q->d_sweep.p + c.off, (int)c.count, (int)c.a, (int)c.b, c.lds_l, c.lds_r, A, F32,
                       h.a_w, h.a_zz, I, h.d_rows.p, s);
      break;
    case kCmdGatherRows:
      launch_gather_rows(Q->d_gath.p + 2 * c.off, (int)c.count, h.d_rows.p, A + h.a_zz, A + h.a_zr, s);
      break;
    case kCmdRowGather:
      launch_row_gather(Q->d_rg_rows.p + c.off, Q->d_rg_ptr.p + c.a, Q->d_rg_contrib.p, c.count,
                        A + h.a_zr, A + h.a_y, s);
      break;
    case kCmdGatherPerm: launch_gather_perm(h.S.n, h.d_perm.p, A + c.a, A + c.b, s); break;
    case kCmdCopy: launch_copy_f64(P->d_copy.p + c.off, (int)c.count, A, s); break;
    case kCmdInterior:
      launch_interior(Q->d_isns.p + c.off, (int)c.count, c.a != 0, A, F32, h.d_rows.p, Q->d_ipull_ptr.p,
                      Q->d_ipull_idx.p, A + h.a_w, A + h.a_t, A + h.a_zr, s);
      break;
    case kCmdCoupling:   // a = 0: y_R -= A(R, C) t (forward); a = 1: t_C = A(C, R) z (backward)
      launch_coupling(Q->d_cp_tgt.p + c.off, Q->d_cp_ptr.p + c.off, Q->d_cp_vidx.p, Q->d_cp_xidx.p, c.count,
                      A + h.a_values, A + (c.a ? h.a_zz : h.a_t), A + (c.a ? h.a_t : h.a_y), c.a == 0, s);
      break;
    case kCmdScatterPerm: launch_scatter_perm(h.S.n, h.d_perm.p, A + c.a, A + c.b, s); break;
    default: break;
  }
}

// Runs a command list; with profiling on, brackets every launch with events.
static Error run_cmds(Handle& h, const std::vector<Cmd>& cmds, const FactorPlan* P,
                      const SolvePlan* Q, hipStream_t s, std::vector<EventPair>* evs,
                      double* part_buf = nullptr) {
  for (const Cmd& c : cmds) {
    if (evs) {
      EventPair ep;
      HIPCHK(hipEventCreate(&ep.a));
      HIPCHK(hipEventCreate(&ep.b));
      ep.klass = c.klass;
      ep.kid = kernel_id(c.type, c.a, c.b, c.post);
      ep.arith = cmd_arith(c);
      ep.flops = c.flops;
      ep.mflops = c.mflops;
      ep.cmd = c.dyn ? &c : nullptr;
      ep.plan = P;
      HIPCHK(hipEventRecord(ep.a, s));
      launch_cmd(h, c, P, Q, s, part_buf);
      HIPCHK(hipEventRecord(ep.b, s));
      evs->push_back(ep);
    } else {
      launch_cmd(h, c, P, Q, s, part_buf);
    }
  }
  HIPCHK(hipGetLastError());
  return kOk;
}

static Error collect_events(Handle& h, std::vector<EventPair>& evs) {
  std::vector<int32_t> ints;
  for (auto& ep : evs) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ep.a, ep.b));
    if (ep.cmd && ep.plan) {
      if (ints.empty()) {
        ints.resize((size_t)h.ints_size);
        HIPCHK(hipMemcpy(ints.data(), h.ints.p, sizeof(int32_t) * ints.size(), hipMemcpyDeviceToHost));
      }
      double mfl = 0;
      ep.flops = recount_flops(*ep.cmd, *ep.plan, ints, &mfl);
      if (ep.cmd->mkind == 1) ep.mflops = mfl;
      else if (ep.cmd->mkind == 2) ep.mflops = ep.flops;
    }
    h.prof.launches[ep.klass] += 1;
    h.prof.ms[ep.klass] += ms;
    h.prof.flops[ep.klass] += ep.mflops;
    h.prof.tile_flops[ep.klass] += ep.flops;
    if (ep.arith >= 0) h.prof.flops_arith[ep.klass][ep.arith] += ep.mflops;
    h.kprof_launches[ep.kid] += 1;
    h.kprof_ms[ep.kid] += ms;
    h.kprof_flops[ep.kid] += ep.mflops;
    h.kprof_tile_flops[ep.kid] += ep.flops;
    (void)hipEventDestroy(ep.a);
    (void)hipEventDestroy(ep.b);
  }
  evs.clear();
  return kOk;
}

static Error capture(Handle& h, const std::function<Error(hipStream_t)>& body, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal));
  Error e = body(h.cap_stream);
  hipError_t ee = hipStreamEndCapture(h.cap_stream, &g);
  if (e.code) { if (g) (void)hipGraphDestroy(g); return e; }
  if (ee != hipSuccess) return Error{RSC_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee)};
  hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return Error{RSC_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie)};
  return kOk;
}

// The solve graphs hold the sweep kernels of one factor operand copy (FP64 arena or
// its FP32 copy): recaptured after a factorization of the other kind.
static void solve_graph_mode(Handle& h) {
  SolvePlan* Q = h.splan.get();
  const int32_t m = h.f32_valid ? 1 : 0;
  if (!Q || Q->f32_mode == m) return;
  if (Q->graph_a) (void)hipGraphExecDestroy(Q->graph_a);
  if (Q->graph_b) (void)hipGraphExecDestroy(Q->graph_b);
  if (Q->graph_apply) (void)hipGraphExecDestroy(Q->graph_apply);
  Q->graph_a = Q->graph_b = Q->graph_apply = nullptr;
  Q->f32_mode = m;
}

// ------------------------------------------------------------------ factor

static Error factor_once(Handle& h, const double* values, double tol, int32_t precision,
                         hipStream_t stream) {
  Error e;
  const bool compressed = tol > 0.0;
  // the layout of this factor: where L^O_j of the compressible supernodes (or V_j, U_j)
  // live, where the level pool starts, and the arena length it needs
  set_layout(h, compressed);
  if ((e = ensure_arena(h, compressed ? h.arena_size_comp : h.arena_size_exact)).code) return e;
  auto& slot = h.fplans[precision];
  if (!slot || slot->compressed != compressed ||
      (compressed && (slot->tol != tol || slot->alpha_D != h.tree_alpha)))
    if ((e = build_factor_plan(h, compressed, tol, precision, stream)).code) return e;
  if (h.splan && h.splan->compressed != compressed) {
    if (h.splan->graph_a) (void)hipGraphExecDestroy(h.splan->graph_a);
    if (h.splan->graph_b) (void)hipGraphExecDestroy(h.splan->graph_b);
    if (h.splan->graph_apply) (void)hipGraphExecDestroy(h.splan->graph_apply);
    h.splan.reset();
  }
  h.fplan = slot.get();
  h.factored = false;
  h.f32_valid = false;
  h.tol = tol;
  FactorPlan* P = h.fplan;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipMemcpyAsync(h.arena.p + h.a_values, values, sizeof(double) * (size_t)h.S.nnz,
                        hipMemcpyDeviceToDevice, stream));
  HIPCHK(hipEventRecord(e0, stream));
  if (h.profiling) {
    std::vector<EventPair> evs;
    if ((e = run_cmds(h, P->cmds, P, nullptr, stream, &evs)).code) return e;
    HIPCHK(hipEventRecord(e1, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if ((e = collect_events(h, evs)).code) return e;
  } else if (h.opt.use_graph) {
    if (!P->graph) {
      e = capture(h, [&](hipStream_t s) { return run_cmds(h, P->cmds, P, nullptr, s, nullptr); },
                  &P->graph);
      if (e.code) return e;
    }
    HIPCHK(hipGraphLaunch(P->graph, stream));
    HIPCHK(hipEventRecord(e1, stream));
  } else {
    if ((e = run_cmds(h, P->cmds, P, nullptr, stream, nullptr)).code) return e;
    HIPCHK(hipEventRecord(e1, stream));
  }
  int32_t st[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(st, h.ints.p + h.i_status, sizeof(st), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h.t_factor_ms = ms;
  if (st[0] != INT_MAX) {
    h.failed_supernode = st[0];
    return Error{RSC_ERR_NOT_SPD, "non-positive pivot in supernode " + std::to_string(st[0])};
  }
  h.failed_supernode = -1;
  h.precision_used = precision;
  h.f32_valid = precision != RSC_FP64;
  h.factored = true;
  return kOk;
}

static Error ensure_solve(Handle& h);

// The restart policy of Sec. 5.3 (raise the accuracy and refactor after an indefinite
// pivot): for block trees the diagonal rank constant alpha_D, by 1.25 per restart; then
// the precision of the products: mixed BF16 -> FP32 products -> FP64.
Error factor(Handle& h, const double* values, double tol, hipStream_t stream) {
  Error e = ensure_device(h);
  if (e.code) return e;
  std::vector<int32_t> ladder{h.opt.precision};
  if (h.opt.retry) {
    if (h.opt.precision == RSC_MIXED_BF16) ladder.push_back(RSC_MIXED_FP32);
    if (h.opt.precision != RSC_FP64) ladder.push_back(RSC_FP64);
  }
  h.retries = 0;
  h.diag_restarts = 0;
  // block trees (Sec. 5.3): a factorization that meets an indefinite pivot restarts with
  // alpha_D raised by a quarter, until it succeeds or every block is sampled at full rank
  bool trees = false;
  if (tol > 0.0)
    for (int32_t d : h.S.depth) trees = trees || d > 0;
  if (trees && h.tree_alpha != h.opt.alpha_D) plan_trees(h, h.opt.alpha_D);
  for (size_t k = 0; k < ladder.size(); ++k) {
    for (;;) {
      e = factor_once(h, values, tol, ladder[k], stream);
      if (e.code != RSC_ERR_NOT_SPD || !trees || trees_exact(h) || h.diag_restarts >= 64) break;
      plan_trees(h, h.tree_alpha * 1.25);
      h.diag_restarts++;
    }
    if (e.code != RSC_ERR_NOT_SPD || k + 1 == ladder.size()) break;
    h.retries++;
  }
  if (e.code) return e;
  return ensure_solve(h);   // the sweep plan of this factor (rsc_apply_preconditioner_noalloc needs it)
}

// ------------------------------------------------------------------ solve plan

static Error build_solve_plan(Handle& h) {
  auto Q = std::make_unique<SolvePlan>();
  const Symbolic& S = h.S;
  const bool comp = h.fplan && h.fplan->compressed;
  Q->compressed = comp;
  auto cmd = [&](int32_t type, int64_t off, int64_t count, int64_t a = 0, int64_t b = 0) {
    if (count <= 0) return;
    Cmd c{};
    c.type = type; c.klass = RSC_K_PCG; c.off = off; c.count = count; c.a = a; c.b = b;
    Q->fwd_bwd.push_back(c);
  };
  // Column-dot launch of one sweep stage.  When the stage has fewer than 2048 tasks,
  // the rows of every task are cut into chunks (so that the stage has about 2048
  // workgroups) whose 16 sums go to partial blocks, stored in order by a second launch.
  // With `kept`, the partial blocks of a chunked output vector are left for the next
  // launch to add (kept[out] = first slot and chunks per 16-column task) instead.
  // Returns the partial blocks used.
  using KeptParts = std::map<int64_t, std::pair<int32_t, int32_t>>;
  auto coldot_stage = [&](std::vector<ColDotTask>& ts, KeptParts* kept = nullptr) -> int32_t {
    if (ts.empty()) return 0;
    const int64_t c0 = (int64_t)Q->coldot.size();
    if (ts.size() >= 2048) {
      for (auto& t : ts) { t.r0 = 0; t.r1 = INT_MAX; t.slot = -1; Q->coldot.push_back(t); }
      cmd(kCmdColDot, c0, (int64_t)ts.size());
      return 0;
    }
    double rows = 0;
    for (auto& t : ts) rows += t.tri ? std::min(t.rows, t.col0 + 16) : t.rows;
    const int32_t chunk = (int32_t)std::max(256.0, 64.0 * std::ceil(rows / 2048.0 / 64.0));
    const int64_t a0 = (int64_t)Q->papply.size();
    int32_t slot = 0;
    for (auto& t : ts) {
      const int32_t R = t.tri ? std::min(t.rows, t.col0 + 16) : t.rows;
      if (R <= chunk) { t.r0 = 0; t.r1 = INT_MAX; t.slot = -1; Q->coldot.push_back(t); continue; }
      const int32_t s0 = slot;
      for (int32_t r0 = 0; r0 < R; r0 += chunk) {
        ColDotTask u = t;
        u.r0 = r0; u.r1 = std::min(R, r0 + chunk); u.slot = slot++;
        Q->coldot.push_back(u);
      }
      if (kept) {
        if (!kept->count(t.out)) (*kept)[t.out] = {s0, slot - s0};
        continue;
      }
      // a static column count ends the block at the supernode's last column; a device
      // rank may not, but those outputs are padded to a multiple of 64
      const int32_t nout = t.ncols >= 0 ? std::min(16, t.ncols - t.col0) : 16;
      Q->papply.push_back(PartApply{t.out + t.col0, nout, s0, slot - s0, 1});
    }
    Q->part_slots = std::max<int64_t>(Q->part_slots, slot);
    cmd(kCmdColDot, c0, (int64_t)Q->coldot.size() - c0);
    if ((int64_t)Q->papply.size() > a0) cmd(kCmdPartApply, a0, (int64_t)Q->papply.size() - a0);
    return slot;
  };
  auto iscomp = [&](int64_t j) { return comp && h.compressible[j]; };
  // the inverse diagonal blocks M_j: in the panels (FP64 sweeps), or the FP32 copy's
  // compact blocks after a mixed factorization
  const bool f32 = h.f32_valid;
  Q->f32_tasks = f32;
  auto m_off = [&](int64_t j) { return f32 ? h.m32_off[j] : h.panel_off[j] + S.c(j); };
  auto m_ld = [&](int64_t j) { return f32 ? S.c(j) : h.panel_ld[j]; };
  // interior blocks (Sec. 5.1): the sweeps use only the rows of L^O_j inside the block
  const bool ib = comp && h.opt.interior != 0;
  auto inter = [&](int64_t j) { return ib && h.iroot[j] >= 0 && S.r(j) > 0; };
  auto rr = [&](int64_t j) { return inter(j) ? h.r_in[j] : S.r(j); };          // rows of R_j used
  auto lox = [&](int64_t j) { return inter(j) ? h.lo_in[j] : h.lo_off[j]; };   // their L^O_j
  double bytes = 0;
  // Small-supernode levels: the lowest levels whose supernodes all fit one workgroup
  // (at most sweep_small_c columns and kSweepMaxR rows) run each sweep step as one launch
  // (k_sweep_fwd / k_sweep_bwd).  Inside them a row pulls its descendants' contributions
  // when its own supernode is solved; the contributions to rows above them are applied
  // by one row gather before the first larger level.
  struct SmallLevel {
    int64_t t0 = 0, nt = 0;
    int32_t threads = 64, cpad = 1, lpad = 0, rmax = 0;
  };
  int32_t nsmall = 0;
  while (h.opt.sweep_small_c > 0 && nsmall < S.nlevels) {
    bool ok = true;
    for (int32_t j : S.by_level[nsmall]) ok = ok && S.c(j) <= h.opt.sweep_small_c && S.r(j) <= kSweepMaxR;
    if (!ok) break;
    ++nsmall;
  }
  Q->small_levels = nsmall;
  std::vector<SmallLevel> small(nsmall);
  std::vector<std::pair<int64_t, int64_t>> outside;   // (row, zr slot) of rows above them
  if (nsmall > 0) {
    auto small_row = [&](int64_t row) { return S.level[S.owner[row]] < nsmall; };
    std::vector<int64_t> ptr((size_t)S.n + 1, 0);
    for (int32_t L = 0; L < nsmall; ++L) {
      SmallLevel& sl = small[L];
      sl.t0 = (int64_t)Q->sweep.size();
      int32_t cmax = 1, rmax = 0, lmax = 0;
      for (int32_t j : S.by_level[L]) {
        const int32_t c = S.c(j), r = S.r(j);
        SweepTask t{};
        t.m = m_off(j); t.ld = m_ld(j);
        t.first = S.first[j]; t.rows = S.rows_ptr[j]; t.c = c; t.r = r;
        t.x = 0; t.u = -1; t.qslot = -1; t.kmax = 0;
        if (iscomp(j)) {
          const CompSlot& C = h.comp[j];
          t.x = C.Vj; t.u = C.Uj; t.qslot = C.qslot; t.kmax = C.ell;
          lmax = std::max(lmax, C.ell);
          bytes += 2.0 * 8.0 * (double)(c + r) * C.ell;
        } else if (r > 0) {
          t.x = lox(j);
          t.r = rr(j);
          bytes += 2.0 * 8.0 * (double)rr(j) * c;
        }
        bytes += 2.0 * 8.0 * c * (c + 1) / 2;
        Q->sweep.push_back(t);
        cmax = std::max(cmax, c);
        rmax = std::max(rmax, r);
        for (int64_t p = S.rows_ptr[j]; p < S.rows_ptr[j] + rr(j); ++p) {
          const int64_t row = S.rows[p];
          if (small_row(row)) ++ptr[row + 1];
          else outside.push_back({row, p});
        }
      }
      sl.nt = (int64_t)Q->sweep.size() - sl.t0;
      sl.threads = (cmax <= 64 && rmax <= 256) ? 64 : 256;
      sl.cpad = cmax; sl.lpad = lmax; sl.rmax = rmax;
    }
    for (int64_t i = 0; i < S.n; ++i) ptr[i + 1] += ptr[i];
    Q->pull_idx.assign((size_t)ptr[S.n], 0);
    std::vector<int64_t> next(ptr.begin(), ptr.end() - 1);
    for (int32_t L = 0; L < nsmall; ++L)
      for (int32_t j : S.by_level[L])
        for (int64_t p = S.rows_ptr[j]; p < S.rows_ptr[j] + rr(j); ++p)
          if (small_row(S.rows[p])) Q->pull_idx[(size_t)next[S.rows[p]]++] = p;
    Q->pull_ptr = std::move(ptr);
    std::stable_sort(outside.begin(), outside.end(), [](const std::pair<int64_t, int64_t>& x,
                                                        const std::pair<int64_t, int64_t>& y) { return x.first < y.first; });
  }
  auto small_cmd = [&](int32_t type, const SmallLevel& sl) {
    if (sl.nt <= 0) return;
    Cmd c{};
    c.type = type; c.klass = RSC_K_PCG; c.off = sl.t0; c.count = sl.nt;
    c.a = sl.threads; c.b = sl.cpad; c.lds_l = sl.lpad; c.lds_r = sl.rmax;
    Q->fwd_bwd.push_back(c);
  };
  // Interior blocks by the level of their root (eq. interiorBlockMult): forward, once the
  // level is solved, t = (L^B)^{-T} w^B (the block's levels from its root down) and
  // y_{R^B} -= A(R^B, C^B) t; backward, before the level, t = A(C^B, R^B) z_{R^B}, then
  // t = (L^B)^{-1} t (the block's levels up to its root, whose step also takes
  // w^B -= t).  A's entries are taken from the lower triangle of the original numbering,
  // as the factorization takes them.
  struct IntLevel {
    std::vector<std::pair<int64_t, int64_t>> steps;   // per block level 0 .. L: task range
    int64_t f0 = 0, nf = 0, g0 = 0, ng = 0;           // coupling targets: forward, backward
  };
  std::vector<IntLevel> il(S.nlevels);
  if (ib) {
    auto lower_entry = [&](int64_t orow, int64_t ocol) {   // CSR index of A(max, min)
      const int64_t i = std::max(orow, ocol), c = std::min(orow, ocol);
      const int32_t* b = h.colind.data() + h.rowptr[i];
      const int32_t* e = h.colind.data() + h.rowptr[i + 1];
      return (int64_t)(std::lower_bound(b, e, (int32_t)c) - h.colind.data());
    };
    std::vector<std::vector<int32_t>> roots(S.nlevels);
    for (int64_t b = 0; b < S.M(); ++b)
      if (h.iroot[b] == b && S.r(b) > 0) roots[S.level[b]].push_back((int32_t)b);
    // the forward solves' pull lists: per column, the zr slots of the in-block rows
    std::vector<int64_t> cnt((size_t)S.n + 1, 0);
    for (int64_t k = 0; k < S.M(); ++k)
      if (inter(k))
        for (int64_t p = S.rows_ptr[k]; p < S.rows_ptr[k] + rr(k); ++p) ++cnt[S.rows[p] + 1];
    for (int64_t i = 0; i < S.n; ++i) cnt[i + 1] += cnt[i];
    Q->ipull_idx.assign((size_t)cnt[S.n], 0);
    {
      std::vector<int64_t> nx(cnt.begin(), cnt.end() - 1);
      for (int64_t k = 0; k < S.M(); ++k)
        if (inter(k))
          for (int64_t p = S.rows_ptr[k]; p < S.rows_ptr[k] + rr(k); ++p) Q->ipull_idx[(size_t)nx[S.rows[p]]++] = p;
    }
    Q->ipull_ptr = std::move(cnt);
    for (int32_t L = 0; L < S.nlevels; ++L) {
      IntLevel& q = il[L];
      if (roots[L].empty()) continue;
      q.steps.assign(L + 1, {0, 0});
      std::vector<std::vector<IntSn>> by_l(L + 1);
      q.g0 = (int64_t)Q->cp_tgt.size();          // backward targets: the blocks' columns
      std::vector<std::array<int64_t, 3>> fe;   // (target row, column, value index)
      for (int32_t b : roots[L]) {
        int64_t s0 = b;
        while (s0 > 0 && h.iroot[s0 - 1] == b) --s0;
        const int64_t a = S.first[s0], e = S.first[b + 1];
        for (int64_t k = s0; k <= b; ++k) {
          IntSn t{};
          t.m = m_off(k); t.mld = m_ld(k); t.lo = h.r_in[k] > 0 ? h.lo_in[k] : 0; t.rh = h.r_in[k];
          t.rows = S.rows_ptr[k]; t.first = S.first[k]; t.c = S.c(k);
          t.a = a; t.b = e; t.root = (k == b);
          by_l[S.level[k]].push_back(t);
          bytes += 2.0 * 8.0 * ((double)t.c * (t.c + 1) / 2 + (double)t.rh * t.c);
        }
        // backward coupling: every column of the block (zero when it has no entry)
        for (int64_t cn = a; cn < e; ++cn) {
          const int64_t old = S.perm[cn];
          std::vector<std::pair<int64_t, int64_t>> ent;   // (row, value index)
          for (int64_t p = h.rowptr[old]; p < h.rowptr[old + 1]; ++p) {
            const int64_t rn = S.iperm[h.colind[p]];
            if (rn >= e) {
              ent.push_back({rn, lower_entry(old, h.colind[p])});
              fe.push_back({rn, cn, ent.back().second});
            }
          }
          std::sort(ent.begin(), ent.end());
          Q->cp_tgt.push_back(cn);
          Q->cp_ptr.push_back((int64_t)Q->cp_vidx.size());
          for (auto& en : ent) { Q->cp_vidx.push_back(en.second); Q->cp_xidx.push_back(en.first); }
          bytes += 24.0 * (double)ent.size() + 8.0;
        }
      }
      q.ng = (int64_t)Q->cp_tgt.size() - q.g0;
      for (int32_t l = 0; l <= L; ++l) {
        q.steps[l] = {(int64_t)Q->isns.size(), (int64_t)by_l[l].size()};
        Q->isns.insert(Q->isns.end(), by_l[l].begin(), by_l[l].end());
      }
      // forward coupling: each target row once, its entries by column
      std::sort(fe.begin(), fe.end());
      q.f0 = (int64_t)Q->cp_tgt.size();
      for (size_t u = 0; u < fe.size(); ++u) {
        if (u == 0 || fe[u][0] != fe[u - 1][0]) {
          Q->cp_tgt.push_back(fe[u][0]);
          Q->cp_ptr.push_back((int64_t)Q->cp_vidx.size());
        }
        Q->cp_vidx.push_back(fe[u][2]);
        Q->cp_xidx.push_back(fe[u][1]);
      }
      q.nf = (int64_t)Q->cp_tgt.size() - q.f0;
      bytes += 24.0 * (double)fe.size() + 16.0 * (double)q.nf;
    }
    Q->cp_ptr.push_back((int64_t)Q->cp_vidx.size());
  }
  auto fwd_tail = [&](int32_t L) {
    if (!ib || il[L].steps.empty()) return;
    for (int32_t l = L; l >= 0; --l) cmd(kCmdInterior, il[L].steps[l].first, il[L].steps[l].second, 0);
    cmd(kCmdCoupling, il[L].f0, il[L].nf, 0);
  };
  auto bwd_tail = [&](int32_t L) {
    if (!ib || il[L].steps.empty()) return;
    cmd(kCmdCoupling, il[L].g0, il[L].ng, 1);
    for (int32_t l = 0; l <= L; ++l) cmd(kCmdInterior, il[L].steps[l].first, il[L].steps[l].second, 1);
  };
  // forward sweep, levels ascending
  for (int32_t L = 0; L < S.nlevels; ++L) {
    if (L < nsmall) {
      small_cmd(kCmdSweepFwd, small[L]);
      fwd_tail(L);
      continue;
    }
    if (L == nsmall && !outside.empty()) {
      const int64_t r0 = (int64_t)Q->rg_rows.size();
      for (size_t u = 0; u < outside.size(); ++u) {
        if (u == 0 || outside[u].first != outside[u - 1].first) {
          Q->rg_rows.push_back(outside[u].first);
          Q->rg_ptr.push_back((int64_t)Q->rg_contrib.size());
        }
        Q->rg_contrib.push_back(outside[u].second);
      }
      cmd(kCmdRowGather, r0, (int64_t)Q->rg_rows.size() - r0, r0);
    }
    const auto& lev = S.by_level[L];
    // f3: w_C = L_j^{-1} y_C with the stored inverse (transposed upper block), and in the
    //     same launch f4: t_j = U_j^T w_C = W_j^T y_C for compressed supernodes
    std::vector<ColDotTask> st;
    for (int32_t j : lev) {
      const int32_t c = S.c(j), r = S.r(j);
      for (int32_t col0 = 0; col0 < c; col0 += 16) {
        ColDotTask t{};
        t.x = m_off(j); t.ldx = m_ld(j);
        t.in = h.a_y + S.first[j]; t.idx = -1; t.out = h.a_w + S.first[j];
        t.rows = c; t.ncols = c; t.col0 = col0; t.tri = 1;
        st.push_back(t);
      }
      bytes += 8.0 * c * (c + 1) / 2;
    }
    for (int32_t j : lev) {
      if (!iscomp(j)) continue;
      const CompSlot& C = h.comp[j];
      for (int32_t col0 = 0; col0 < C.ell; col0 += 16) {
        ColDotTask t{};
        t.x = C.Uj; t.ldx = S.c(j); t.in = h.a_y + S.first[j]; t.idx = -1; t.out = C.tvq;
        t.rows = S.c(j); t.ncols = -(1 + C.qslot); t.kmax = C.ell; t.col0 = col0; t.tri = 0;
        st.push_back(t);
      }
    }
    coldot_stage(st);
    // f5: t_j = L^O_j w_C (explicit) or V_j t (compressed), column-major products in
    //     64-row pieces (coalesced over the rows), into the R_j rows of the zr buffer
    {
      const int64_t g0 = (int64_t)Q->gemv.size();
      for (int32_t j : lev) {
        const int32_t c = S.c(j), r = rr(j);
        for (int32_t t0 = 0; t0 < r; t0 += 64) {
          GemvTask t{};
          if (iscomp(j)) {
            const CompSlot& C = h.comp[j];
            t.x = C.Vj + t0; t.kdim = -(1 + C.qslot); t.kmax = C.ell; t.v = C.tvq;
          } else {
            t.x = lox(j) + t0; t.kdim = c; t.kmax = c; t.v = h.a_w + S.first[j];
          }
          t.ldx = r; t.rows = std::min(64, r - t0);
          t.out = h.a_zr + S.rows_ptr[j] + t0;
          Q->gemv.push_back(t);
        }
      }
      cmd(kCmdGemvN, g0, (int64_t)Q->gemv.size() - g0);
    }
    // f6: y_i -= the level's t entries of row i, in supernode order (each row once per launch)
    {
      std::vector<std::pair<int64_t, int64_t>> tc;   // (target row, zr index)
      for (int32_t j : lev)
        for (int64_t p = S.rows_ptr[j]; p < S.rows_ptr[j] + rr(j); ++p) tc.push_back({S.rows[p], p});
      std::stable_sort(tc.begin(), tc.end(), [](const std::pair<int64_t, int64_t>& x,
                                                const std::pair<int64_t, int64_t>& y) { return x.first < y.first; });
      const int64_t r0 = (int64_t)Q->rg_rows.size();
      for (size_t u = 0; u < tc.size(); ++u) {
        if (u == 0 || tc[u].first != tc[u - 1].first) {
          Q->rg_rows.push_back(tc[u].first);
          Q->rg_ptr.push_back((int64_t)Q->rg_contrib.size());
        }
        Q->rg_contrib.push_back(tc[u].second);
      }
      const int64_t nr = (int64_t)Q->rg_rows.size() - r0;
      if (nr > 0) cmd(kCmdRowGather, r0, nr, r0);
    }
    fwd_tail(L);
  }
  Q->rg_ptr.push_back((int64_t)Q->rg_contrib.size());
  // backward sweep, levels descending
  for (int32_t L = S.nlevels - 1; L >= 0; --L) {
    bwd_tail(L);
    if (L < nsmall) {
      small_cmd(kCmdSweepBwd, small[L]);
      continue;
    }
    const auto& lev = S.by_level[L];
    // b0: z over R_j gathered once per supernode into the contiguous buffer zr
    {
      const int64_t g0q = (int64_t)Q->gath.size() / 2;
      for (int32_t j : lev)
        for (int32_t t0 = 0; t0 < rr(j); t0 += 1024) {   // pieces of <= 1024 rows, one workgroup each
          Q->gath.push_back(S.rows_ptr[j] + t0);
          Q->gath.push_back(std::min(1024, rr(j) - t0));
        }
      const int64_t ng = (int64_t)Q->gath.size() / 2 - g0q;
      if (ng > 0) {
        Cmd c{};
        c.type = kCmdGatherRows; c.klass = RSC_K_PCG; c.off = g0q; c.count = ng;
        Q->fwd_bwd.push_back(c);
      }
    }
    // b1: s_C = (L^O_j)^T z_R (dense) or u = V_j^T z_R (compressed)
    std::vector<ColDotTask> st;
    for (int32_t j : lev) {
      const int32_t c = S.c(j), r = S.r(j);
      if (r == 0) continue;
      if (iscomp(j)) {
        const CompSlot& C = h.comp[j];
        for (int32_t col0 = 0; col0 < C.ell; col0 += 16) {
          ColDotTask t{};
          t.x = C.Vj; t.ldx = r; t.in = h.a_zr + S.rows_ptr[j]; t.idx = -1; t.out = C.u;
          t.rows = r; t.ncols = -(1 + C.qslot); t.kmax = C.ell; t.col0 = col0; t.tri = 0;
          st.push_back(t);
        }
      } else {
        if (rr(j) == 0) continue;   // an interior supernode with no rows inside its block
        for (int32_t col0 = 0; col0 < c; col0 += 16) {
          ColDotTask t{};
          t.x = lox(j); t.ldx = rr(j); t.in = h.a_zr + S.rows_ptr[j];
          t.idx = -1; t.out = h.a_s + S.first[j];
          t.rows = rr(j); t.ncols = c; t.col0 = col0; t.tri = 0;
          st.push_back(t);
        }
        bytes += 2.0 * 8.0 * (double)rr(j) * c;   // read by both sweeps
      }
    }
    KeptParts kept;                // chunked s_C and u: added up by the b2 chunks below
    const int32_t b1_slots = coldot_stage(st, &kept);
    for (int32_t j : lev)
      if (iscomp(j)) bytes += 2.0 * 8.0 * (double)(S.c(j) + S.r(j)) * h.comp[j].ell;
    // b2: z_C = L_j^{-T} (w_C - s_C) by 64-row blocks, the columns of each block cut
    // into chunks (about 1024 per level) whose partial blocks are then stored in order;
    // for a compressed supernode z_C = M_j w_C - W_j u (s_C = U_j u), the rows of W_j u
    // as further chunks of the same blocks
    {
      double cols = 0;
      for (int32_t j : lev)
        for (int32_t i0 = 0; i0 < S.c(j); i0 += 64) cols += S.c(j) - i0;
      const int32_t width =
          (int32_t)std::min<double>(kRowChunkMax, std::max(256.0, std::ceil(cols / 1024.0)));
      const int64_t c0r = (int64_t)Q->rchunks.size(), a0 = (int64_t)Q->papply.size();
      int32_t slot = b1_slots;     // past the column dots' blocks that the chunks read
      for (int32_t j : lev) {
        const int32_t c = S.c(j);
        const int64_t sout = iscomp(j) ? h.comp[j].u : h.a_s + S.first[j];
        const auto kp = kept.find(sout);
        const int32_t sbase = kp == kept.end() ? 0 : kp->second.first;
        const int32_t sns = kp == kept.end() ? 0 : kp->second.second;
        for (int32_t i0 = 0; i0 < c; i0 += 64) {
          const int32_t s0 = slot;
          for (int32_t t0 = i0; t0 < c; t0 += width) {
            RowChunk t{};
            t.m = m_off(j); t.ld = m_ld(j); t.c = c; t.i0 = i0;
            t.w = h.a_w + S.first[j];
            t.s = (!iscomp(j) && rr(j) > 0 && sns == 0) ? h.a_s + S.first[j] : -1;
            if (!iscomp(j)) { t.sbase = sbase; t.sns = sns; }
            t.t0 = t0; t.t1 = std::min(c, t0 + width); t.slot = slot++;
            Q->rchunks.push_back(t);
          }
          if (iscomp(j)) {
            const CompSlot& C = h.comp[j];
            for (int32_t t0 = 0; t0 < C.ell; t0 += width) {
              RowChunk t{};
              t.kind = 1; t.m = C.Uj; t.ld = c; t.c = c; t.i0 = i0; t.w = C.u; t.s = -1;
              t.qslot = C.qslot; t.kmax = C.ell; t.sbase = sbase; t.sns = sns;
              t.t0 = t0; t.t1 = std::min(C.ell, t0 + width); t.slot = slot++;
              Q->rchunks.push_back(t);
            }
          }
          Q->papply.push_back(PartApply{h.a_zz + S.first[j] + i0, std::min(64, c - i0), s0, slot - s0, 1});
        }
        bytes += 8.0 * c * (c + 1) / 2;
      }
      Q->part_slots = std::max<int64_t>(Q->part_slots, slot);
      cmd(kCmdRowPart, c0r, (int64_t)Q->rchunks.size() - c0r);
      cmd(kCmdPartApply, a0, (int64_t)Q->papply.size() - a0);
    }
  }
  Q->bytes = bytes;
  Error e;
  if ((e = upload(Q->d_gemv, Q->gemv)).code) return e;
  if ((e = upload(Q->d_isns, Q->isns)).code) return e;
  if ((e = upload(Q->d_ipull_ptr, Q->ipull_ptr)).code) return e;
  if ((e = upload(Q->d_ipull_idx, Q->ipull_idx)).code) return e;
  if ((e = upload(Q->d_cp_tgt, Q->cp_tgt)).code) return e;
  if ((e = upload(Q->d_cp_ptr, Q->cp_ptr)).code) return e;
  if ((e = upload(Q->d_cp_vidx, Q->cp_vidx)).code) return e;
  if ((e = upload(Q->d_cp_xidx, Q->cp_xidx)).code) return e;
  if ((e = upload(Q->d_coldot, Q->coldot)).code) return e;
  if ((e = upload(Q->d_rchunks, Q->rchunks)).code) return e;
  if ((e = upload(Q->d_papply, Q->papply)).code) return e;
  {
    std::vector<double> zero((size_t)std::max<int64_t>(Q->part_slots, 1) * 64, 0.0);
    if ((e = upload(Q->d_part, zero)).code) return e;
  }
  if ((e = upload(Q->d_gath, Q->gath)).code) return e;
  if ((e = upload(Q->d_rg_rows, Q->rg_rows)).code) return e;
  if ((e = upload(Q->d_rg_ptr, Q->rg_ptr)).code) return e;
  if ((e = upload(Q->d_rg_contrib, Q->rg_contrib)).code) return e;
  if ((e = upload(Q->d_sweep, Q->sweep)).code) return e;
  if ((e = upload(Q->d_pull_ptr, Q->pull_ptr)).code) return e;
  if ((e = upload(Q->d_pull_idx, Q->pull_idx)).code) return e;
  h.splan = std::move(Q);
  return kOk;
}

// One preconditioner apply: z (arena a_z) = M^{-1} r (arena a_r).
static Error apply_cmds(Handle& h, hipStream_t s, std::vector<EventPair>* evs,
                        double* part_buf = nullptr) {
  Cmd g{}; g.type = kCmdGatherPerm; g.klass = RSC_K_PCG; g.count = 1; g.a = h.a_r; g.b = h.a_y;
  Cmd z{}; z.type = kCmdScatterPerm; z.klass = RSC_K_PCG; z.count = 1; z.a = h.a_zz; z.b = h.a_z;
  std::vector<Cmd> all;
  all.push_back(g);
  all.insert(all.end(), h.splan->fwd_bwd.begin(), h.splan->fwd_bwd.end());
  all.push_back(z);
  return run_cmds(h, all, nullptr, h.splan.get(), s, evs, part_buf);
}

static Error ensure_solve(Handle& h) {
  if (!h.factored) return Error{RSC_ERR_STATE, "no successful rsc_factor on this handle"};
  if (h.splan && h.splan->f32_tasks != h.f32_valid) {   // M_j read from the other copy
    SolvePlan& Q = *h.splan;
    if (Q.graph_a) (void)hipGraphExecDestroy(Q.graph_a);
    if (Q.graph_b) (void)hipGraphExecDestroy(Q.graph_b);
    if (Q.graph_apply) (void)hipGraphExecDestroy(Q.graph_apply);
    h.splan.reset();
  }
  if (!h.splan) return build_solve_plan(h);
  return kOk;
}

Error apply_preconditioner(Handle& h, const double* r, double* z, hipStream_t stream) {
  Error e = ensure_solve(h);
  if (e.code) return e;
  HIPCHK(hipMemcpyAsync(h.arena.p + h.a_r, r, sizeof(double) * (size_t)h.S.n, hipMemcpyDeviceToDevice, stream));
  solve_graph_mode(h);
  if (h.opt.use_graph && !h.profiling) {
    if (!h.splan->graph_apply)
      if ((e = capture(h, [&](hipStream_t s) { return apply_cmds(h, s, nullptr); }, &h.splan->graph_apply)).code)
        return e;
    HIPCHK(hipGraphLaunch(h.splan->graph_apply, stream));
  } else {
    if ((e = apply_cmds(h, stream, nullptr)).code) return e;
  }
  HIPCHK(hipMemcpyAsync(z, h.arena.p + h.a_z, sizeof(double) * (size_t)h.S.n, hipMemcpyDeviceToDevice, stream));
  return kOk;
}

// The same apply launched eagerly on the caller's stream with the sweeps' partial sums
// in the static per-GPU buffer: allocates nothing (the sweep plan was built by
// rsc_factor).  Every stage writes each partial block it reads before reading it, so
// the buffer needs no clearing between calls.
Error apply_preconditioner_noalloc(Handle& h, const double* r, double* z, hipStream_t stream) {
  if (!h.factored || !h.dev_ready) return Error{RSC_ERR_STATE, "no successful rsc_factor on this handle"};
  if (!h.splan) return Error{RSC_ERR_STATE, "no sweep plan (rsc_factor builds it)"};
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != h.device) return Error{RSC_ERR_STATE, "handle is bound to another device"};
  const int64_t need = std::max<int64_t>(h.splan->part_slots, 1) * 64;
  if (need > kApplyScratchDoubles)
    return Error{RSC_ERR_INVALID_ARG, "the sweeps need " + std::to_string(8 * need) +
                                          " bytes of partial sums; the static buffer holds " +
                                          std::to_string(8 * kApplyScratchDoubles)};
  double* part = nullptr;
  HIPCHK(apply_scratch(&part));
  HIPCHK(hipMemcpyAsync(h.arena.p + h.a_r, r, sizeof(double) * (size_t)h.S.n, hipMemcpyDeviceToDevice, stream));
  Error e = apply_cmds(h, stream, nullptr, part);
  if (e.code) return e;
  HIPCHK(hipMemcpyAsync(z, h.arena.p + h.a_z, sizeof(double) * (size_t)h.S.n, hipMemcpyDeviceToDevice, stream));
  return kOk;
}

// ------------------------------------------------------------------ PCG

Error pcg(Handle& h, const double* b, double* x, double rtol, int32_t max_iter, hipStream_t stream,
          rsc_pcg_result* out) {
  Error e = ensure_solve(h);
  if (e.code) return e;
  double* A = h.arena.p;
  int32_t* I = h.ints.p;
  const int64_t n = h.S.n;
  const int32_t nseg = (int32_t)h.seg_first.size() - 1;
  const int nc = h.nchunks;
  const Chunk* ch = h.d_chunks.p;
  const PcgScalars sc = h.sc;
  double* partial = A + h.a_partial;
  const double* vals = A + h.a_values;
  std::vector<EventPair> evs;
  std::vector<EventPair>* pe = h.profiling ? &evs : nullptr;

  auto part_a = [&](hipStream_t s) -> Error {
    launch_spmv_dot(ch, nc, h.d_rowptr.p, h.d_colind.p, vals, A + sc.p, A + sc.Ap, partial, s);
    launch_seg_step(h.d_seg_chunk_ptr.p, nseg, partial, sc, rtol, A, I, 0, s);   // p^T A p, alpha
    launch_pcg_xr(ch, nc, sc, A, I, partial, s);
    launch_seg_step(h.d_seg_chunk_ptr.p, nseg, partial, sc, rtol, A, I, 1, s);   // r^T r, test
    HIPCHK(hipGetLastError());
    return kOk;
  };
  auto part_b = [&](hipStream_t s) -> Error {
    Error r = apply_cmds(h, s, nullptr);
    if (r.code) return r;
    launch_dot_partial(ch, nc, A + sc.r, A + sc.z, partial, s);
    launch_seg_step(h.d_seg_chunk_ptr.p, nseg, partial, sc, rtol, A, I, 2, s);   // r^T z, beta
    launch_pcg_p(ch, nc, sc, A, I, 0, s);
    HIPCHK(hipGetLastError());
    return kOk;
  };

  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipMemcpyAsync(A + h.a_b, b, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, stream));
  HIPCHK(hipEventRecord(e0, stream));
  // start: x = 0, r = b, bnorm, z = M r, rz = r.z, p = z
  launch_fill(A + sc.x, n, 0.0, stream);
  launch_copy(n, A + h.a_b, A + sc.r, stream);
  launch_dot_partial(ch, nc, A + h.a_b, A + h.a_b, partial, stream);
  launch_seg_sum(h.d_seg_chunk_ptr.p, nseg, partial, A + sc.bnorm, stream);
  launch_pcg_start(nseg, sc, A, I, stream);
  if ((e = apply_cmds(h, stream, pe)).code) return e;
  launch_dot_partial(ch, nc, A + sc.r, A + sc.z, partial, stream);
  launch_seg_sum(h.d_seg_chunk_ptr.p, nseg, partial, A + sc.rz, stream);
  launch_pcg_p(ch, nc, sc, A, I, 1, stream);
  HIPCHK(hipGetLastError());

  const bool graphs = h.opt.use_graph && !h.profiling;
  solve_graph_mode(h);
  SolvePlan* Q = h.splan.get();
  if (graphs && Q->graph_a && Q->v_rtol != rtol) {
    (void)hipGraphExecDestroy(Q->graph_a);
    Q->graph_a = nullptr;
  }
  if (graphs && !Q->graph_a) {
    if ((e = capture(h, part_a, &Q->graph_a)).code) return e;
    Q->v_rtol = rtol;
  }
  if (graphs && !Q->graph_b)
    if ((e = capture(h, part_b, &Q->graph_b)).code) return e;
  int32_t flags[2] = {0, 0};
  int32_t it = 0;
  bool breakdown = false;
  for (; it < max_iter; ++it) {
    if (graphs) { HIPCHK(hipGraphLaunch(Q->graph_a, stream)); }
    else if ((e = part_a(stream)).code) return e;
    HIPCHK(hipMemcpyAsync(flags, I + sc.any, sizeof(flags), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (flags[1]) { breakdown = true; break; }
    if (!flags[0]) break;
    if (graphs) { HIPCHK(hipGraphLaunch(Q->graph_b, stream)); }
    else {
      if (pe) {
        if ((e = apply_cmds(h, stream, pe)).code) return e;
        launch_dot_partial(ch, nc, A + sc.r, A + sc.z, partial, stream);
        launch_seg_step(h.d_seg_chunk_ptr.p, nseg, partial, sc, rtol, A, I, 2, stream);
        launch_pcg_p(ch, nc, sc, A, I, 0, stream);
      } else if ((e = part_b(stream)).code) {
        return e;
      }
    }
  }
  HIPCHK(hipEventRecord(e1, stream));
  // true residual ||b - A x|| / ||b|| per system
  launch_spmv_dot(ch, nc, h.d_rowptr.p, h.d_colind.p, vals, A + sc.x, A + sc.Ap, partial, stream);
  launch_resid_partial(ch, nc, A + h.a_b, A + sc.Ap, partial, stream);
  launch_seg_sum(h.d_seg_chunk_ptr.p, nseg, partial, A + h.a_seg + 8 * (int64_t)nseg, stream);
  HIPCHK(hipGetLastError());
  std::vector<int32_t> iters(nseg);
  std::vector<double> rel(nseg), bn(nseg), tr(nseg);
  HIPCHK(hipMemcpyAsync(iters.data(), I + sc.iters, sizeof(int32_t) * nseg, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(rel.data(), A + sc.rel, sizeof(double) * nseg, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(bn.data(), A + sc.bnorm, sizeof(double) * nseg, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(tr.data(), A + h.a_seg + 8 * (int64_t)nseg, sizeof(double) * nseg,
                        hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(x, A + sc.x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (pe && (e = collect_events(h, evs)).code) return e;
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h.t_pcg_ms = ms;
  bool all_conv = true;
  for (int32_t s = 0; s < nseg; ++s) {
    out[s].iters = iters[s];
    out[s].rel_residual = rel[s];
    out[s].true_residual = bn[s] > 0 ? std::sqrt(tr[s]) / bn[s] : 0.0;
    out[s].converged = (bn[s] == 0.0 || rel[s] <= rtol) ? 1 : 0;
    if (!out[s].converged) all_conv = false;
  }
  if (breakdown) return Error{RSC_ERR_BREAKDOWN, "non-positive curvature or r^T z in PCG"};
  if (!all_conv) return Error{RSC_ERR_NOT_CONVERGED, "PCG did not reach rtol within max_iter"};
  return kOk;
}

Error grad_values(Handle& h, const double* lam, const double* x, double* g, hipStream_t stream) {
  Error e = ensure_device(h);
  if (e.code) return e;
  launch_grad_values(h.S.n, h.d_rowptr.p, h.d_colind.p, lam, x, g, stream);
  HIPCHK(hipGetLastError());
  return kOk;
}

}  // namespace rsc
