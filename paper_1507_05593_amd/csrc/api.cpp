// C ABI of the solver (declarations and contracts in include/rsc.h).
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/rsc.h"
#include "kernels.h"
#include "runtime.h"

// Counts live handles; declared before the handle state so that it is destroyed after
// the state has returned its device memory to the allocator that gave it.
struct HandleCount {
  HandleCount() { rsc::handle_count(+1); }
  ~HandleCount() { rsc::handle_count(-1); }
};

struct rsc_handle_s {
  HandleCount count;
  rsc::Handle h;
};

namespace {

thread_local std::string g_last_error;

rsc_status fail(rsc_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

rsc_status ret(const rsc::Error& e) {
  if (e.code != RSC_OK) g_last_error = e.msg;
  return e.code;
}

rsc_status check_options(const rsc_options& o) {
  if (o.leaf_max < 1 || o.tau_O < 1 || o.oversample < 0 || o.power_iters < 0 || !(o.alpha_O > 0) ||
      o.precision < RSC_FP64 || o.precision > RSC_MIXED_FP32 ||
      (o.gemm_tile != 0 && o.gemm_tile != 64 && o.gemm_tile != 128) || o.sweep_small_c < 0 ||
      o.sweep_small_c > 1024 || o.tau_D < 0 || o.tau_D == 1 || o.interior < 0 || o.interior > 1 || !(o.alpha_D > 0) || !(o.alpha_D < 1e6))
    return fail(RSC_ERR_INVALID_ARG, "option out of range");
  return RSC_OK;
}

rsc_status analyze_impl(int32_t count, const int64_t* n, const int64_t* const* rowptr,
                        const int32_t* const* colind, const double* xyz, const rsc_options* opt,
                        rsc_handle* out) {
  if (!out || count < 1 || !n || !rowptr || !colind) return fail(RSC_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  rsc_options o;
  rsc_default_options(&o);
  if (opt) o = *opt;
  if (rsc_status s = check_options(o)) return s;
  auto t0 = std::chrono::steady_clock::now();
  rsc_handle_s* H = new (std::nothrow) rsc_handle_s();
  if (!H) return fail(RSC_ERR_OUT_OF_MEMORY, "handle");
  rsc::Handle& h = H->h;
  h.opt = o;
  try {
    int64_t total = 0, nnz = 0;
    for (int32_t s = 0; s < count; ++s) {
      if (n[s] < 0 || !rowptr[s] || (n[s] > 0 && !colind[s])) {
        delete H;
        return fail(RSC_ERR_INVALID_ARG, "bad system " + std::to_string(s));
      }
      std::string msg = rsc::check_pattern(n[s], rowptr[s], colind[s]);
      if (!msg.empty()) {
        delete H;
        return fail(RSC_ERR_PATTERN, "system " + std::to_string(s) + ": " + msg);
      }
      total += n[s];
      nnz += rowptr[s][n[s]];
    }
    if (total > INT32_MAX - 1) {
      delete H;
      return fail(RSC_ERR_INVALID_ARG, "order exceeds the int32 column index range");
    }
    h.rowptr.assign(1, 0);
    h.colind.reserve(nnz);
    h.seg_first.assign(1, 0);
    int64_t base = 0;
    for (int32_t s = 0; s < count; ++s) {
      for (int64_t i = 0; i < n[s]; ++i) {
        for (int64_t p = rowptr[s][i]; p < rowptr[s][i + 1]; ++p)
          h.colind.push_back((int32_t)(colind[s][p] + base));
        h.rowptr.push_back((int64_t)h.colind.size());
      }
      base += n[s];
      h.seg_first.push_back(base);
    }
    if (xyz)
      for (int64_t i = 0; i < 3 * total; ++i)
        if (!std::isfinite(xyz[i])) {
          delete H;
          return fail(RSC_ERR_INVALID_ARG, "non-finite position of index " + std::to_string(i / 3));
        }
    rsc::build_symbolic(total, h.rowptr.data(), h.colind.data(), o.leaf_max, o.tau_D, xyz, h.S);
    h.S.systems = count;
    h.S.sys_first = h.seg_first;
    rsc::plan_layout(h);
  } catch (const std::bad_alloc&) {
    delete H;
    return fail(RSC_ERR_OUT_OF_MEMORY, "host memory during analysis");
  } catch (const std::exception& e) {
    delete H;
    return fail(RSC_ERR_PATTERN, e.what());
  }
  h.t_analyze_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = H;
  return RSC_OK;
}

}  // namespace

extern "C" {

void rsc_default_options(rsc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->leaf_max = 64;
  o->tau_O = 32;
  o->oversample = 10;
  o->power_iters = 0;
  o->alpha_O = 1.0;
  o->seed = 0;
  o->precision = RSC_FP64;
  o->use_graph = 1;
  o->retry = 1;
  o->sweep_small_c = 64;
  o->tau_D = 0;
  o->alpha_D = 0.5;
}

rsc_status rsc_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind,
                       const rsc_options* opt, rsc_handle* out) {
  return analyze_impl(1, &n, &rowptr, &colind, nullptr, opt, out);
}

rsc_status rsc_analyze_coords(int64_t n, const int64_t* rowptr, const int32_t* colind,
                              const double* xyz, const rsc_options* opt, rsc_handle* out) {
  if (!xyz && n > 0) {
    if (out) *out = nullptr;
    return fail(RSC_ERR_INVALID_ARG, "null positions");
  }
  return analyze_impl(1, &n, &rowptr, &colind, xyz, opt, out);
}

rsc_status rsc_analyze_batch(int32_t count, const int64_t* n, const int64_t* const* rowptr,
                             const int32_t* const* colind, const rsc_options* opt, rsc_handle* out) {
  return analyze_impl(count, n, rowptr, colind, nullptr, opt, out);
}

rsc_status rsc_factor(rsc_handle H, const double* values, double tol, void* stream) {
  if (!H || (!values && H->h.S.nnz > 0)) return fail(RSC_ERR_INVALID_ARG, "null argument");
  if (!(tol >= 0.0) || !(tol < 1.0)) return fail(RSC_ERR_INVALID_ARG, "tol must be in [0, 1)");
  return ret(rsc::factor(H->h, values, tol, (hipStream_t)stream));
}

rsc_status rsc_pcg(rsc_handle H, const double* b, double* x, double rtol, int32_t max_iter,
                   void* stream, rsc_pcg_result* out) {
  if (!H || !out || (H->h.S.n > 0 && (!b || !x))) return fail(RSC_ERR_INVALID_ARG, "null argument");
  if (!(rtol > 0.0) || max_iter < 0) return fail(RSC_ERR_INVALID_ARG, "rtol must be > 0, max_iter >= 0");
  return ret(rsc::pcg(H->h, b, x, rtol, max_iter, (hipStream_t)stream, out));
}

rsc_status rsc_apply_preconditioner(rsc_handle H, const double* r, double* z, void* stream) {
  if (!H || (H->h.S.n > 0 && (!r || !z))) return fail(RSC_ERR_INVALID_ARG, "null argument");
  if (r == z && r) return fail(RSC_ERR_INVALID_ARG, "r and z may not alias");
  return ret(rsc::apply_preconditioner(H->h, r, z, (hipStream_t)stream));
}

rsc_status rsc_apply_preconditioner_noalloc(rsc_handle H, const double* r, double* z, void* stream) {
  if (!H || (H->h.S.n > 0 && (!r || !z))) return fail(RSC_ERR_INVALID_ARG, "null argument");
  if (r == z && r) return fail(RSC_ERR_INVALID_ARG, "r and z may not alias");
  return ret(rsc::apply_preconditioner_noalloc(H->h, r, z, (hipStream_t)stream));
}

rsc_status rsc_spectral_coordinates(rsc_handle H, int32_t steps, uint64_t seed, double* xyz, double* ritz,
                                    void* stream) {
  if (!H || !xyz) return fail(RSC_ERR_INVALID_ARG, "null argument");
  return ret(rsc::spectral_coordinates(H->h, steps, seed, xyz, ritz, (hipStream_t)stream));
}

rsc_status rsc_grad_values(rsc_handle H, const double* lambda, const double* x, double* g, void* stream) {
  if (!H || (H->h.S.n > 0 && (!lambda || !x || !g))) return fail(RSC_ERR_INVALID_ARG, "null argument");
  return ret(rsc::grad_values(H->h, lambda, x, g, (hipStream_t)stream));
}

rsc_status rsc_grad_faces(int64_t nfaces, const int32_t* face_i, const int32_t* face_j,
                          const double* lambda, const double* x, double* g, void* stream) {
  if (nfaces < 0) return fail(RSC_ERR_INVALID_ARG, "negative face count");
  if (nfaces == 0) return RSC_OK;
  if (!face_i || !face_j || !lambda || !x || !g) return fail(RSC_ERR_INVALID_ARG, "null argument");
  rsc::launch_grad_faces(nfaces, face_i, face_j, lambda, x, g, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RSC_ERR_DEVICE, hipGetErrorString(e));
  return RSC_OK;
}

rsc_status rsc_get_sizes(rsc_handle H, int64_t* n, int64_t* nnz, int64_t* supernodes,
                         int64_t* levels, int64_t* systems) {
  if (!H) return fail(RSC_ERR_INVALID_ARG, "null handle");
  if (n) *n = H->h.S.n;
  if (nnz) *nnz = H->h.S.nnz;
  if (supernodes) *supernodes = H->h.S.M();
  if (levels) *levels = H->h.S.nlevels;
  if (systems) *systems = (int64_t)H->h.seg_first.size() - 1;
  return RSC_OK;
}

rsc_status rsc_get_permutation(rsc_handle H, int64_t* perm) {
  if (!H || !perm) return fail(RSC_ERR_INVALID_ARG, "null argument");
  std::memcpy(perm, H->h.S.perm.data(), sizeof(int64_t) * H->h.S.perm.size());
  return RSC_OK;
}

rsc_status rsc_get_supernodes(rsc_handle H, int64_t* first, int32_t* parent, int32_t* level,
                              int32_t* kind) {
  if (!H) return fail(RSC_ERR_INVALID_ARG, "null handle");
  const rsc::Symbolic& S = H->h.S;
  if (first) std::memcpy(first, S.first.data(), sizeof(int64_t) * S.first.size());
  if (parent) std::memcpy(parent, S.parent.data(), sizeof(int32_t) * S.parent.size());
  if (level) std::memcpy(level, S.level.data(), sizeof(int32_t) * S.level.size());
  if (kind) std::memcpy(kind, S.kind.data(), sizeof(int32_t) * S.kind.size());
  return RSC_OK;
}

rsc_status rsc_get_rowsets(rsc_handle H, int64_t* rowptr, int64_t* rows) {
  if (!H) return fail(RSC_ERR_INVALID_ARG, "null handle");
  const rsc::Symbolic& S = H->h.S;
  if (rowptr) std::memcpy(rowptr, S.rows_ptr.data(), sizeof(int64_t) * S.rows_ptr.size());
  if (rows) std::memcpy(rows, S.rows.data(), sizeof(int64_t) * S.rows.size());
  return RSC_OK;
}

rsc_status rsc_get_ranks(rsc_handle H, int32_t* ell, int32_t* q) {
  if (!H) return fail(RSC_ERR_INVALID_ARG, "null handle");
  rsc::Handle& h = H->h;
  const int64_t M = h.S.M();
  const bool comp = h.factored && h.fplan && h.fplan->compressed;
  if (ell)
    for (int64_t j = 0; j < M; ++j) ell[j] = (comp && h.compressible[j]) ? h.comp[j].ell : 0;
  if (q) {
    for (int64_t j = 0; j < M; ++j) q[j] = 0;
    if (comp) {
      if (hipMemcpy(q, h.ints.p + h.i_ranks, sizeof(int32_t) * M, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(RSC_ERR_DEVICE, "copy of ranks");
      for (int64_t j = 0; j < M; ++j)
        if (!h.compressible[j]) q[j] = 0;
    }
  }
  return RSC_OK;
}

rsc_status rsc_get_block(rsc_handle H, int64_t j, double* LD, double* LO, double* V, double* U) {
  if (!H) return fail(RSC_ERR_INVALID_ARG, "null handle");
  rsc::Handle& h = H->h;
  if (j < 0 || j >= h.S.M()) return fail(RSC_ERR_INVALID_ARG, "supernode out of range");
  if (!h.factored) return fail(RSC_ERR_STATE, "no factor");
  const int64_t c = h.S.c(j), r = h.S.r(j), ld = h.panel_ld[j];
  const double* P = h.arena.p + h.panel_off[j];
  if (hipDeviceSynchronize() != hipSuccess) return fail(RSC_ERR_DEVICE, "synchronize");
  const bool comp = h.fplan->compressed && h.compressible[j];
  if (LD && c > 0 &&
      hipMemcpy2D(LD, c * 8, P, ld * 8, c * 8, c, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(RSC_ERR_DEVICE, "copy LD");
  if (LO && comp && !h.opt.keep_lo)
    return fail(RSC_ERR_STATE, "L^O of a compressed supernode is not kept (rsc_options.keep_lo)");
  const bool inb = h.fplan->compressed && h.opt.interior && h.iroot[j] >= 0 && r > 0;
  if (LO && r > 0 && c > 0 && inb) {
    // an interior block's supernode: its rows inside the block, the rest not stored
    const int64_t ri = h.r_in[j];
    std::memset(LO, 0, sizeof(double) * r * c);
    if (ri > 0 && hipMemcpy2D(LO, r * 8, h.arena.p + h.lo_in[j], ri * 8, ri * 8, c, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(RSC_ERR_DEVICE, "copy LO");
  } else if (LO && r > 0 && c > 0) {
    if (hipMemcpy(LO, h.arena.p + h.lo_off[j], sizeof(double) * r * c,
                         hipMemcpyDeviceToHost) != hipSuccess) {
      return fail(RSC_ERR_DEVICE, "copy LO");
    }
  }
  if (comp && (V || U)) {
    int32_t q = 0;
    if (hipMemcpy(&q, h.ints.p + h.comp[j].qslot, 4, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(RSC_ERR_DEVICE, "copy rank");
    if (V && q > 0 &&
        hipMemcpy(V, h.arena.p + h.comp[j].Vj, sizeof(double) * r * q, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(RSC_ERR_DEVICE, "copy V");
    if (U && q > 0) {
      // the factor keeps W_j = (L^D_j)^{-T} U_j (the form the sweeps use): U_j = (L^D_j)^T W_j
      std::vector<double> W((size_t)c * q), L((size_t)c * c);
      if (hipMemcpy(W.data(), h.arena.p + h.comp[j].Uj, sizeof(double) * c * q, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy2D(L.data(), c * 8, P, ld * 8, c * 8, c, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(RSC_ERR_DEVICE, "copy U");
      for (int64_t k = 0; k < q; ++k)
        for (int64_t i = 0; i < c; ++i) {
          double acc = 0.0;
          for (int64_t t = i; t < c; ++t) acc += L[(size_t)t + (size_t)i * c] * W[(size_t)t + (size_t)k * c];
          U[i + k * c] = acc;
        }
    }
  }
  return RSC_OK;
}

rsc_status rsc_get_tree_depths(rsc_handle H, int32_t* depth) {
  if (!H || !depth) return fail(RSC_ERR_INVALID_ARG, "null argument");
  const rsc::Symbolic& S = H->h.S;
  for (int64_t j = 0; j < S.M(); ++j) depth[j] = S.depth[j];
  return RSC_OK;
}

rsc_status rsc_get_stats(rsc_handle H, rsc_stats* out) {
  if (!H || !out) return fail(RSC_ERR_INVALID_ARG, "null argument");
  rsc::Handle& h = H->h;
  const rsc::Symbolic& S = h.S;
  std::memset(out, 0, sizeof(*out));
  out->n = S.n;
  out->nnz = S.nnz;
  out->supernodes = S.M();
  out->levels = S.nlevels;
  out->systems = (int64_t)h.seg_first.size() - 1;
  out->failed_supernode = h.failed_supernode;
  out->precision_used = h.precision_used;
  out->retries = h.retries;
  out->t_analyze_ms = h.t_analyze_ms;
  out->t_factor_ms = h.t_factor_ms;
  out->t_pcg_ms = h.t_pcg_ms;
  out->device_bytes = 8.0 * (double)h.arena.n + 4.0 * (double)h.ints_size;
  out->device_bytes += 4.0 * (double)h.arena32.n;
  if (h.fplan) {
    out->device_bytes += 8.0 * (double)h.fplan->d_xc.n;
    out->gemm_tuned = h.fplan->tuned;
    out->gemm_tile128 = h.fplan->tuned128;
  }
  const bool comp = h.factored && h.fplan && h.fplan->compressed;
  std::vector<int32_t> q(S.M(), 0);
  if (comp && hipMemcpy(q.data(), h.ints.p + h.i_ranks, sizeof(int32_t) * S.M(), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(RSC_ERR_DEVICE, "copy of ranks");
  int64_t entries = 0;
  double fl_update = 0;
  const bool tree = comp && h.fplan->alpha_D > 0;
  for (int64_t j = 0; j < S.M(); ++j) {
    const int64_t c = S.c(j), r = S.r(j);
    if (tree && !h.tree[j].empty()) {
      // the block tree's storage: leaf triangles and every block's V_s, U_s
      int64_t te = 0;
      out->tree_supernodes++;
      for (const rsc::TreeNode& t : h.tree[j]) {
        const int64_t nc = t.cb - t.ca, nr = t.rb - t.ra;
        if (t.ht == 0) { te += nc * (nc + 1) / 2; continue; }
        out->tree_blocks++;
        out->tree_rank_sum += t.ell;
        te += (nr + nc) * t.ell;
      }
      out->tree_entries += te;
      entries += te;
    } else {
      entries += c * (c + 1) / 2;
    }
    if (comp && h.compressible[j]) {
      out->compressed++;
      out->rank_sum += q[j];
      out->sample_sum += h.comp[j].ell;
      if (q[j] == h.comp[j].ell && h.comp[j].ell < std::min(c, r)) out->rank_saturated++;
      entries += (c + r) * q[j];
    } else if (comp && h.opt.interior && h.iroot[j] >= 0 && r > 0) {
      entries += c * h.r_in[j];
      out->interior_dropped += c * (r - h.r_in[j]);
    } else {
      entries += c * r;
    }
    if (comp && h.opt.interior && h.iroot[j] == j && r > 0) out->interior_blocks++;
  }
  for (const rsc::Pair& pr : S.pairs) {
    const double m = (comp && h.compressible[pr.k]) ? q[pr.k] : S.c(pr.k);
    fl_update += 2.0 * m * ((double)pr.nD * (pr.nD + 1) / 2.0 + (double)(pr.nrows - pr.nD) * pr.nD);
  }
  out->factor_entries = entries;
  if (h.fplan) {
    out->flops_potrf = h.fplan->flops[0];
    out->flops_trsm = h.fplan->flops[1];
    out->flops_sample = h.fplan->flops[3];
    out->flops_orth = h.fplan->flops[4];
    out->flops_trunc = h.fplan->flops[5];
    if (comp)   // the kept basis U Z_q, V Z_q at the ranks
      for (int64_t j = 0; j < S.M(); ++j)
        if (h.compressible[j]) out->flops_trunc += 2.0 * (S.c(j) + S.r(j)) * (double)h.comp[j].ell * q[j];
  }
  out->flops_update = fl_update + (h.fplan ? h.fplan->flops[2] : 0.0);
  out->alpha_D_used = tree ? h.fplan->alpha_D : 0.0;
  out->diag_restarts = h.diag_restarts;
  out->bytes_factor = h.splan ? h.splan->bytes * (h.f32_valid ? 0.5 : 1.0) : 0.0;
  return RSC_OK;
}

rsc_status rsc_profile_enable(rsc_handle H, int32_t on) {
  if (!H) return fail(RSC_ERR_INVALID_ARG, "null handle");
  H->h.profiling = on != 0;
  std::memset(&H->h.prof, 0, sizeof(H->h.prof));
  for (int k = 0; k < RSC_KERNELS; ++k) {
    H->h.kprof_launches[k] = 0;
    H->h.kprof_ms[k] = 0.0;
    H->h.kprof_flops[k] = 0.0;
    H->h.kprof_tile_flops[k] = 0.0;
  }
  return RSC_OK;
}

rsc_status rsc_get_kernel_profile(rsc_handle H, int32_t k, const char** name, int64_t* launches,
                                  double* ms, double* flops, double* tile_flops) {
  if (!H) return fail(RSC_ERR_INVALID_ARG, "null handle");
  if (k < 0 || k >= RSC_KERNELS) return fail(RSC_ERR_INVALID_ARG, "kernel index out of range");
  if (name) *name = rsc::kernel_name(k);
  if (launches) *launches = H->h.kprof_launches[k];
  if (ms) *ms = H->h.kprof_ms[k];
  if (flops) *flops = H->h.kprof_flops[k];
  if (tile_flops) *tile_flops = H->h.kprof_tile_flops[k];
  return RSC_OK;
}

rsc_status rsc_get_profile(rsc_handle H, rsc_profile* out) {
  if (!H || !out) return fail(RSC_ERR_INVALID_ARG, "null argument");
  *out = H->h.prof;
  return RSC_OK;
}

const char* rsc_status_string(rsc_status s) {
  switch (s) {
    case RSC_OK: return "RSC_OK";
    case RSC_ERR_INVALID_ARG: return "RSC_ERR_INVALID_ARG";
    case RSC_ERR_PATTERN: return "RSC_ERR_PATTERN";
    case RSC_ERR_NOT_SPD: return "RSC_ERR_NOT_SPD";
    case RSC_ERR_NOT_CONVERGED: return "RSC_ERR_NOT_CONVERGED";
    case RSC_ERR_BREAKDOWN: return "RSC_ERR_BREAKDOWN";
    case RSC_ERR_OUT_OF_MEMORY: return "RSC_ERR_OUT_OF_MEMORY";
    case RSC_ERR_DEVICE: return "RSC_ERR_DEVICE";
    case RSC_ERR_STATE: return "RSC_ERR_STATE";
  }
  return "RSC_ERR_UNKNOWN";
}

const char* rsc_last_error(void) { return g_last_error.c_str(); }

rsc_status rsc_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                             void (*release)(void* ptr, void* stream, void* ctx), void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(RSC_ERR_INVALID_ARG, "allocator and release must be given together");
  if (!rsc::set_allocator(alloc, release, ctx))
    return fail(RSC_ERR_STATE, "the allocator can only change while no handle exists");
  return RSC_OK;
}

void rsc_destroy(rsc_handle H) {
  if (!H) return;
  rsc::release_device(H->h);
  delete H;
}

}  // extern "C"
