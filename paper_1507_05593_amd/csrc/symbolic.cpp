// Host symbolic analysis (paper Sec. 2.1, 2.2, 3.1).
//
// Ordering: level-structure nested dissection on the pattern alone (the paper asks
// for nested dissection on a matrix with no mesh data and gives no algorithm):
//   ND(S): |S| <= leaf_max -> emit S as a leaf supernode.  Otherwise split G[S] into
//   connected components, recursing in order of their smallest vertex.  For a
//   connected S: pseudo-peripheral root (start at min S; move to the minimum
//   (degree in G[S], id) vertex of the last breadth-first level while that raises
//   the eccentricity); levels L_0..L_h; h < 2 -> leaf; m = first level with
//   2|L_0..L_m| >= |S|, clamped to [1, h-1]; separator = vertices of L_m adjacent to
//   L_{m+1}; recurse on the lower part, then the upper part, then emit the separator.
// Supernodes: one per emitted set.  Row sets are the union pattern (neighbours of
// C_j after C_j plus the children's row sets), parent = owner of min R_j.
// Large separators (Sec. 4.1): more than tau_D columns -> a complete block tree of
// depth ceil(log2(c / tau_D)); given positions, the columns are first reordered by the
// recursive split along the longest side of each piece's bounding box (stable sort,
// first of equal sides, first half m / 2), which leaves the supernode's pattern as is.
#include "symbolic.h"

#include <algorithm>
#include <functional>
#include <numeric>
#include <stdexcept>

namespace rsc {

std::string check_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind) {
  if (n < 0) return "negative order";
  if (rowptr[0] != 0) return "rowptr[0] != 0";
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return "rowptr not monotone";
    bool diag = false;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int32_t c = colind[p];
      if (c < 0 || c >= n) return "column index out of range";
      if (p > rowptr[i] && colind[p - 1] >= c) return "unsorted or duplicate column index";
      if (c == i) diag = true;
    }
    if (!diag) return "missing diagonal entry in row " + std::to_string(i);
  }
  // symmetry: every (i, c) has (c, i)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int32_t c = colind[p];
      const int32_t* b = colind + rowptr[c];
      const int32_t* e = colind + rowptr[c + 1];
      if (!std::binary_search(b, e, (int32_t)i)) return "pattern not symmetric";
    }
  }
  return "";
}

namespace {

struct LocalGraph {
  std::vector<int64_t> ptr;
  std::vector<int32_t> adj;
  int32_t size() const { return (int32_t)ptr.size() - 1; }
};

class Dissector {
 public:
  Dissector(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t leaf_max)
      : n_(n), rowptr_(rowptr), colind_(colind), leaf_max_(leaf_max), pos_(n, -1) {}

  void run(std::vector<int64_t>& perm, std::vector<int64_t>& first, std::vector<int32_t>& kind) {
    std::vector<int32_t> all(n_);
    std::iota(all.begin(), all.end(), 0);
    if (n_ > 0) nd(all);
    perm.clear(); first.assign(1, 0); kind.clear();
    for (auto& e : emits_) {
      for (int32_t v : e.first) perm.push_back(v);
      first.push_back((int64_t)perm.size());
      kind.push_back(e.second);
    }
  }

 private:
  int64_t n_;
  const int64_t* rowptr_;
  const int32_t* colind_;
  int32_t leaf_max_;
  std::vector<int32_t> pos_;   // global -> local index of the current subgraph, -1 outside
  std::vector<std::pair<std::vector<int32_t>, int32_t>> emits_;

  void emit(std::vector<int32_t>&& S, int32_t k) { emits_.emplace_back(std::move(S), k); }

  // Induced subgraph on the ascending vertex list S (self loops dropped).
  LocalGraph induce(const std::vector<int32_t>& S) {
    const int32_t m = (int32_t)S.size();
    for (int32_t i = 0; i < m; ++i) pos_[S[i]] = i;
    LocalGraph g;
    g.ptr.assign(m + 1, 0);
    for (int32_t i = 0; i < m; ++i) {
      int32_t v = S[i];
      for (int64_t p = rowptr_[v]; p < rowptr_[v + 1]; ++p) {
        int32_t u = colind_[p];
        if (u != v && pos_[u] >= 0) g.adj.push_back(pos_[u]);
      }
      g.ptr[i + 1] = (int64_t)g.adj.size();
    }
    for (int32_t i = 0; i < m; ++i) pos_[S[i]] = -1;
    return g;
  }

  // Breadth-first distances from root; returns the eccentricity.
  static int32_t bfs(const LocalGraph& g, int32_t root, std::vector<int32_t>& lev) {
    const int32_t m = g.size();
    lev.assign(m, -1);
    std::vector<int32_t> queue;
    queue.reserve(m);
    lev[root] = 0;
    queue.push_back(root);
    int32_t ecc = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
      int32_t v = queue[h];
      for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; ++p) {
        int32_t u = g.adj[p];
        if (lev[u] < 0) {
          lev[u] = lev[v] + 1;
          ecc = std::max(ecc, lev[u]);
          queue.push_back(u);
        }
      }
    }
    return ecc;
  }

  void nd(const std::vector<int32_t>& S) {
    const int32_t m = (int32_t)S.size();
    if (m <= leaf_max_) {
      emit(std::vector<int32_t>(S), kLeaf);
      return;
    }
    LocalGraph g = induce(S);
    // connected components, ordered by their smallest (local == global order) vertex
    std::vector<int32_t> comp(m, -1);
    int32_t ncomp = 0;
    {
      std::vector<int32_t> stack;
      for (int32_t s = 0; s < m; ++s) {
        if (comp[s] >= 0) continue;
        comp[s] = ncomp;
        stack.push_back(s);
        while (!stack.empty()) {
          int32_t v = stack.back();
          stack.pop_back();
          for (int64_t p = g.ptr[v]; p < g.ptr[v + 1]; ++p) {
            int32_t u = g.adj[p];
            if (comp[u] < 0) { comp[u] = ncomp; stack.push_back(u); }
          }
        }
        ++ncomp;
      }
    }
    if (ncomp > 1) {
      std::vector<std::vector<int32_t>> parts(ncomp);
      for (int32_t i = 0; i < m; ++i) parts[comp[i]].push_back(S[i]);
      g = LocalGraph();
      for (auto& P : parts) nd(P);
      return;
    }
    // pseudo-peripheral root from the smallest vertex
    std::vector<int32_t> lev, levx;
    int32_t r = 0;
    int32_t ecc = bfs(g, r, lev);
    for (;;) {
      int32_t x = -1;
      int64_t bestdeg = 0;
      for (int32_t i = 0; i < m; ++i) {
        if (lev[i] != ecc) continue;
        int64_t d = g.ptr[i + 1] - g.ptr[i];
        if (x < 0 || d < bestdeg) { x = i; bestdeg = d; }   // ascending i breaks ties by id
      }
      int32_t eccx = bfs(g, x, levx);
      if (eccx > ecc) { r = x; ecc = eccx; lev.swap(levx); } else break;
    }
    const int32_t h = ecc;
    if (h < 2) {
      emit(std::vector<int32_t>(S), kLeaf);
      return;
    }
    std::vector<int64_t> cnt(h + 1, 0);
    for (int32_t i = 0; i < m; ++i) cnt[lev[i]]++;
    int32_t lm = 0;
    int64_t cum = 0;
    for (int32_t t = 0; t <= h; ++t) {
      cum += cnt[t];
      if (2 * cum >= m) { lm = t; break; }
    }
    lm = std::min(std::max(lm, 1), h - 1);
    std::vector<int32_t> lower, upper, sep;
    for (int32_t i = 0; i < m; ++i) {
      if (lev[i] < lm) lower.push_back(S[i]);
      else if (lev[i] > lm) upper.push_back(S[i]);
      else {
        bool up = false;
        for (int64_t p = g.ptr[i]; p < g.ptr[i + 1]; ++p)
          if (lev[g.adj[p]] == lm + 1) { up = true; break; }
        (up ? sep : lower).push_back(S[i]);
      }
    }
    g = LocalGraph();
    lev.clear(); levx.clear();
    nd(lower);
    nd(upper);
    emit(std::move(sep), kSeparator);
  }
};

}  // namespace

void nested_dissection(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t leaf_max,
                       std::vector<int64_t>& perm, std::vector<int64_t>& first,
                       std::vector<int32_t>& kind) {
  Dissector d(n, rowptr, colind, leaf_max);
  d.run(perm, first, kind);
}

int32_t split_depth(int64_t c, int32_t tau_D) {
  if (tau_D <= 0) return 0;
  int32_t d = 0;
  while (((c + (int64_t(1) << d) - 1) >> d) > tau_D) ++d;
  return d;
}

void coordinate_order(const double* xyz, std::vector<int64_t>& idx, int32_t d) {
  std::function<void(int64_t, int64_t, int32_t)> rec = [&](int64_t lo, int64_t hi, int32_t depth) {
    if (depth == 0 || hi - lo < 2) return;
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) { mn[a] = xyz[3 * idx[lo] + a]; mx[a] = mn[a]; }
    for (int64_t i = lo; i < hi; ++i)
      for (int a = 0; a < 3; ++a) {
        const double v = xyz[3 * idx[i] + a];
        mn[a] = std::min(mn[a], v);
        mx[a] = std::max(mx[a], v);
      }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (mx[a] - mn[a] > mx[axis] - mn[axis]) axis = a;
    std::stable_sort(idx.begin() + lo, idx.begin() + hi,
                     [&](int64_t u, int64_t v) { return xyz[3 * u + axis] < xyz[3 * v + axis]; });
    const int64_t h = (hi - lo) / 2;
    rec(lo, lo + h, depth - 1);
    rec(lo + h, hi, depth - 1);
  };
  rec(0, (int64_t)idx.size(), d);
}

void build_symbolic(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t leaf_max,
                    int32_t tau_D, const double* coords, Symbolic& S) {
  S.n = n;
  S.nnz = rowptr[n];
  nested_dissection(n, rowptr, colind, leaf_max, S.perm, S.first, S.kind);
  const int64_t M = S.M();
  S.depth.assign(M, 0);
  for (int64_t j = 0; j < M; ++j) {
    const int64_t c = S.first[j + 1] - S.first[j];
    if (S.kind[j] != kSeparator || tau_D <= 0 || c <= tau_D) continue;
    S.depth[j] = split_depth(c, tau_D);
    if (!coords) continue;
    std::vector<int64_t> pos(c), old(S.perm.begin() + S.first[j], S.perm.begin() + S.first[j + 1]);
    std::iota(pos.begin(), pos.end(), 0);
    std::vector<double> xyz(3 * c);
    for (int64_t i = 0; i < c; ++i)
      for (int a = 0; a < 3; ++a) xyz[3 * i + a] = coords[3 * old[i] + a];
    coordinate_order(xyz.data(), pos, S.depth[j]);
    for (int64_t i = 0; i < c; ++i) S.perm[S.first[j] + i] = old[pos[i]];
  }
  S.iperm.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) S.iperm[S.perm[i]] = i;
  S.owner.assign(n, 0);
  for (int64_t j = 0; j < M; ++j)
    for (int64_t i = S.first[j]; i < S.first[j + 1]; ++i) S.owner[i] = (int32_t)j;

  // union-pattern row sets, parents and children
  S.rows_ptr.assign(M + 1, 0);
  S.rows.clear();
  S.parent.assign(M, -1);
  std::vector<std::vector<int32_t>> children(M);
  std::vector<int64_t> marker(n, -1);
  std::vector<int64_t> list;
  for (int64_t j = 0; j < M; ++j) {
    const int64_t hi = S.first[j + 1];
    list.clear();
    for (int64_t v = S.first[j]; v < hi; ++v) {
      int64_t old = S.perm[v];
      for (int64_t p = rowptr[old]; p < rowptr[old + 1]; ++p) {
        int64_t u = S.iperm[colind[p]];
        if (u >= hi && marker[u] != j) { marker[u] = j; list.push_back(u); }
      }
    }
    for (int32_t k : children[j]) {
      for (int64_t p = S.rows_ptr[k]; p < S.rows_ptr[k + 1]; ++p) {
        int64_t u = S.rows[p];
        if (u >= hi && marker[u] != j) { marker[u] = j; list.push_back(u); }
      }
    }
    std::sort(list.begin(), list.end());
    S.rows.insert(S.rows.end(), list.begin(), list.end());
    S.rows_ptr[j + 1] = (int64_t)S.rows.size();
    if (!list.empty()) {
      S.parent[j] = S.owner[list[0]];
      children[S.parent[j]].push_back((int32_t)j);
    }
  }
  S.level.assign(M, 0);
  for (int64_t j = 0; j < M; ++j)
    for (int32_t k : children[j]) S.level[j] = std::max(S.level[j], S.level[k] + 1);
  S.nlevels = 0;
  for (int64_t j = 0; j < M; ++j) S.nlevels = std::max(S.nlevels, S.level[j] + 1);
  S.by_level.assign(S.nlevels, {});
  for (int64_t j = 0; j < M; ++j) S.by_level[S.level[j]].push_back((int32_t)j);

  // descendant pairs: split each R_k into runs owned by one ancestor
  std::vector<std::vector<Pair>> per_target(M);
  for (int64_t k = 0; k < M; ++k) {
    const int64_t b = S.rows_ptr[k], e = S.rows_ptr[k + 1];
    int64_t p = b;
    while (p < e) {
      int32_t j = S.owner[S.rows[p]];
      int64_t q = p;
      while (q < e && S.owner[S.rows[q]] == j) ++q;
      Pair pr;
      pr.k = (int32_t)k; pr.j = j;
      pr.p0 = (int32_t)(p - b); pr.nD = (int32_t)(q - p); pr.nrows = (int32_t)(e - p);
      pr.map_off = 0;
      per_target[j].push_back(pr);
      p = q;
    }
  }
  S.pair_ptr.assign(M + 1, 0);
  S.pairs.clear();
  S.relmap.clear();
  for (int64_t j = 0; j < M; ++j) {
    const int64_t lo = S.first[j], hi = S.first[j + 1];
    const int64_t* Rj = S.rows.data() + S.rows_ptr[j];
    const int64_t rj = S.rows_ptr[j + 1] - S.rows_ptr[j];
    for (Pair pr : per_target[j]) {
      pr.map_off = (int64_t)S.relmap.size();
      const int64_t* Rk = S.rows.data() + S.rows_ptr[pr.k];
      int64_t cursor = 0;
      for (int32_t t = 0; t < pr.nrows; ++t) {
        int64_t g = Rk[pr.p0 + t];
        if (g < hi) {
          S.relmap.push_back((int32_t)(g - lo));
        } else {
          // R_j is sorted and the tail of R_k is ascending: a forward cursor suffices
          while (cursor < rj && Rj[cursor] < g) ++cursor;
          if (cursor >= rj || Rj[cursor] != g)
            throw std::logic_error("descendant row missing from ancestor row set");
          S.relmap.push_back((int32_t)((hi - lo) + cursor));
        }
      }
      S.pairs.push_back(pr);
    }
    S.pair_ptr[j + 1] = (int64_t)S.pairs.size();
  }
  S.sys_of_sn.assign(M, 0);
}

}  // namespace rsc
