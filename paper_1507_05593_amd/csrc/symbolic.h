// Host-side symbolic analysis: nested-dissection ordering, supernodes, row sets,
// elimination tree, levels and descendant pairs (paper Sec. 2.1, 2.2, 3.1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace rsc {

enum SupernodeKind : int32_t { kLeaf = 0, kSeparator = 1 };

// A descendant k of target j (Sec. 2.1): the rows R_k[p0 : p0+nD) lie in C_j
// (the list R^D_{k->j}), and every later row of R_k lies in R_j (R^O_{k->j}).
struct Pair {
  int32_t k, j;
  int32_t p0, nD;
  int32_t nrows;    // r_k - p0: rows of the gathered operand X = L^O_k[p0:, :]
  int64_t map_off;  // offset of this pair's relative map (nrows entries)
};

struct Symbolic {
  int64_t n = 0, nnz = 0;
  int32_t systems = 1;
  std::vector<int64_t> sys_first;    // systems+1 boundaries in the original numbering

  std::vector<int64_t> perm, iperm;  // new -> old, old -> new
  std::vector<int64_t> first;        // M+1 supernode column boundaries
  std::vector<int32_t> kind, parent, level;
  std::vector<int64_t> rows_ptr;     // M+1
  std::vector<int64_t> rows;         // R_j concatenated (new indices, ascending)
  std::vector<int32_t> owner;        // new index -> supernode
  std::vector<int32_t> sys_of_sn;    // supernode -> system
  std::vector<int32_t> depth;        // depth of the diagonal block tree (Sec. 4.1), 0: dense
  int32_t nlevels = 0;
  std::vector<std::vector<int32_t>> by_level;

  // descendant pairs grouped by target j (ascending k inside a target)
  std::vector<int64_t> pair_ptr;     // M+1
  std::vector<Pair> pairs;
  // local panel row (in [0, c_j + r_j)) of every gathered row of every pair
  std::vector<int32_t> relmap;

  int64_t M() const { return (int64_t)first.size() - 1; }
  int32_t c(int64_t j) const { return (int32_t)(first[j + 1] - first[j]); }
  int32_t r(int64_t j) const { return (int32_t)(rows_ptr[j + 1] - rows_ptr[j]); }
};

// Validates a full symmetric CSR pattern; returns an empty string or a message.
std::string check_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind);

// Level-structure nested dissection on the off-diagonal pattern.  Emits the
// permutation (new -> old) and one supernode per emitted set.
void nested_dissection(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t leaf_max,
                       std::vector<int64_t>& perm, std::vector<int64_t>& first,
                       std::vector<int32_t>& kind);

// Depth d of the complete block tree over c columns: the smallest d with
// ceil(c / 2^d) <= tau_D (0 when tau_D <= 0 or c <= tau_D).
int32_t split_depth(int64_t c, int32_t tau_D);

// Reorders idx (positions into xyz, n x 3 row-major) by d rounds of the coordinate
// split of Sec. 4.1: each piece is sorted stably along the longest side of its bounding
// box (the first of equal sides) and cut into its first m / 2 entries and the rest.
void coordinate_order(const double* xyz, std::vector<int64_t>& idx, int32_t d);

// Full symbolic analysis.  With tau_D > 0 every separator of more than tau_D columns
// gets a block tree of depth split_depth(c, tau_D); with coords (n x 3, original
// numbering, row-major) its columns are reordered by coordinate_order first.
void build_symbolic(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t leaf_max,
                    int32_t tau_D, const double* coords, Symbolic& S);

}  // namespace rsc
