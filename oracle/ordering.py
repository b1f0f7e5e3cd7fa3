"""Oracle: nested-dissection ordering and supernodal symbolic analysis (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this module; the product path never does.

What is computed
----------------
* A fill-reducing nested-dissection ordering (paper §2.2 and §3.1: separators
  are numbered after the subdomains they split).  The paper cites George's nested
  dissection and treats the matrix as a black box without mesh data, but gives
  no algorithm; this oracle takes the pattern-only level-structure dissection
  below, fully specified so that two independent implementations agree bit for
  bit:

  ``ND(S)``: if ``|S| <= leaf_max`` emit ``S`` (ascending) as one leaf
  supernode.  Otherwise split the subgraph induced on ``S`` into connected
  components and recurse on each in order of its smallest vertex.  For a
  connected ``S``: start from ``r = min(S)``, take its breadth-first level sets,
  pick ``x`` in the last level with the smallest (degree inside ``S``, vertex id);
  if ``x`` has a larger eccentricity than ``r`` then ``r = x`` and repeat, else
  keep ``r`` (a pseudo-peripheral vertex).  With the levels ``L_0..L_h`` from
  ``r``: if ``h < 2`` emit ``S`` as one leaf; else ``m`` is the smallest level
  with ``2 * |L_0 u .. u L_m| >= |S|``, clamped to ``[1, h-1]``; the separator
  is the part of ``L_m`` with a neighbour in ``L_{m+1}``; recurse on the lower
  part (``L_0..L_{m-1}`` plus the rest of ``L_m``), then on the upper part
  (``L_{m+1}..L_h``), then emit the separator (ascending) as one separator
  supernode.

* Supernodes (paper §2.1): every emitted set is one supernode ``C_j`` (a
  contiguous range of the new numbering).  The paper groups the non-separator
  columns "as CHOLMOD does"; here each leaf set is one supernode.  The
  off-diagonal row list ``R_j`` is the union pattern: the neighbours of ``C_j``
  numbered after ``C_j``, together with the ``R_k`` of its children, restricted
  to rows after ``C_j``.  The parent of ``j`` is the supernode holding
  ``min R_j``; ``level = 0`` for a supernode without children, else
  ``1 + max(child levels)``.

* Diagonal block trees (§4.1, ``oracle.diagonal``): with ``tau_D > 0`` a separator
  of more than ``tau_D`` columns gets the depth of its complete block tree and, when
  positions are given, its columns are reordered by the recursive coordinate split.
  Reordering inside a supernode leaves its pattern unchanged.

* Descendant pairs (paper §2.1, descendant set and the row lists ``R^D_{k->j}``,
  ``R^O_{k->j}``): for each ``k`` the rows of ``R_k`` fall into runs owned by
  ancestors ``j``; for each run, ``p0`` is its first position in ``R_k`` and
  ``nD`` its length; the rows after the run are all in ``R_j``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse import csgraph

LEAF = 0
SEPARATOR = 1


def check_pattern(n, rowptr, colind):
    """Reject what the method cannot take: the pattern must be a full symmetric
    CSR with sorted, duplicate-free rows and every diagonal entry present."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    if rowptr.shape != (n + 1,) or rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise ValueError("bad row pointer")
    if rowptr[-1] != colind.size or (colind.size and (colind.min() < 0 or colind.max() >= n)):
        raise ValueError("bad column index")
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    d = np.diff(colind)
    same_row = rows[1:] == rows[:-1]
    if np.any(d[same_row] <= 0):
        raise ValueError("unsorted or duplicate column index")
    if np.count_nonzero(rows == colind) != n:
        raise ValueError("missing diagonal entry")
    P = sp.csr_matrix((np.ones(colind.size), colind, rowptr), shape=(n, n))
    if (P != P.T).nnz:
        raise ValueError("pattern not symmetric")


def adjacency(n, rowptr, colind) -> sp.csr_matrix:
    """Off-diagonal pattern as a 0/1 CSR matrix."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    keep = rows != colind
    return sp.csr_matrix((np.ones(int(keep.sum()), dtype=np.int8), (rows[keep], colind[keep])),
                         shape=(n, n))


def _ranges(indptr, nodes):
    """Concatenated column-index positions of the given rows of a CSR."""
    starts = indptr[nodes]
    lens = indptr[nodes + 1] - starts
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    offs = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens)
    return offs + np.arange(total)


def bfs_levels(sub: sp.csr_matrix, root: int) -> np.ndarray:
    """Breadth-first distance from ``root`` of every vertex of a connected graph."""
    n = sub.shape[0]
    lev = np.full(n, -1, dtype=np.int64)
    lev[root] = 0
    frontier = np.array([root], dtype=np.int64)
    d = 0
    while frontier.size:
        nb = sub.indices[_ranges(sub.indptr, frontier)]
        nb = np.unique(nb[lev[nb] < 0])
        d += 1
        lev[nb] = d
        frontier = nb
    return lev


def pseudo_peripheral(sub: sp.csr_matrix):
    """Start at local vertex 0 (the smallest id); move to the minimum
    (degree, id) vertex of the last level while that raises the eccentricity."""
    deg = np.diff(sub.indptr)
    r = 0
    lev = bfs_levels(sub, r)
    ecc = int(lev.max())
    while True:
        last = np.nonzero(lev == ecc)[0]
        x = int(last[np.lexsort((last, deg[last]))[0]])
        levx = bfs_levels(sub, x)
        eccx = int(levx.max())
        if eccx > ecc:
            r, lev, ecc = x, levx, eccx
        else:
            return r, lev


def nested_dissection(n, rowptr, colind, leaf_max: int = 64):
    """Return (perm new->old, supernode first columns, supernode kinds)."""
    adj = adjacency(n, rowptr, colind)
    emits = []   # (vertex array, kind)

    def emit(S, kind):
        emits.append((S, kind))

    def nd(S):
        if S.size <= leaf_max:
            emit(S, LEAF)
            return
        sub = adj[S][:, S].tocsr()
        ncomp, labels = csgraph.connected_components(sub, directed=False)
        if ncomp > 1:
            _, first = np.unique(labels, return_index=True)
            for lab in labels[np.sort(first)]:
                nd(S[labels == lab])
            return
        _, lev = pseudo_peripheral(sub)
        h = int(lev.max())
        if h < 2:
            emit(S, LEAF)
            return
        cum = np.cumsum(np.bincount(lev, minlength=h + 1))
        m = int(np.nonzero(2 * cum >= S.size)[0][0])
        m = min(max(m, 1), h - 1)
        in_m = lev == m
        # part of L_m with a neighbour in L_{m+1}
        entry_rows = np.repeat(np.arange(S.size), np.diff(sub.indptr))
        hits = lev[sub.indices] == m + 1
        has_up = np.zeros(S.size, dtype=bool)
        has_up[entry_rows[hits]] = True
        sep = in_m & has_up
        lower = (lev < m) | (in_m & ~sep)
        upper = lev > m
        nd(S[lower])
        nd(S[upper])
        emit(S[sep], SEPARATOR)

    nd(np.arange(n, dtype=np.int64))
    perm = np.concatenate([e[0] for e in emits]) if emits else np.zeros(0, dtype=np.int64)
    sizes = np.array([e[0].size for e in emits], dtype=np.int64)
    first = np.concatenate(([0], np.cumsum(sizes)))
    kinds = np.array([e[1] for e in emits], dtype=np.int32)
    return perm.astype(np.int64), first, kinds


@dataclass
class Symbolic:
    n: int
    perm: np.ndarray        # new -> old
    iperm: np.ndarray       # old -> new
    first: np.ndarray       # M + 1 supernode column boundaries
    kind: np.ndarray        # LEAF / SEPARATOR
    rows: list              # R_j (sorted new indices), one array per supernode
    parent: np.ndarray
    level: np.ndarray
    owner: np.ndarray       # new index -> supernode
    pairs: list             # per target j: list of (k, p0, nD) in ascending k
    depth: np.ndarray = None   # per supernode: depth of its diagonal block tree (0: dense)

    @property
    def M(self):
        return self.first.size - 1

    def c(self, j):
        return int(self.first[j + 1] - self.first[j])

    def r(self, j):
        return int(self.rows[j].size)


def symbolic(n, rowptr, colind, leaf_max: int = 64, tau_D: int = 0, coords=None) -> Symbolic:
    """Ordering and symbolic analysis.  With ``tau_D > 0`` every separator of more than
    ``tau_D`` columns gets a diagonal block tree (§4.1); with ``coords`` (``n x 3``
    positions of the original indices) its columns are first reordered by the
    recursive coordinate split of that tree."""
    from .diagonal import coordinate_order, split_depth
    check_pattern(n, rowptr, colind)
    perm, first, kind = nested_dissection(n, rowptr, colind, leaf_max)
    depth = np.zeros(first.size - 1, dtype=np.int64)
    for j in range(first.size - 1):
        lo, hi = int(first[j]), int(first[j + 1])
        if kind[j] == SEPARATOR and tau_D > 0 and hi - lo > tau_D:
            depth[j] = split_depth(hi - lo, tau_D)
            if coords is not None:
                xyz = np.asarray(coords, dtype=np.float64)[perm[lo:hi]]
                perm[lo:hi] = perm[lo:hi][coordinate_order(xyz, int(depth[j]))]
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    M = first.size - 1
    owner = np.repeat(np.arange(M), np.diff(first))
    adj = adjacency(n, rowptr, colind)
    # adjacency in the new numbering
    adjn = adj[perm][:, perm].tocsr()
    rows = [None] * M
    parent = np.full(M, -1, dtype=np.int64)
    children = [[] for _ in range(M)]
    for j in range(M):
        lo, hi = int(first[j]), int(first[j + 1])
        cand = [adjn.indices[adjn.indptr[lo]:adjn.indptr[hi]]]
        cand += [rows[k] for k in children[j]]
        u = np.unique(np.concatenate(cand)) if cand else np.zeros(0, dtype=np.int64)
        rows[j] = u[u >= hi].astype(np.int64)
        if rows[j].size:
            parent[j] = owner[rows[j][0]]
            children[parent[j]].append(j)
    level = np.zeros(M, dtype=np.int64)
    for j in range(M):
        if children[j]:
            level[j] = 1 + max(level[k] for k in children[j])
    pairs = [[] for _ in range(M)]
    for k in range(M):
        Rk = rows[k]
        if Rk.size == 0:
            continue
        own = owner[Rk]
        starts = np.concatenate(([0], np.nonzero(np.diff(own))[0] + 1))
        ends = np.concatenate((starts[1:], [Rk.size]))
        for s, e in zip(starts, ends):
            pairs[int(own[s])].append((k, int(s), int(e - s)))
    return Symbolic(n=n, perm=perm, iperm=iperm, first=first, kind=kind, rows=rows,
                    parent=parent, level=level, owner=owner, pairs=pairs, depth=depth)


def scatter_rows(B, R1, R2):
    """``scatterRows`` of paper §2.1: place the rows of ``B`` (indexed by the
    ordered list ``R1``) at the positions of ``R1``'s entries within ``R2``."""
    R1 = np.asarray(R1); R2 = np.asarray(R2)
    pos = np.searchsorted(R2, R1)
    if np.any(pos >= R2.size) or np.any(R2[np.minimum(pos, R2.size - 1)] != R1):
        raise ValueError("R1 must be a subset of R2")
    out = np.zeros((R2.size,) + np.asarray(B).shape[1:], dtype=np.asarray(B).dtype)
    out[pos] = B
    return out


def gather_rows(C, R2, R1):
    """``gatherRows`` of paper §2.1: the inverse of ``scatter_rows``."""
    pos = np.searchsorted(np.asarray(R2), np.asarray(R1))
    return np.asarray(C)[pos]
