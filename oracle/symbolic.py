"""Oracle symbolic phase: aggregate pattern, chordal extension, cliques.

Section 2.1 of the paper: the aggregate sparsity pattern collects every
(i, j) where some A_k (k = 0..m) is nonzero; the rows/columns are permuted
by an ordering, the fill of the Cholesky factor Y = N N^T extends the
pattern to a chordal one, and E is the union of C_r x C_r over its cliques.
Section 3.1: the cliques are taken as the supernodes of the symbolic
factorization (row set C_r, column set S_r); with supernodes numbered by
their first column they satisfy the running intersection property, S_r is
made of the first |S_r| members of C_r (ascending) and U_r = C_r minus S_r.

Readings (the paper leaves these to CHOLMOD's heuristics):
  * the ordering is an input: natural, a caller-given permutation, or the
    exact minimum-degree rule below (ties go to the lowest index);
  * supernodes are the fundamental ones: column j+1 joins j's supernode
    iff it is j's parent in the elimination tree, j is its only child and
    struct(j) = {j} + struct(j+1).

Everything here works on Python sets and lists; it is meant for clarity,
not speed, and shares no code with the GPU library.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp


def sym_sparse(prob, k: int) -> sp.csr_matrix:
    """A_k as a full symmetric scipy CSR matrix (duplicates summed)."""
    r, c, v = prob.triplets(k)
    off = r != c
    rr = np.concatenate([r, c[off]])
    cc = np.concatenate([c, r[off]])
    vv = np.concatenate([v, v[off]])
    a = sp.coo_matrix((vv, (rr, cc)), shape=(prob.n, prob.n)).tocsr()
    a.sum_duplicates()
    return a


def aggregate_pattern(prob):
    """Lower-triangle (row >= col) positions of the aggregate pattern, the
    diagonal always included."""
    keys = set((i, i) for i in range(prob.n))
    for k in range(prob.m + 1):
        r, c, _ = prob.triplets(k)
        keys.update(zip(r.tolist(), c.tolist()))
    rc = np.array(sorted(keys), dtype=np.int64)
    return rc[:, 0], rc[:, 1]


def min_degree_order(n: int, rows, cols) -> np.ndarray:
    """Exact minimum-degree ordering by the elimination game: repeatedly
    eliminate a vertex of smallest current degree (lowest index on ties) and
    make its remaining neighbours a clique."""
    adj = [set() for _ in range(n)]
    for i, j in zip(rows, cols):
        if i != j:
            adj[i].add(j)
            adj[j].add(i)
    alive = set(range(n))
    order = []
    while alive:
        v = min(alive, key=lambda u: (len(adj[u]), u))
        nb = adj[v]
        for a in nb:
            adj[a].discard(v)
            adj[a].update(nb - {a})
        alive.discard(v)
        adj[v] = set()
        order.append(v)
    return np.asarray(order, dtype=np.int64)


@dataclasses.dataclass
class Chordal:
    n: int
    order: np.ndarray            # order[i] = original index placed at position i
    pos: np.ndarray              # pos[original] = position
    struct: List[np.ndarray]     # struct[j]: sorted rows >= j of column j (positions)
    parent: np.ndarray           # elimination-tree parent, -1 at a root
    first: np.ndarray            # supernode r owns columns first[r] .. first[r+1]-1
    cliques: List[np.ndarray]    # C_r = struct[first[r]] (ascending)
    nS: np.ndarray               # |S_r|

    @property
    def ell(self) -> int:
        return len(self.cliques)

    def E_lower(self):
        """(rows, cols) of the lower triangle of E, column by column."""
        rr = np.concatenate(self.struct)
        cc = np.concatenate([np.full(len(s), j) for j, s in enumerate(self.struct)])
        return rr, cc

    def E_mask(self) -> np.ndarray:
        m = np.zeros((self.n, self.n), dtype=bool)
        rr, cc = self.E_lower()
        m[rr, cc] = True
        m[cc, rr] = True
        return m

    def permute(self, a: np.ndarray) -> np.ndarray:
        """Dense matrix in original indices -> positions."""
        return a[np.ix_(self.order, self.order)]

    def unpermute(self, a: np.ndarray) -> np.ndarray:
        return a[np.ix_(self.pos, self.pos)]


def chordal_structure(n: int, rows, cols, order=None) -> Chordal:
    """Chordal extension of the pattern (rows, cols) for the given order by
    symbolic elimination, then the elimination tree and the supernodes."""
    order = np.arange(n) if order is None else np.asarray(order, dtype=np.int64)
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    higher = [set() for _ in range(n)]
    for i, j in zip(np.asarray(rows), np.asarray(cols)):
        a, b = int(pos[i]), int(pos[j])
        if a == b:
            continue
        lo, hi = min(a, b), max(a, b)
        higher[lo].add(hi)
    parent = np.full(n, -1, dtype=np.int64)
    struct = []
    for v in range(n):
        s = higher[v]
        if s:
            p = min(s)
            parent[v] = p
            higher[p].update(s - {p})
        struct.append(np.asarray(sorted({v} | s), dtype=np.int64))
    nchild = np.zeros(n, dtype=np.int64)
    for v in range(n):
        if parent[v] >= 0:
            nchild[parent[v]] += 1
    first = [0]
    for j in range(n - 1):
        same = (parent[j] == j + 1 and nchild[j + 1] == 1
                and len(struct[j]) == len(struct[j + 1]) + 1)
        if not same:
            first.append(j + 1)
    first.append(n)
    first = np.asarray(first, dtype=np.int64)
    cliques = [struct[first[r]] for r in range(len(first) - 1)]
    nS = np.diff(first)
    return Chordal(n=n, order=order, pos=pos, struct=struct, parent=parent,
                   first=first, cliques=cliques, nS=nS)
