"""Seeded synthetic SDP instances in the primal-dual standard form (P)/(D).

    (P)  min A_0 . X   s.t.  A_k . X = b_k (k = 1..m),  X psd
    (D)  max sum_k b_k z_k  s.t.  sum_k A_k z_k + Y = A_0,  Y psd

This module only builds input data (graphs, weights, data matrices, dense
random states).  It holds none of the solver's arithmetic, and both the
CPU oracle and the GPU library consume what it returns.

Instances are stored the way the C library receives them: for every matrix
A_k (k = 0..m) the lower-triangle triplets (row >= col, 0-based), packed
one matrix after the other and delimited by ``ptr`` (length m + 2).

Workload families (shapes follow the paper's experiments, Section 4):
  * max-cut relaxation (Goemans-Williamson form used in Section 4):
    A_0 = -(Diag(W e) - W)/4, A_k = e_k e_k^T, b_k = 1;
  * norm minimisation with an arrow-shaped aggregate pattern;
  * small graph families with known SDP values (cycles, complete graphs,
    bipartite grids) and the paper's lattice graph.
"""
from __future__ import annotations

import dataclasses
from typing import Iterable, List, Sequence, Tuple

import numpy as np

__all__ = [
    "Problem", "from_matrices", "maxcut", "cycle_graph", "complete_graph",
    "grid_graph", "lattice_graph", "random_graph", "chordal_band_graph",
    "maxcut_cycle_chords", "maxcut_band", "maxcut_adjoint_case", "normmin", "random_ktree_graph",
    "maxcut_ktree_batch", "random_pd_dense", "random_pd_on_pattern",
]


@dataclasses.dataclass
class Problem:
    """An SDP in standard form, matrices as packed lower-triangle triplets."""
    n: int
    m: int
    ptr: np.ndarray   # int64 [m + 2]; entries of A_k are ptr[k]:ptr[k+1]
    row: np.ndarray   # int32, row >= col
    col: np.ndarray   # int32
    val: np.ndarray   # float64
    b: np.ndarray     # float64 [m]
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    def triplets(self, k: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        s, e = int(self.ptr[k]), int(self.ptr[k + 1])
        return self.row[s:e], self.col[s:e], self.val[s:e]

    def dense(self, k: int) -> np.ndarray:
        """Dense symmetric A_k (small n only)."""
        r, c, v = self.triplets(k)
        a = np.zeros((self.n, self.n))
        np.add.at(a, (r, c), v)
        off = r != c
        np.add.at(a, (c[off], r[off]), v[off])
        return a


def from_matrices(n: int, mats: Sequence[Tuple[np.ndarray, np.ndarray, np.ndarray]],
                  b: Iterable[float], name: str = "", meta: dict | None = None) -> Problem:
    """Pack [(rows, cols, vals)] for A_0..A_m; entries above the diagonal are
    mirrored into the lower triangle."""
    ptr = [0]
    rows: List[np.ndarray] = []
    cols: List[np.ndarray] = []
    vals: List[np.ndarray] = []
    for r, c, v in mats:
        r = np.asarray(r, dtype=np.int64)
        c = np.asarray(c, dtype=np.int64)
        v = np.asarray(v, dtype=np.float64)
        lo = np.maximum(r, c)
        hi = np.minimum(r, c)
        rows.append(lo.astype(np.int32))
        cols.append(hi.astype(np.int32))
        vals.append(v)
        ptr.append(ptr[-1] + len(v))
    b = np.asarray(list(b), dtype=np.float64)
    m = len(mats) - 1
    assert b.shape == (m,)
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return Problem(n=n, m=m, ptr=np.asarray(ptr, dtype=np.int64),
                   row=cat(rows, np.int32), col=cat(cols, np.int32),
                   val=cat(vals, np.float64), b=b, name=name, meta=dict(meta or {}))


# --------------------------------------------------------------------------
# graphs: edge lists (i < j) in lexicographic order, weights drawn afterwards
# --------------------------------------------------------------------------

def _sorted_edges(edges) -> np.ndarray:
    e = {(min(i, j), max(i, j)) for i, j in edges if i != j}
    return np.asarray(sorted(e), dtype=np.int64).reshape(-1, 2)


def cycle_graph(n: int) -> np.ndarray:
    return _sorted_edges((i, (i + 1) % n) for i in range(n))


def complete_graph(n: int) -> np.ndarray:
    return _sorted_edges((i, j) for i in range(n) for j in range(i + 1, n))


def grid_graph(a: int, b: int) -> np.ndarray:
    """a x b grid (bipartite); vertex (i, j) -> i + a*j."""
    e = []
    for j in range(b):
        for i in range(a):
            v = i + a * j
            if i + 1 < a:
                e.append((v, v + 1))
            if j + 1 < b:
                e.append((v, v + a))
    return _sorted_edges(e)


def lattice_graph(p: int, q: int) -> np.ndarray:
    """The lattice graph of the paper's experiments (Section 4): vertices
    i + (j-1) p, horizontal edges inside each of the q rows of length p and
    vertical edges between consecutive rows.  Same as grid_graph(p, q)."""
    return grid_graph(p, q)


def random_graph(n: int, p: float, rng: np.random.Generator) -> np.ndarray:
    e = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return _sorted_edges(e)


def chordal_band_graph(n: int, w: int) -> np.ndarray:
    return _sorted_edges((i, j) for i in range(n) for j in range(i + 1, min(n, i + w + 1)))


def random_ktree_graph(n: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """Random k-tree: start from a (k+1)-clique; each new vertex picks a
    uniform existing (k+1)-clique, drops one uniform member and joins the
    remaining k."""
    k = min(k, n - 1)
    cliques = [list(range(k + 1))]
    edges = [(i, j) for i in range(k + 1) for j in range(i + 1, k + 1)]
    for v in range(k + 1, n):
        base = cliques[rng.integers(len(cliques))]
        drop = rng.integers(len(base))
        sep = [u for t, u in enumerate(base) if t != drop]
        edges += [(u, v) for u in sep]
        cliques.append(sep + [v])
    return _sorted_edges(edges)


# --------------------------------------------------------------------------
# max-cut relaxation: min A_0.X s.t. X_kk = 1, A_0 = -(Diag(W e) - W)/4
# --------------------------------------------------------------------------

def maxcut(n: int, edges: np.ndarray, w: np.ndarray, name: str = "maxcut",
           meta: dict | None = None) -> Problem:
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.asarray(w, dtype=np.float64)
    deg = np.zeros(n)
    np.add.at(deg, edges[:, 0], w)
    np.add.at(deg, edges[:, 1], w)
    r0 = np.concatenate([np.arange(n), edges[:, 1]])
    c0 = np.concatenate([np.arange(n), edges[:, 0]])
    v0 = np.concatenate([-deg / 4.0, w / 4.0])
    keep = v0 != 0.0
    mats = [(r0[keep], c0[keep], v0[keep])]
    for k in range(n):
        mats.append((np.array([k]), np.array([k]), np.array([1.0])))
    md = {"edges": edges, "weights": w, "family": "maxcut"}
    md.update(meta or {})
    return from_matrices(n, mats, np.ones(n), name=name, meta=md)


def maxcut_cycle_chords(n: int = 64, seed: int = 0) -> Problem:
    """Cycle plus chords between vertices at cyclic distance d in {2,3,4},
    each chord present with probability 1/2; weights U[0,1]."""
    rng = np.random.default_rng(seed)
    e = [(i, (i + 1) % n) for i in range(n)]
    for i in range(n):
        for d in (2, 3, 4):
            if rng.random() < 0.5:
                e.append((i, (i + d) % n))
    edges = _sorted_edges(e)
    w = rng.uniform(0.0, 1.0, len(edges))
    return maxcut(n, edges, w, name=f"maxcut_cycle_chords_n{n}_s{seed}")


def maxcut_band(n: int = 4000, bw: int = 20, p: float = 0.5, seed: int = 0,
                wlo: float = 0.0, whi: float = 1.0) -> Problem:
    """Banded graph: each pair 1 <= j - i <= bw present with probability p
    (p = 1 keeps the whole band); weights U[wlo, whi]."""
    rng = np.random.default_rng(seed)
    ii, jj = [], []
    for i in range(n):
        hi = min(n, i + bw + 1)
        cand = np.arange(i + 1, hi)
        if p < 1.0:
            cand = cand[rng.random(len(cand)) < p]
        ii.append(np.full(len(cand), i))
        jj.append(cand)
    edges = np.stack([np.concatenate(ii), np.concatenate(jj)], axis=1).astype(np.int64)
    w = rng.uniform(wlo, whi, len(edges))
    return maxcut(n, edges, w, name=f"maxcut_band_n{n}_bw{bw}_s{seed}",
                  meta={"bandwidth": bw})


def maxcut_adjoint_case(n: int = 2000, bw: int = 16, seed: int = 0, nedges: int = 20):
    """Differentiation workload: the max-cut SDP over the full band of width bw
    (every pair 1 <= j - i <= bw, weights U[0.5, 1.5]), a loss matrix G_L that is
    symmetric with N(0,1) entries on |i - j| <= bw (diagonal included; returned as
    lower triplets), and nedges edge indices sampled uniformly without
    replacement.  Returns (problem, (rows, cols, vals) of G_L, edge indices)."""
    prob = maxcut_band(n, bw, 1.0, seed, 0.5, 1.5)
    rng = np.random.default_rng(seed + 1)
    gr, gc = [], []
    for j in range(n):
        hi = min(n, j + bw + 1)
        gr.append(np.arange(j, hi))
        gc.append(np.full(hi - j, j))
    gr = np.concatenate(gr).astype(np.int32)
    gc = np.concatenate(gc).astype(np.int32)
    gv = rng.standard_normal(len(gr))
    sel = rng.choice(len(prob.meta["weights"]), size=min(nedges, len(prob.meta["weights"])), replace=False)
    return prob, (gr, gc, gv), np.sort(sel)


def maxcut_lattice(p: int = 400, q: int = 10, seed: int = 0, wlo: float = 0.0, whi: float = 1.0) -> Problem:
    """Max-cut over the p x q lattice graph of the paper's experiments (Section 4,
    the max-cut workloads MaxCut400 .. MaxCut1200 take q = 10), in the paper's
    vertex numbering; the paper states no weights, these are U[wlo, whi].  The
    lattice is bipartite, so the relaxation's optimum is minus the total weight."""
    rng = np.random.default_rng(seed)
    edges = lattice_graph(p, q)
    w = rng.uniform(wlo, whi, len(edges))
    return maxcut(p * q, edges, w, name=f"maxcut_lattice_p{p}_q{q}_s{seed}", meta={"p": p, "q": q})


def lattice_short_first_order(p: int, q: int) -> np.ndarray:
    """An elimination order of the p x q lattice (paper's numbering) that walks the
    short side first: vertex i + j p for j = 0..q-1, then i + 1, and so on.  In that
    order every edge joins vertices at most q apart, so the chordal extension is a
    band of width q with cliques of q + 1 vertices.  perm[k] = the vertex
    eliminated k-th."""
    return np.array([i + j * p for i in range(p) for j in range(q)], dtype=np.int32)


def maxcut_ktree_batch(count: int = 256, seed: int = 0, nlo: int = 50, nhi: int = 800,
                       klo: int = 3, khi: int = 12, drop: float = 0.3) -> List[Problem]:
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(rng.integers(nlo, nhi + 1))
        k = int(rng.integers(klo, khi + 1))
        e = random_ktree_graph(n, k, rng)
        e = e[rng.random(len(e)) >= drop]
        w = rng.uniform(0.0, 1.0, len(e))
        out.append(maxcut(n, e, w, name=f"ktree{t}_n{n}_k{k}"))
    return out


# --------------------------------------------------------------------------
# norm minimisation: min t s.t. [[t I_p, F(y)], [F(y)^T, t I_q]] psd
# --------------------------------------------------------------------------

def normmin(p: int = 2000, q: int = 10, ny: int = 63, seed: int = 0) -> Problem:
    """z = (t, y_1..y_ny); F_i ~ N(0,1)/sqrt(p) dense p x q, i = 0..ny.
    A_0 = [[0, F_0], [F_0^T, 0]], A_1 = -I (t), A_{1+i} = -[[0, F_i], [F_i^T, 0]],
    b = (-1, 0, ..., 0).  The p-block is numbered first, the q-block last."""
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((ny + 1, p, q)) / np.sqrt(p)
    n = p + q
    rr = (p + np.arange(q))[None, :].repeat(p, 0).ravel()   # rows in the q-block
    cc = np.arange(p)[:, None].repeat(q, 1).ravel()          # cols in the p-block
    mats = [(rr, cc, F[0].ravel())]
    mats.append((np.arange(n), np.arange(n), -np.ones(n)))
    for i in range(1, ny + 1):
        mats.append((rr, cc, -F[i].ravel()))
    b = np.zeros(ny + 1)
    b[0] = -1.0
    return from_matrices(n, mats, b, name=f"normmin_p{p}_q{q}_ny{ny}_s{seed}",
                         meta={"family": "normmin", "F": F, "p": p, "q": q})


def random_sparse_sdp(n: int, m: int, seed: int = 0, nnz_per: int = 3,
                      band: int | None = None) -> Problem:
    """Random sparse SDP with a strictly feasible primal (X = I) and dual
    (z0 random, Y0 diagonally dominant): A_k has nnz_per random symmetric
    off-diagonal entries plus one diagonal entry (kept within |i-j| <= band
    when band is given); b_k = A_k . I; A_0 = sum z0_k A_k + Y0."""
    rng = np.random.default_rng(seed)
    mats = []
    dense = []
    for _ in range(m):
        a = np.zeros((n, n))
        d = rng.integers(n)
        a[d, d] = rng.uniform(0.5, 1.5)
        for _ in range(nnz_per):
            i = int(rng.integers(n))
            j = int(rng.integers(n)) if band is None else int(
                np.clip(i + rng.integers(-band, band + 1), 0, n - 1))
            if i == j:
                continue
            v = rng.uniform(-1.0, 1.0)
            a[i, j] += v
            a[j, i] += v
        dense.append(a)
    z0 = rng.uniform(-1.0, 1.0, m)
    s = sum(z * a for z, a in zip(z0, dense))
    y0 = np.diag(np.abs(s).sum(1) + 1.0 + rng.uniform(0.0, 1.0, n))  # Y0 = A_0 - sum z0_k A_k
    a0 = s + y0
    for a in [a0] + dense:
        r, c = np.nonzero(np.tril(a))
        mats.append((r, c, a[r, c]))
    b = np.array([np.trace(a) for a in dense])
    return from_matrices(n, mats, b, name=f"random_sdp_n{n}_m{m}_s{seed}",
                         meta={"family": "random"})


# --------------------------------------------------------------------------
# random states for replaying one SCM evaluation
# --------------------------------------------------------------------------

def random_pd_dense(n: int, rng: np.random.Generator, cond: float = 10.0) -> np.ndarray:
    """Dense symmetric positive definite matrix with eigenvalues in [1, cond]."""
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.exp(rng.uniform(0.0, np.log(cond), n))
    return (q * ev) @ q.T


def random_pd_on_pattern(n: int, rows: np.ndarray, cols: np.ndarray,
                         rng: np.random.Generator, shift: float = 1.0) -> np.ndarray:
    """Dense symmetric matrix supported on the given lower-triangle pattern
    (plus the diagonal), made strictly diagonally dominant (hence PD)."""
    a = np.zeros((n, n))
    off = rows != cols
    v = rng.uniform(-1.0, 1.0, int(off.sum()))
    a[rows[off], cols[off]] = v
    a[cols[off], rows[off]] = v
    d = np.abs(a).sum(1) + shift + rng.uniform(0.0, 1.0, n)
    a[np.arange(n), np.arange(n)] = d
    return a
