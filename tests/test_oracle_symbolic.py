"""Pins for the oracle's symbolic phase (Section 2.1 chordal extension,
Section 3.1 supernodes as cliques): closed-form structures and the defining
properties (chordality, E contains the aggregate pattern, running
intersection, S_r leads C_r)."""
import itertools

import numpy as np
import pytest

import sdpgen
from oracle.symbolic import aggregate_pattern, chordal_structure, min_degree_order


def _check_invariants(ch, rows, cols):
    n = ch.n
    E = ch.E_mask()
    # E covers the aggregate pattern (in positions)
    assert E[ch.pos[rows], ch.pos[cols]].all()
    # perfect elimination: the higher neighbours of every vertex form a clique
    for j in range(n):
        s = ch.struct[j]
        assert s[0] == j
        assert E[np.ix_(s, s)].all()
    # fill closure: struct(j) minus {j, parent} lies in struct(parent)
    for j in range(n):
        p = ch.parent[j]
        if p >= 0:
            assert set(ch.struct[j][1:]) <= set(ch.struct[p])
    # cliques: S_r is the first |S_r| members, consecutive columns
    covered = np.zeros(n, dtype=int)
    for r, C in enumerate(ch.cliques):
        k = ch.nS[r]
        assert np.array_equal(C[:k], np.arange(ch.first[r], ch.first[r + 1]))
        covered[C[:k]] += 1
        # running intersection: U_r inside some later clique
        U = set(C[k:].tolist())
        later = set().union(*[set(c.tolist()) for c in ch.cliques[r + 1:]]) if r + 1 < ch.ell else set()
        assert U <= later
        if U:
            assert any(U <= set(c.tolist()) for c in ch.cliques[r + 1:])
        # S_r = C_r minus the later cliques
        assert not (set(C[:k].tolist()) & later)
    assert (covered == 1).all()
    # E is the union of the clique blocks
    E2 = np.zeros_like(E)
    for C in ch.cliques:
        E2[np.ix_(C, C)] = True
    assert np.array_equal(E, E2)


def test_band_natural_order_closed_form():
    n, w = 40, 5
    e = sdpgen.chordal_band_graph(n, w)
    p = sdpgen.maxcut(n, e, np.ones(len(e)))
    rows, cols = aggregate_pattern(p)
    ch = chordal_structure(n, rows, cols)
    for j in range(n):
        assert np.array_equal(ch.struct[j], np.arange(j, min(n, j + w + 1)))
    # cliques are the windows {j..j+w}, the last one holds the final w+1 columns
    assert ch.ell == n - w
    for r, C in enumerate(ch.cliques):
        assert len(C) == w + 1
    _check_invariants(ch, rows, cols)


def test_arrow_closed_form():
    pp, qq = 30, 4
    prob = sdpgen.normmin(p=pp, q=qq, ny=3, seed=1)
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    # p leaf cliques {r} + dense block, then the root supernode (the dense
    # block itself: a supernode, contained in every leaf clique)
    assert ch.ell == pp + 1
    dense = np.arange(pp, pp + qq)
    for r, C in enumerate(ch.cliques[:pp]):
        assert np.array_equal(C, np.concatenate([[r], dense]))
    assert np.array_equal(ch.cliques[pp], dense) and ch.nS[pp] == qq
    _check_invariants(ch, rows, cols)


def test_min_degree_puts_dense_rows_last():
    # arrow with the dense vertices numbered FIRST: min degree must move them last
    pp, qq = 25, 3
    prob = sdpgen.normmin(p=pp, q=qq, ny=2, seed=2)
    rows, cols = aggregate_pattern(prob)
    n = prob.n
    flip = np.concatenate([np.arange(pp, n), np.arange(pp)])   # dense block first
    inv = np.empty(n, dtype=np.int64)
    inv[flip] = np.arange(n)
    order = min_degree_order(n, inv[rows], inv[cols])
    # the leaves go before the dense block (up to a final degree tie)
    assert set(order[:pp - 1].tolist()) <= set(range(qq, n))
    ch = chordal_structure(n, inv[rows], inv[cols], order)
    assert max(len(C) for C in ch.cliques) == qq + 1
    # the only fill is the q x q block made a clique
    nnzE = sum(len(s) for s in ch.struct) - n
    assert nnzE == pp * qq + qq * (qq - 1) // 2


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_invariants(seed):
    rng = np.random.default_rng(seed)
    n = 30
    e = sdpgen.random_graph(n, 0.12, rng)
    p = sdpgen.maxcut(n, e, np.ones(len(e)))
    rows, cols = aggregate_pattern(p)
    for order in (None, rng.permutation(n), min_degree_order(n, rows, cols)):
        ch = chordal_structure(n, rows, cols, order)
        _check_invariants(ch, rows, cols)


def test_ktree_clique_bound():
    rng = np.random.default_rng(3)
    for k in (2, 3, 5):
        e = sdpgen.random_ktree_graph(40, k, rng)
        p = sdpgen.maxcut(40, e, np.ones(len(e)))
        rows, cols = aggregate_pattern(p)
        ch = chordal_structure(40, rows, cols, min_degree_order(40, rows, cols))
        # a k-tree is chordal: min degree finds a perfect order, no fill
        assert max(len(C) for C in ch.cliques) <= k + 1
        nnzE = sum(len(s) for s in ch.struct) - 40
        assert nnzE == len(e)


def test_fill_matches_bruteforce_elimination():
    # brute force: eliminate vertices on a dense boolean matrix
    rng = np.random.default_rng(7)
    n = 14
    e = sdpgen.random_graph(n, 0.25, rng)
    p = sdpgen.maxcut(n, e, np.ones(len(e)))
    rows, cols = aggregate_pattern(p)
    order = rng.permutation(n)
    ch = chordal_structure(n, rows, cols, order)
    pos = np.empty(n, dtype=int)
    pos[order] = np.arange(n)
    G = np.zeros((n, n), dtype=bool)
    G[pos[rows], pos[cols]] = True
    G |= G.T
    F = G.copy()
    for v in range(n):
        nb = [u for u in range(v + 1, n) if F[v, u]]
        for a, b in itertools.combinations(nb, 2):
            F[a, b] = F[b, a] = True
    F |= np.eye(n, dtype=bool)
    assert np.array_equal(F, ch.E_mask())
