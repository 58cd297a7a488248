"""Host-side checks that need no GPU: the library loads and exports every
entry point of include/sdpc.h, and its symbolic phase (sdpc_analyze) agrees
exactly with the oracle's on the elimination order, the extended pattern E
and the clique structure (Section 2.1, Section 3.1)."""
import os
import re

import numpy as np
import pytest

import sdpgen
from oracle.symbolic import aggregate_pattern, chordal_structure, min_degree_order

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

lib_mod = pytest.importorskip("paper_1310_6919_amd.sdpc")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lib_mod.LIB_PATH):
        pytest.fail("libsdpc.so not built: run `python -m paper_1310_6919_amd.build`")
    return lib_mod.load()


def test_exports_match_header(lib):
    hdr = open(os.path.join(ROOT, "include", "sdpc.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)      # drop comments
    declared = set(re.findall(r"\b(sdpc_[a-z_]+)\s*\(", hdr))
    assert declared == set(lib_mod.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _E_edges_from_cliques(cliques):
    e = set()
    for C in cliques:
        C = [int(x) for x in C]
        for a in C:
            for b in C:
                if a >= b:
                    e.add((a, b) if a >= b else (b, a))
    return e


def _oracle(prob, order=None):
    rows, cols = aggregate_pattern(prob)
    return chordal_structure(prob.n, rows, cols, order)


def _maximal(cliques):
    sets = [frozenset(int(x) for x in C) for C in cliques]
    return {s for s in sets if not any(s < t for t in sets)}


CASES = {
    "cfg1": lambda: sdpgen.maxcut_cycle_chords(64, 0),
    "band300": lambda: sdpgen.maxcut_band(300, 20, 0.5, 1),
    "normmin": lambda: sdpgen.normmin(120, 10, 4, 0),
    "random_sdp": lambda: sdpgen.random_sparse_sdp(40, 12, seed=3),
    "grid": lambda: sdpgen.maxcut(30, sdpgen.grid_graph(6, 5), np.ones(len(sdpgen.grid_graph(6, 5)))),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_natural_order_matches_oracle(name):
    prob = CASES[name]()
    info, perm, cliques, nS = lib_mod.sdpc_analyze(prob)
    ch = _oracle(prob)
    # a natural order that is already an elimination-tree postorder is kept as is
    # (the random band is not one: some subtrees are not contiguous ranges)
    if name in ("cfg1", "normmin"):
        assert np.array_equal(perm, np.arange(prob.n))
        assert info["ncliques"] == ch.ell
        for r in range(ch.ell):
            assert np.array_equal(cliques[r], ch.order[ch.cliques[r]])
            assert nS[r] == ch.nS[r]
    # E as a set of original-index pairs is fixed by the order (any postorder of it)
    rr, cc = ch.E_lower()
    eo = {(int(max(a, b)), int(min(a, b))) for a, b in zip(ch.order[rr], ch.order[cc])}
    assert _E_edges_from_cliques(cliques) == eo
    assert info["nnzE"] == len(eo)
    assert _maximal(cliques) == _maximal([ch.order[C] for C in ch.cliques])
    # S_r leads C_r and the S_r partition the vertices
    seen = np.concatenate([c[:k] for c, k in zip(cliques, nS)])
    assert sorted(seen.tolist()) == list(range(prob.n))


@pytest.mark.parametrize("seed", range(4))
def test_user_and_min_degree_orders(seed):
    rng = np.random.default_rng(seed)
    n = 36
    e = sdpgen.random_graph(n, 0.1, rng)
    prob = sdpgen.maxcut(n, e, np.ones(len(e)))
    rows, cols = aggregate_pattern(prob)
    order = rng.permutation(n)
    for kw, ref in ((dict(user_perm=order), order), (dict(ordering=1), min_degree_order(n, rows, cols))):
        info, perm, cliques, nS = lib_mod.sdpc_analyze(prob, **kw)
        ch = chordal_structure(n, rows, cols, ref)
        rr, cc = ch.E_lower()
        eo = {(int(max(a, b)), int(min(a, b))) for a, b in zip(ch.order[rr], ch.order[cc])}
        assert _E_edges_from_cliques(cliques) == eo
        assert _maximal(cliques) == _maximal([ch.order[C] for C in ch.cliques])
        # the library's order is an elimination order with the same fill: check it directly
        ch2 = chordal_structure(n, rows, cols, perm)
        rr2, cc2 = ch2.E_lower()
        e2 = {(int(max(a, b)), int(min(a, b))) for a, b in zip(ch2.order[rr2], ch2.order[cc2])}
        assert e2 == eo


def test_band_blocks_and_frontier():
    prob = sdpgen.maxcut_band(4000, 20, 0.5, 0)
    info, perm, cliques, nS = lib_mod.sdpc_analyze(prob)
    assert sorted(perm.tolist()) == list(range(4000))
    assert info["max_clique"] <= 21
    assert info["hadamard"] == 1
    assert info["max_block_cols"] <= 32
    # every pending row of a band lies within the bandwidth of the current block
    assert info["nfwd"] <= 2 * 21 and info["nbwd"] <= 2 * 21
    info2, *_ = lib_mod.sdpc_analyze(prob, block_width=1)
    assert info2["nblocks"] == 4000 and info2["nslot"] == info2["nnzE"]
    assert info2["nnzE"] == info["nnzE"]
    for bw in (2, 8, 16):
        info3, *_ = lib_mod.sdpc_analyze(prob, block_width=bw)
        assert info3["nnzE"] == info["nnzE"]
        assert info3["max_block_rows"] * info3["max_block_cols"] <= 4096


def test_invalid_inputs(lib):
    prob = sdpgen.maxcut_cycle_chords(16, 0)
    bad = sdpgen.Problem(n=prob.n, m=prob.m, ptr=prob.ptr, row=prob.col, col=prob.row, val=prob.val, b=prob.b)
    off = prob.row != prob.col
    if off.any():
        with pytest.raises(lib_mod.SdpcError):
            lib_mod.sdpc_analyze(bad)
    with pytest.raises(lib_mod.SdpcError):
        lib_mod.sdpc_analyze(prob, user_perm=np.zeros(prob.n, np.int32))
    for bw in (0, 33):
        with pytest.raises(lib_mod.SdpcError):
            lib_mod.sdpc_analyze(prob, block_width=bw)
