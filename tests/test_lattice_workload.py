"""The lattice max-cut workloads (the paper's MaxCut400 .. MaxCut1200 family,
Section 4): generator structure and the oracle against the closed form.

The lattice graph is bipartite, so the max-cut relaxation attains the total
edge weight (every edge cut): with the objective -(Diag(W e) - W) / 4 the
optimum is minus the total weight, exactly, at any size.
"""
import numpy as np
import pytest

import sdpgen
from oracle.pdipm import Params, dense_pdipm, mc_pdipm


@pytest.mark.parametrize("p,q", [(4, 3), (7, 10), (40, 10)])
def test_lattice_graph_structure(p, q):
    prob = sdpgen.maxcut_lattice(p, q, seed=2)
    e = prob.meta["edges"]
    assert prob.n == prob.m == p * q
    assert len(e) == (p - 1) * q + p * (q - 1)
    # the edges of the paper's definition: along a row (i, i + 1) and between rows (i, i + p)
    d = e[:, 1] - e[:, 0]
    assert set(np.unique(d)) <= {1, p}
    assert np.all((d != 1) | (e[:, 0] % p != p - 1))
    # bipartite: colour (i + j) of vertex i + j p
    col = (e % p + e // p) % 2
    assert np.all(col[:, 0] != col[:, 1])
    w = prob.meta["weights"]
    assert np.all((w >= 0.0) & (w <= 1.0))


@pytest.mark.parametrize("p,q", [(5, 3), (30, 10)])
def test_short_first_order_is_a_band_of_width_q(p, q):
    perm = sdpgen.lattice_short_first_order(p, q)
    assert np.array_equal(np.sort(perm), np.arange(p * q))
    pos = np.empty(p * q, np.int64)
    pos[perm] = np.arange(p * q)
    e = sdpgen.lattice_graph(p, q)
    assert np.abs(pos[e[:, 0]] - pos[e[:, 1]]).max() == q


@pytest.mark.parametrize("p,q,seed", [(6, 4, 0), (9, 5, 1)])
def test_oracle_reaches_minus_total_weight(p, q, seed):
    prob = sdpgen.maxcut_lattice(p, q, seed)
    total = prob.meta["weights"].sum()
    res = dense_pdipm(prob, Params(gap_tol=1e-9, feas_tol=1e-9))
    assert res["status"] == "optimal"
    assert abs((res["pobj"] + res["dobj"]) / 2 + total) <= 1e-8 * total


def test_mc_oracle_same_optimum_in_either_order():
    """The matrix-completion oracle in the natural order and in the short-side-first
    order: different chordal extensions, the same optimum (minus the total weight)."""
    p, q = 8, 4
    prob = sdpgen.maxcut_lattice(p, q, 3)
    total = prob.meta["weights"].sum()
    P = Params(gap_tol=1e-9, feas_tol=1e-9)
    for order in (None, sdpgen.lattice_short_first_order(p, q)):
        res = mc_pdipm(prob, P, order=order)
        assert res["status"] == "optimal"
        assert abs((res["pobj"] + res["dobj"]) / 2 + total) <= 1e-8 * total
