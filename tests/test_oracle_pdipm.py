"""Pins for the oracle PDIPMs against values fixed by combinatorics and
closed forms, and against the termination invariants.

  * brute-force max-cut (n <= 12): maxcut <= SDP <= maxcut / 0.87856
    (Goemans-Williamson ratio);
  * bipartite graphs (even cycles, grids, the paper's lattice): SDP = total
    weight, since every term (1 - X_ij)/2 <= 1;
  * unit-weight cycle C_n: SDP = (n/2)(1 - cos(2 pi floor(n/2)/n)); the dual
    is uniform, z_i = -lambda_max(L)/4;
  * K_n (unit weights): SDP = n^2 / 4;
  * norm minimisation: t* = sigma_max(F_0 + sum y_i* F_i), and
    t* = sigma_max(F_0) without y variables;
  * invariances: a vertex relabelling leaves the value unchanged and permutes
    z; scaling the weights by s scales value and z by s;
  * at termination: gap and infeasibilities below tolerance, X and Y psd,
    diag X = 1 for max-cut;
  * the matrix-completion variant reaches the same optimum, and its step
    lengths sit on the boundary of the psd cone.
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle.pdipm import Params, dense_pdipm, mc_pdipm, step_length_cliques, step_length_dense

TIGHT = Params(gap_tol=1e-9, feas_tol=1e-9)


def _value(res):
    return -(res["pobj"] + res["dobj"]) / 2.0


@pytest.mark.parametrize("seed", range(4))
def test_bruteforce_maxcut_bounds(seed):
    rng = np.random.default_rng(seed)
    n = 9 + seed
    e = sdpgen.random_graph(n, 0.4, rng)
    w = rng.uniform(0, 1, len(e))
    prob = sdpgen.maxcut(n, e, w)
    res = dense_pdipm(prob, TIGHT)
    assert res["status"] == "optimal"
    mc = oracle.brute_force_maxcut(n, e, w)
    sdp = _value(res)
    assert mc <= sdp * (1 + 1e-9)
    assert sdp <= mc / 0.87856 * (1 + 1e-9)


@pytest.mark.parametrize("kind", ["cycle8", "grid3x4", "lattice5x3"])
def test_bipartite_equals_total_weight(kind):
    rng = np.random.default_rng(1)
    if kind == "cycle8":
        e = sdpgen.cycle_graph(8)
    elif kind == "grid3x4":
        e = sdpgen.grid_graph(3, 4)
    else:
        e = sdpgen.lattice_graph(5, 3)
    n = int(e.max()) + 1
    w = rng.uniform(0.1, 1, len(e))
    res = dense_pdipm(sdpgen.maxcut(n, e, w), TIGHT)
    assert abs(_value(res) - w.sum()) <= 1e-8 * w.sum()


@pytest.mark.parametrize("n", [3, 4, 5, 7, 9, 12])
def test_cycle_closed_form(n):
    e = sdpgen.cycle_graph(n)
    res = dense_pdipm(sdpgen.maxcut(n, e, np.ones(len(e))), TIGHT)
    val = oracle.cycle_sdp_value(n)
    assert abs(_value(res) - val) <= 1e-8 * val
    lmax = 2.0 - 2.0 * np.cos(2 * np.pi * (n // 2) / n)
    assert np.allclose(res["z"], -lmax / 4.0, atol=1e-6)


def test_complete_graph():
    n = 7
    e = sdpgen.complete_graph(n)
    res = dense_pdipm(sdpgen.maxcut(n, e, np.ones(len(e))), TIGHT)
    assert abs(_value(res) - n * n / 4.0) <= 1e-8 * n * n


def test_normmin_sigma_max():
    prob = sdpgen.normmin(p=40, q=5, ny=6, seed=3)
    res = dense_pdipm(prob, TIGHT)
    F = prob.meta["F"]
    t, y = res["z"][0], res["z"][1:]
    Fy = F[0] + np.einsum("i,ijk->jk", y, F[1:])
    smax = np.linalg.svd(Fy, compute_uv=False)[0]
    assert abs(t - smax) <= 1e-7 * smax
    assert abs(res["pobj"] + t) <= 1e-7 * t
    p0 = sdpgen.normmin(p=40, q=5, ny=0, seed=3)
    r0 = dense_pdipm(p0, TIGHT)
    s0 = np.linalg.svd(p0.meta["F"][0], compute_uv=False)[0]
    assert abs(r0["z"][0] - s0) <= 1e-7 * s0


def test_invariances():
    prob = sdpgen.maxcut_cycle_chords(16, 2)
    e, w = prob.meta["edges"], prob.meta["weights"]
    res = dense_pdipm(prob, TIGHT)
    perm = np.random.default_rng(0).permutation(16)
    pe = perm[e]
    rp = dense_pdipm(sdpgen.maxcut(16, pe, w), TIGHT)
    assert abs(_value(rp) - _value(res)) <= 1e-8 * abs(_value(res))
    assert np.allclose(rp["z"][perm], res["z"], atol=1e-6)
    rs = dense_pdipm(sdpgen.maxcut(16, e, 3.0 * w), TIGHT)
    assert abs(_value(rs) - 3 * _value(res)) <= 1e-8 * abs(_value(rs))
    assert np.allclose(rs["z"], 3 * res["z"], atol=3e-6)


def test_termination_invariants_and_mc_agreement():
    prob = sdpgen.maxcut_cycle_chords(32, 4)
    P = Params()
    rd = dense_pdipm(prob, P)
    rm = mc_pdipm(prob, P)
    for r in (rd, rm):
        assert r["status"] == "optimal"
        assert r["relgap"] <= P.gap_tol and r["pinf"] <= P.feas_tol and r["dinf"] <= P.feas_tol
        assert np.linalg.eigvalsh(r["Y"])[0] > 0
    assert np.linalg.eigvalsh(rd["X"])[0] > 0
    assert np.allclose(np.diag(rd["X"]), 1.0, atol=1e-6)
    assert np.allclose(np.diag(rm["Xbar"]), 1.0, atol=1e-6)
    # the completion of the final partial matrix is PD and keeps its entries
    Xh = rm["Xhat"]
    assert np.linalg.eigvalsh(Xh)[0] > 0
    nz = rm["Xbar"] != 0
    assert np.array_equal(Xh[nz], rm["Xbar"][nz])
    assert abs(_value(rd) - _value(rm)) <= 5e-7 * abs(_value(rd))
    tight_d = dense_pdipm(prob, TIGHT)
    tight_m = mc_pdipm(prob, TIGHT)
    assert np.allclose(tight_d["z"], tight_m["z"], atol=1e-6)


def test_step_length_boundary():
    rng = np.random.default_rng(8)
    n = 12
    X = sdpgen.random_pd_dense(n, rng)
    D = rng.standard_normal((n, n))
    D = (D + D.T) * 3
    a = step_length_dense(X, D)
    assert 0 < a < 1
    assert abs(np.linalg.eigvalsh(X + a * D)[0]) <= 1e-9 * np.abs(np.linalg.eigvalsh(X)).max()
    assert np.linalg.eigvalsh(X + 0.999 * a * D)[0] > 0
    assert step_length_dense(X, np.eye(n)) == 1.0
    # clique-wise version: each clique block is singular at its own alpha
    prob = sdpgen.maxcut_band(30, bw=3, p=0.8, seed=1)
    rows, cols = oracle.aggregate_pattern(prob)
    ch = oracle.chordal_structure(30, rows, cols)
    E = ch.E_mask()
    Xb = np.where(E, sdpgen.random_pd_dense(30, rng), 0.0)
    Dd = rng.standard_normal((30, 30))
    Dd = np.where(E, Dd + Dd.T, 0.0) * 4
    ap, al = step_length_cliques(ch, Xb, Dd)
    assert ap == al.min()
    for r, C in enumerate(ch.cliques):
        if al[r] < 1:
            blk = Xb[np.ix_(C, C)] + al[r] * Dd[np.ix_(C, C)]
            assert abs(np.linalg.eigvalsh(blk)[0]) <= 1e-9 * np.abs(Xb[np.ix_(C, C)]).max()
