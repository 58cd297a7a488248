"""GPU parity of the earlier factorisation X^ = L^T D L (Section 2.1, eqs.
sparse_fact, orig_L, orig_D; factorization = 1), through the C ABI, against the
oracle's sparse_factors and its max-determinant completion.

L^{-1} depends on how the columns are grouped into supernodes, so the oracle is
built for the library's own elimination order and its supernodes are checked
to be the library's.  Tolerances as in the other parity tests (FP64, states with
cond <= ~50): 1e-10 relative for L^{-1}, X^ and B; full solves to the
matrix-completion oracle's objective (1e-7) and z (1e-6).
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle.symbolic import aggregate_pattern, chordal_structure
from tests.gpu_common import dev, host, rel_err, to_E

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_6919_amd import load
    load()


CASES = {
    "cfg1": lambda: sdpgen.maxcut_cycle_chords(64, 0),
    "band300": lambda: sdpgen.maxcut_band(300, 20, 0.5, 1),
    "band_ragged": lambda: sdpgen.maxcut_band(333, 7, 0.7, 2),
    "normmin": lambda: sdpgen.normmin(100, 10, 8, 0),
    "random_sdp": lambda: sdpgen.random_sparse_sdp(40, 12, 5),
}


def _create(prob, **kw):
    from paper_1310_6919_amd import sdpc_create
    return sdpc_create(prob, factorization=1, **kw)


def _state(prob, rng):
    rows, cols = aggregate_pattern(prob)
    return sdpgen.random_pd_dense(prob.n, rng, cond=8.0), sdpgen.random_pd_on_pattern(prob.n, rows, cols, rng)


def _oracle_in_library_order(h, prob):
    """The oracle's chordal structure for the library's elimination order, with the
    supernodes checked against the library's clique list."""
    _, _, perm = h.sdpc_get_pattern()
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols, perm)
    cl, nS = h.sdpc_get_cliques()
    assert len(cl) == ch.ell and np.array_equal(nS, ch.nS)
    for C, Co in zip(cl, ch.cliques):
        assert np.array_equal(np.sort(ch.pos[C]), Co)
    return ch


@pytest.mark.parametrize("name", sorted(CASES))
def test_ldl_factor_matches_oracle(name):
    prob = CASES[name]()
    rng = np.random.default_rng(21)
    Xfull, Y = _state(prob, rng)
    h = _create(prob)
    h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)))
    _, Linv = h.sdpc_get_factors()          # factorization 1: L^{-1} of X^ = L^T D L
    ch = _oracle_in_library_order(h, prob)
    E = ch.E_mask()
    L, D = oracle.sparse_factors(ch, np.where(E, ch.permute(Xfull), 0.0))
    Lref = np.linalg.inv(L)
    iE, jE, _ = h.sdpc_get_pattern()
    ok = iE >= 0
    pi, pj = ch.pos[iE[ok]], ch.pos[jE[ok]]
    lo_i, lo_j = np.maximum(pi, pj), np.minimum(pi, pj)
    assert rel_err(host(Linv)[ok], Lref[lo_i, lo_j]) <= 1e-10
    assert np.all(host(Linv)[~ok] == 0)
    # L^{-1} lies within E (the property the substitutions rely on): the stored
    # slots carry all of it
    Lg = np.zeros((prob.n, prob.n))
    Lg[lo_i, lo_j] = host(Linv)[ok]
    assert rel_err(Lg, Lref) <= 1e-10
    h.close()


@pytest.mark.parametrize("name", sorted(CASES))
def test_ldl_scm_and_completion_match_oracle(name):
    prob = CASES[name]()
    rng = np.random.default_rng(7)
    Xfull, Y = _state(prob, rng)
    h = _create(prob)
    B = np.tril(host(h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)))))
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    Xh = oracle.maxdet_complete(ch, np.where(ch.E_mask(), Xfull, 0.0))
    Bref = oracle.dense_scm(oracle.scm.problem_mats(prob), Xh, np.linalg.inv(Y))
    assert rel_err(B, np.tril(Bref)) <= 1e-10
    Xg, _ = h.sdpc_get_dense()
    _, _, perm = h.sdpc_get_pattern()
    assert rel_err(host(Xg), Xh[np.ix_(perm, perm)]) <= 1e-10
    # the completion of the handle's current X, in original indices
    h.sdpc_set_state(dev(to_E(h, Xfull)), dev(to_E(h, Y)), dev(np.zeros(prob.m)))
    assert rel_err(host(h.sdpc_complete_dense()), Xh) <= 1e-10
    h.close()


@pytest.mark.parametrize("name,gap", [("cfg1", 1e-7), ("band_ragged", 1e-8), ("normmin", 1e-8)])
def test_ldl_solve_matches_mc_oracle(name, gap):
    prob = CASES[name]()
    h = _create(prob, gap_tol=gap, feas_tol=gap)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    ref = oracle.mc_pdipm(prob, oracle.Params(gap_tol=gap, feas_tol=gap))
    assert ref["status"] == "optimal" and r["iters"] == ref["iters"]
    obj, robj = (r["pobj"] + r["dobj"]) / 2, (ref["pobj"] + ref["dobj"]) / 2
    assert abs(obj - robj) <= 1e-7 * max(1.0, abs(robj))
    _, _, z = h.sdpc_get_solution()
    z = host(z)
    assert np.abs(z - ref["z"]).max() <= 1e-6 * max(1.0, np.abs(ref["z"]).max())
    # the same optimum and iteration count as the Algorithm 1 route
    from paper_1310_6919_amd import sdpc_create
    h0 = sdpc_create(prob, gap_tol=gap, feas_tol=gap)
    r0 = h0.sdpc_solve()
    assert r0["iters"] == r["iters"]
    assert abs((r0["pobj"] + r0["dobj"]) / 2 - obj) <= 1e-8 * max(1.0, abs(obj))
    h0.close()
    h.close()


def test_ldl_rejects_supernode_split_over_blocks():
    # one-column storage blocks cut the band's multi-column supernodes: D_r would span
    # several blocks, which the substitution walks cannot apply
    from paper_1310_6919_amd import SdpcError
    from paper_1310_6919_amd.sdpc import SDPC_E_PATTERN
    with pytest.raises(SdpcError) as e:
        _create(CASES["band300"](), block_width=1)
    assert e.value.status == SDPC_E_PATTERN
