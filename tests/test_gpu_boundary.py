"""GPU: the remaining entry points and paths of the C ABI against the oracle.

  * the generic substitution walk (solve_kernel = 1, and the default choice
    when the matrix-core walk does not fit) against the oracle's completion,
    inverse and Schur complement matrix;
  * the Schur complement matrix at a general (not central) state at the
    full sizes of the max-cut band workload (n = m = 4000) and the
    norm-minimisation workload (n = 2010, m = 64), on seeded samples of its
    columns;
  * sdpc_complete_dense (the max-determinant completion of the current
    iterate, Section 2.1) against the oracle's completion;
  * a failed iteration leaves the iterate untouched;
  * two identical solves are bit for bit identical;
  * the Schur complement phase a step enqueues ahead is dropped when the state
    changes, and calls between steps leave the iterates as they would be.

Tolerances as in test_gpu_parity (1e-10 relative to max |B| for states with
cond <= ~50).
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle.symbolic import aggregate_pattern, chordal_structure
from tests.gpu_common import dev, from_E, host, rel_err, to_E

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_6919_amd import load
    load()


def _create(prob, **kw):
    from paper_1310_6919_amd import sdpc_create
    return sdpc_create(prob, **kw)


CASES = {
    "cfg1": lambda: sdpgen.maxcut_cycle_chords(64, 0),
    "band300": lambda: sdpgen.maxcut_band(300, 20, 0.5, 1),
    "band_ragged": lambda: sdpgen.maxcut_band(333, 7, 0.7, 2),
    "normmin": lambda: sdpgen.normmin(100, 10, 8, 0),
    "random_sdp": lambda: sdpgen.random_sparse_sdp(45, 20, seed=4),
    "band_wide": lambda: sdpgen.maxcut_band(260, 50, 0.9, 5),
}


def _state(prob, rng, cond=8.0):
    rows, cols = aggregate_pattern(prob)
    Xfull = sdpgen.random_pd_dense(prob.n, rng, cond=cond)
    Y = sdpgen.random_pd_on_pattern(prob.n, rows, cols, rng)
    return Xfull, Y


def _oracle_completion(prob, Xfull):
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)   # natural order, the library's default
    return oracle.maxdet_complete(ch, np.where(ch.E_mask(), Xfull, 0.0))


def _check_scm(prob, h, rng, cols=None):
    Xfull, Y = _state(prob, rng)
    B = np.tril(host(h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)))))
    Xh = _oracle_completion(prob, Xfull)
    Yi = np.linalg.inv(Y)
    A = oracle.scm.problem_mats(prob)
    Bref = oracle.dense_scm(A, Xh, Yi, cols=None if cols is None else set(int(c) for c in cols))
    if cols is None:
        assert rel_err(B, np.tril(Bref)) <= 1e-10
    else:
        low = np.arange(prob.m)[:, None] >= np.asarray(cols)[None, :]
        assert rel_err(np.where(low, B[:, cols], 0.0), np.where(low, Bref[:, cols], 0.0)) <= 1e-10
    _, _, perm = h.sdpc_get_pattern()
    Xd, Yd = h.sdpc_get_dense()
    assert rel_err(host(Xd), Xh[np.ix_(perm, perm)]) <= 1e-10
    assert rel_err(host(Yd), Yi[np.ix_(perm, perm)]) <= 1e-10


# ----------------------------------------------------------------- generic substitution walk
@pytest.mark.parametrize("name", sorted(CASES))
def test_scm_generic_walk_matches_oracle(name):
    """solve_kernel = 1: X^ and Y^{-1} from the generic walk, and B from them."""
    prob = CASES[name]()
    h = _create(prob, solve_kernel=1)
    _check_scm(prob, h, np.random.default_rng(7))
    h.close()


def test_scm_one_column_blocks_match_oracle():
    """3000 storage blocks of one column: the matrix-core walk's descriptor table does
    not fit its LDS, so the default choice is the generic walk."""
    prob = sdpgen.maxcut_band(3000, 3, 0.7, 3)
    from paper_1310_6919_amd.sdpc import sdpc_analyze
    assert sdpc_analyze(prob, block_width=1)[0]["nblocks"] == 3000
    h = _create(prob, block_width=1)
    _check_scm(prob, h, np.random.default_rng(8))
    h.close()


# ----------------------------------------------------------------- full sizes, general state
def test_scm_general_state_bench_workload():
    """max-cut band n = m = 4000 (the bench workload, default parameters): B at a
    random positive definite state on 64 seeded columns, and the whole X^ and Y^{-1}."""
    prob = sdpgen.maxcut_band(4000, 20, 0.5, 0)
    rng = np.random.default_rng(31)
    cols = np.sort(np.random.default_rng(32).choice(prob.m, 64, replace=False))
    h = _create(prob)
    _check_scm(prob, h, rng, cols=cols)
    h.close()


def test_scm_general_state_normmin_full_size():
    """norm minimisation p = 2000, q = 10, 63 coefficients (n = 2010, m = 64): B at a
    random positive definite state on 8 seeded columns (the general, non-Hadamard path)."""
    prob = sdpgen.normmin(2000, 10, 63, 0)
    rng = np.random.default_rng(41)
    cols = np.sort(np.random.default_rng(42).choice(prob.m, 8, replace=False))
    h = _create(prob)
    _check_scm(prob, h, rng, cols=cols)
    h.close()


# ----------------------------------------------------------------- completion of the current iterate
@pytest.mark.parametrize("name", ["cfg1", "band_ragged", "normmin", "random_sdp", "band_wide"])
def test_complete_dense_matches_oracle(name):
    prob = CASES[name]()
    rng = np.random.default_rng(13)
    Xfull, Y = _state(prob, rng)
    z = rng.standard_normal(prob.m) * 0.1
    h = _create(prob)
    h.sdpc_set_state(dev(to_E(h, Xfull)), dev(to_E(h, Y)), dev(z))
    Xh = host(h.sdpc_complete_dense())
    assert rel_err(Xh, _oracle_completion(prob, Xfull)) <= 1e-10
    # after two iterations: the completion of the iterate the handle now holds
    h.sdpc_reset()
    h.sdpc_step()
    h.sdpc_step()
    X_E, _, _ = h.sdpc_get_solution()
    Xbar = from_E(h, host(X_E))
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    ref = oracle.maxdet_complete(ch, Xbar)
    assert rel_err(host(h.sdpc_complete_dense()), ref) <= 1e-10
    h.close()


def test_complete_dense_rejects_non_pd_clique():
    prob = CASES["cfg1"]()
    h = _create(prob)
    X = np.eye(prob.n)
    X[4, 4] = -1.0
    h.sdpc_set_state(dev(to_E(h, X)), dev(to_E(h, np.eye(prob.n))), dev(np.zeros(prob.m)))
    from paper_1310_6919_amd import SdpcError
    from paper_1310_6919_amd.sdpc import SDPC_E_NOT_PD
    with pytest.raises(SdpcError) as e:
        h.sdpc_complete_dense()
    assert e.value.status == SDPC_E_NOT_PD
    h.close()


# ----------------------------------------------------------------- failed iterations
def _snapshot(h):
    return [host(t).copy() for t in h.sdpc_get_solution()]


def test_failed_step_keeps_iterate_when_y_not_pd():
    """A Y that is not positive definite: the Y factorisation reports it, and the
    iteration changes none of X, Y and z."""
    prob = CASES["band_ragged"]()
    rng = np.random.default_rng(17)
    Xfull, Y = _state(prob, rng)
    Y[5, 5] = -1.0
    z = rng.standard_normal(prob.m) * 0.1
    h = _create(prob)
    h.sdpc_set_state(dev(to_E(h, Xfull)), dev(to_E(h, Y)), dev(z))
    before = _snapshot(h)
    from paper_1310_6919_amd import SdpcError
    from paper_1310_6919_amd.sdpc import SDPC_E_NOT_PD
    with pytest.raises(SdpcError) as e:
        h.sdpc_step()
    assert e.value.status == SDPC_E_NOT_PD
    for a, b in zip(before, _snapshot(h)):
        assert np.array_equal(a, b)
    h.close()


def test_failed_step_keeps_iterate_when_scm_singular():
    """A constraint matrix that is zero makes B singular (a zero row and column): the
    SCM Cholesky reports the pivot, and the iteration changes none of X, Y and z."""
    base = sdpgen.random_sparse_sdp(30, 8, seed=6)
    mats = [base.triplets(k) for k in range(base.m + 1)]
    mats[3] = (np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    b = base.b.copy()
    b[2] = 0.0
    prob = sdpgen.from_matrices(base.n, mats, b, name="zero_constraint")
    h = _create(prob)
    h.sdpc_reset()
    before = _snapshot(h)
    from paper_1310_6919_amd import SdpcError
    from paper_1310_6919_amd.sdpc import SDPC_E_NOT_PD
    with pytest.raises(SdpcError) as e:
        h.sdpc_step()
    assert e.value.status == SDPC_E_NOT_PD
    assert "pivot 2" in str(e.value)
    for a, b_ in zip(before, _snapshot(h)):
        assert np.array_equal(a, b_)
    h.close()


# ----------------------------------------------------------------- determinism
@pytest.mark.parametrize("name", ["band_ragged", "normmin"])
def test_solves_are_bitwise_reproducible(name):
    """Every reduction has a fixed order: two solves of one problem (and on two
    handles) give the same iterates bit for bit."""
    prob = CASES[name]()
    out = []
    h = _create(prob)
    for _ in range(2):
        r = h.sdpc_solve()
        assert r["status"] == 0, r
        out.append((r["iters"], r["pobj"], r["dobj"], *_snapshot(h)))
    h.close()
    h = _create(prob)
    r = h.sdpc_solve()
    out.append((r["iters"], r["pobj"], r["dobj"], *_snapshot(h)))
    h.close()
    for o in out[1:]:
        assert o[0] == out[0][0] and o[1] == out[0][1] and o[2] == out[0][2]
        for a, b in zip(o[3:], out[0][3:]):
            assert np.array_equal(a, b)


# ----------------------------------------------------------------- the phase enqueued ahead
@pytest.mark.parametrize("name", ["band_ragged", "normmin", "random_sdp"])
def test_state_set_between_steps_discards_phase_enqueued_ahead(name):
    """A step leaves the next iteration's Schur complement phase enqueued (for the
    iterate it produced); a new state set before the next step must not use it:
    that step's direction is the oracle's at the new state."""
    prob = CASES[name]()
    h = _create(prob)
    h.sdpc_reset()
    h.sdpc_step()
    h.sdpc_step()
    rng = np.random.default_rng(23)
    Xfull, Y = _state(prob, rng)
    z = rng.standard_normal(prob.m) * 0.1
    h.sdpc_set_state(dev(to_E(h, Xfull)), dev(to_E(h, Y)), dev(z))
    h.sdpc_step()
    dz, dX, dY, (ap, ad) = h.sdpc_get_direction()
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    A = oracle.pdipm.permuted_mats(prob, ch)
    ref = oracle.mc_direction(ch, A, prob.b, np.where(ch.E_mask(), Xfull, 0.0), Y, z)
    assert rel_err(host(dz), ref["dz"]) <= 1e-9
    assert rel_err(from_E(h, host(dY)), ref["dY"]) <= 1e-9
    assert rel_err(from_E(h, host(dX)), ref["dX"]) <= 1e-9
    assert abs(ap - ref["alpha_p"]) <= 1e-9 * max(1.0, ref["alpha_p"])
    assert ref["alpha_d"] * (1 - 1e-4) <= ad <= ref["alpha_d"] * (1 + 1e-12)
    h.close()


@pytest.mark.parametrize("name", ["band_ragged", "normmin"])
def test_calls_between_steps_leave_the_iterates(name):
    """sdpc_complete_dense, sdpc_scm, sdpc_get_factors and sdpc_get_dense between
    steps overwrite the buffers of the phase a step enqueued ahead; the following
    steps recompute it and the iterates stay those of uninterrupted steps (up to
    the rounding of the Y factor, formed afresh instead of taken from the dual
    step's twin)."""
    prob = CASES[name]()
    ref = _create(prob)
    ref.sdpc_reset()
    for _ in range(5):
        ref.sdpc_step()
    want = _snapshot(ref)
    ref.close()
    h = _create(prob)
    h.sdpc_reset()
    h.sdpc_step()
    h.sdpc_complete_dense()
    h.sdpc_step()
    X_E, Y_E, _ = h.sdpc_get_solution()
    B = h.sdpc_scm(X_E, Y_E)
    assert np.isfinite(host(B)).all()
    h.sdpc_step()
    h.sdpc_get_factors()
    h.sdpc_get_dense()
    h.sdpc_step()
    h.sdpc_step()
    for a, b in zip(_snapshot(h), want):
        assert rel_err(a, b) <= 1e-10
    h.close()


# ----------------------------------------------------------------- storage blocks
def _ktree_case():
    prob = sdpgen.maxcut_ktree_batch(4, 0)[1]
    return prob, {"user_perm": np.arange(prob.n)[::-1].astype(np.int32)}


@pytest.mark.parametrize("name", ["normmin", "normmin_wide", "ktree"])
def test_sibling_merged_blocks_match_chain_blocks(name):
    """merge_siblings only adds explicit zeros to the storage panels: the Schur
    complement matrix and whole solves agree with the chain-only blocks, and B
    with the oracle."""
    if name == "ktree":
        prob, kw = _ktree_case()
    elif name == "normmin_wide":
        prob, kw = sdpgen.normmin(300, 10, 12, 2), {}
    else:
        prob, kw = CASES[name](), {}
    rng = np.random.default_rng(31)
    Xfull, Y = _state(prob, rng)
    Bs, res = [], []
    for ms in (0, 1):
        h = _create(prob, merge_siblings=ms, gap_tol=1e-8, feas_tol=1e-8, **kw)
        Bs.append(np.tril(host(h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y))))))
        res.append(h.sdpc_solve())
        _, _, perm = h.sdpc_get_pattern()
        h.close()
    assert rel_err(Bs[1], Bs[0]) <= 1e-12
    # the oracle's completion on the E of the library's elimination order
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols, perm)
    Xh = ch.unpermute(oracle.maxdet_complete(ch, np.where(ch.E_mask(), ch.permute(Xfull), 0.0)))
    Bref = oracle.dense_scm(oracle.scm.problem_mats(prob), Xh, np.linalg.inv(Y))
    assert rel_err(Bs[1], np.tril(Bref)) <= 1e-10
    assert res[0]["status"] == 0 and res[1]["status"] == 0
    assert res[0]["iters"] == res[1]["iters"]
    o0, o1 = [(r["pobj"] + r["dobj"]) / 2 for r in res]
    assert abs(o1 - o0) <= 1e-9 * max(1.0, abs(o0))
