"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (FP64 throughout; derived from the arithmetic, the paper fixes
none): one SCM evaluation involves two sparse triangular inversions and a
dense product, each backward stable, so entries of B agree to a few hundred
ulps times the conditioning of the factors; the states used here keep
cond(X), cond(Y) <= ~50, hence 1e-10 relative to max|B|.  Full solves are
compared on the objective (1e-7 relative at gap 1e-7) and on z (1e-6 at a
tighter gap), the targets of the method's comparison with the oracle.
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle.symbolic import aggregate_pattern, chordal_structure
from tests.gpu_common import dev, from_E, golden, host, rel_err, to_E

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
    # cliques of 51 and storage blocks of 82 rows: the Y factor's tall-panel kernel
    "band_wide": lambda: sdpgen.maxcut_band(260, 50, 0.9, 5),
}


# ----------------------------------------------------------------- dense Cholesky
# last blocks of every width class: one column, at and just over each 16-column
# panel boundary of a block (later panels empty, exactly full, partly real), full
@pytest.mark.parametrize("m", [1, 5, 63, 64, 65, 80, 81, 96, 97, 100, 112, 113, 128, 130, 200, 257])
@pytest.mark.parametrize("kernel", [0, 1])
def test_potrf_matches_lapack(m, kernel):
    rng = np.random.default_rng(m)
    prob = sdpgen.maxcut_band(300, 3, 1.0, 0)
    h = _create(prob, chol_kernel=kernel)
    A = sdpgen.random_pd_dense(m, rng, cond=1e3)
    Bt = dev(A.T.copy()).T            # column-major view
    upper_marker = np.triu(np.full((m, m), 7.0), 1)
    Bt += dev(upper_marker.T.copy()).T
    h.sdpc_potrf(Bt, m)
    R = np.tril(host(Bt))
    Rref = np.linalg.cholesky(A)
    assert rel_err(R, Rref) <= 1e-12 * 1e3
    assert np.array_equal(np.triu(host(Bt), 1), np.triu(A, 1) + upper_marker)   # strict upper untouched
    h.close()


# Many more tiles than the GPU holds resident workgroups (m = 8000: 125 column blocks,
# about 7900 tasks of the one-launch form), factorised three times each: every run
# matches LAPACK and the runs agree bit for bit, so no hand-over between tasks reads
# a tile before it is final.
@pytest.mark.parametrize("kernel", [0, 1])
def test_potrf_large_repeatable(kernel):
    m = 8000
    rng = np.random.default_rng(8000)
    G = rng.standard_normal((m, m))
    A = G @ G.T / m + 0.05 * np.eye(m)
    Rref = np.linalg.cholesky(A)
    h = _create(sdpgen.maxcut_band(m, 3, 1.0, 0), chol_kernel=kernel)
    first = None
    for _ in range(3):
        Bt = dev(A.T.copy()).T            # column-major view
        h.sdpc_potrf(Bt, m)
        R = np.tril(host(Bt))
        assert rel_err(R, Rref) <= 1e-12
        if first is None:
            first = R
        else:
            assert np.array_equal(R, first)
    h.close()


# the failing pivot in each 16-column panel of a block, in the first block and a
# later one, and the last pivot of a ragged last block
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("m,piv", [(80, 3), (80, 20), (80, 40), (80, 50), (130, 70), (130, 127), (130, 129)])
def test_potrf_reports_not_pd(m, piv, kernel):
    prob = sdpgen.maxcut_band(300, 3, 1.0, 0)   # handle sized for m <= 300
    h = _create(prob, chol_kernel=kernel)
    A = np.eye(m)
    A[piv, piv] = -1.0
    Bt = dev(A.T.copy()).T
    from paper_1310_6919_amd import SdpcError
    with pytest.raises(SdpcError) as e:
        h.sdpc_potrf(Bt, m)
    assert f"pivot {piv}" in str(e.value)
    h.close()


# ----------------------------------------------------------------- one SCM evaluation
def _state(prob, rng):
    rows, cols = aggregate_pattern(prob)
    Xfull = sdpgen.random_pd_dense(prob.n, rng, cond=8.0)
    Y = sdpgen.random_pd_on_pattern(prob.n, rows, cols, rng)
    return Xfull, Y


@pytest.mark.parametrize("name", sorted(CASES))
def test_scm_parity(name):
    prob = CASES[name]()
    rng = np.random.default_rng(7)
    Xfull, Y = _state(prob, rng)
    h = _create(prob)
    B = h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)))
    Bg = np.tril(host(B))          # column-major storage -> numpy
    # oracle: its own chordal extension for the natural order (same E as any postorder of it)
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    E = ch.E_mask()
    Xh = oracle.maxdet_complete(ch, np.where(E, Xfull, 0.0))
    A = oracle.scm.problem_mats(prob)
    Bref = oracle.dense_scm(A, Xh, np.linalg.inv(Y))
    assert rel_err(Bg, np.tril(Bref)) <= 1e-10
    # the dense intermediates, in the library's elimination order
    _, _, perm = h.sdpc_get_pattern()
    Xd, Yd = h.sdpc_get_dense()
    assert rel_err(host(Xd), Xh[np.ix_(perm, perm)]) <= 1e-10
    assert rel_err(host(Yd), np.linalg.inv(Y)[np.ix_(perm, perm)]) <= 1e-10
    h.close()


@pytest.mark.parametrize("name", ["cfg1", "band_ragged", "normmin"])
def test_factors_match_textbook(name):
    prob = CASES[name]()
    rng = np.random.default_rng(11)
    Xfull, Y = _state(prob, rng)
    h = _create(prob)
    h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)))
    N, L = h.sdpc_get_factors()
    iE, jE, perm = h.sdpc_get_pattern()
    pos = np.empty(prob.n, dtype=int)
    pos[perm] = np.arange(prob.n)
    ok = iE >= 0
    # Y = N N^T and X^{-1} = Lhat Lhat^T in the library's order (unique Cholesky factors)
    Nref = np.linalg.cholesky(Y[np.ix_(perm, perm)])
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    Xh = oracle.maxdet_complete(ch, np.where(ch.E_mask(), Xfull, 0.0))
    Lref = oracle.lhat_textbook(Xh[np.ix_(perm, perm)])
    pi, pj = pos[iE[ok]], pos[jE[ok]]
    lo_i, lo_j = np.maximum(pi, pj), np.minimum(pi, pj)
    assert rel_err(host(N)[ok], Nref[lo_i, lo_j]) <= 1e-11
    assert rel_err(host(L)[ok], Lref[lo_i, lo_j]) <= 1e-10
    # padding slots hold exact zeros; factors vanish off E (Algorithm 1 keeps Lhat within E)
    assert np.all(host(N)[~ok] == 0) and np.all(host(L)[~ok] == 0)
    Lfull = np.zeros((prob.n, prob.n))
    Lfull[lo_i, lo_j] = host(L)[ok]
    assert rel_err(Lfull, np.tril(Lref)) <= 1e-10
    h.close()


def test_scm_central_point_pin():
    # X = mu Y^{-1} on E: X^ = mu Y^{-1}, Lhat = N / sqrt(mu) and B = mu (Y^{-1} o Y^{-1})
    prob = sdpgen.maxcut_band(200, 6, 0.8, 3)
    rng = np.random.default_rng(3)
    rows, cols = aggregate_pattern(prob)
    Y = sdpgen.random_pd_on_pattern(prob.n, rows, cols, rng)
    mu = 0.3
    Yi = np.linalg.inv(Y)
    h = _create(prob)
    B = h.sdpc_scm(dev(to_E(h, mu * Yi)), dev(to_E(h, Y)))
    assert rel_err(np.tril(host(B)), np.tril(mu * Yi * Yi)) <= 1e-10
    N, L = h.sdpc_get_factors()
    assert rel_err(host(L), host(N) / np.sqrt(mu)) <= 1e-10
    h.close()


def test_scm_iteration0_gram():
    # X = Y = lambda I: B = [A_p . A_q]
    prob = sdpgen.normmin(60, 6, 5, 1)
    h = _create(prob)
    lam = 100.0
    I = np.eye(prob.n)
    B = np.tril(host(h.sdpc_scm(dev(to_E(h, lam * I)), dev(to_E(h, lam * I)))))
    Ad = [prob.dense(k) for k in range(1, prob.m + 1)]
    G = np.array([[np.sum(a * b) for b in Ad] for a in Ad])
    assert rel_err(B, np.tril(G)) <= 1e-12
    h.close()


def test_scm_factor_flag():
    prob = CASES["band300"]()
    rng = np.random.default_rng(5)
    Xfull, Y = _state(prob, rng)
    h = _create(prob)
    B0 = h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)))
    Bl = np.tril(host(B0))
    R = h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)), factor=True)
    Rl = np.tril(host(R))
    Bs = Bl + np.tril(Bl, -1).T
    assert rel_err(Rl, np.linalg.cholesky(Bs)) <= 1e-10
    h.close()


def test_scm_rejects_non_pd():
    prob = CASES["cfg1"]()
    h = _create(prob)
    from paper_1310_6919_amd import SdpcError
    I = np.eye(prob.n)
    bad = I.copy()
    bad[3, 3] = -1.0
    with pytest.raises(SdpcError):
        h.sdpc_scm(dev(to_E(h, I)), dev(to_E(h, bad)))
    with pytest.raises(SdpcError):
        h.sdpc_scm(dev(to_E(h, bad)), dev(to_E(h, I)))
    h.close()


# ----------------------------------------------------------------- one PDIPM iteration
@pytest.mark.parametrize("name", ["cfg1", "band_ragged", "normmin", "random_sdp", "normmin_split"])
def test_iteration_matches_oracle(name):
    """normmin_split: the column group holding the arrow's dense columns has a row union
    of 610 rows, more than the 512 above which the products X^ M are cut into pieces."""
    prob = sdpgen.normmin(600, 10, 8, 0) if name == "normmin_split" else CASES[name]()
    rng = np.random.default_rng(21)
    Xfull, Y = _state(prob, rng)
    z = rng.standard_normal(prob.m) * 0.1
    h = _create(prob)
    h.sdpc_set_state(dev(to_E(h, Xfull)), dev(to_E(h, Y)), dev(z))
    h.sdpc_step()
    dz, dX, dY, (ap, ad) = h.sdpc_get_direction()
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    A = oracle.pdipm.permuted_mats(prob, ch)
    E = ch.E_mask()
    ref = oracle.mc_direction(ch, A, prob.b, np.where(E, Xfull, 0.0), Y, z)
    assert rel_err(host(dz), ref["dz"]) <= 1e-9
    assert rel_err(from_E(h, host(dY)), ref["dY"]) <= 1e-9
    assert rel_err(from_E(h, host(dX)), ref["dX"]) <= 1e-9
    assert abs(ap - ref["alpha_p"]) <= 1e-9 * max(1.0, ref["alpha_p"])
    # the dual step is bracketed by parallel positive-definiteness tests: relative 1e-4
    assert ad <= ref["alpha_d"] * (1 + 1e-12)
    assert ad >= ref["alpha_d"] * (1 - 1e-4)
    h.close()


# ----------------------------------------------------------------- full solves
@pytest.mark.parametrize("seed", range(5))
def test_solve_cfg1_matches_golden(seed):
    """Objective against the dense oracle's solution at gap 1e-10 (stored by
    tests/golden/make_golden.py)."""
    prob = sdpgen.maxcut_cycle_chords(64, seed)
    g = golden(f"cfg1_s{seed}")
    ref_obj = (g["pobj"] + g["dobj"]) / 2
    h = _create(prob)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    obj = (r["pobj"] + r["dobj"]) / 2
    assert abs(obj - ref_obj) <= 1e-7 * max(1.0, abs(ref_obj))
    assert r["rel_gap"] <= 1e-7 and r["pinf"] <= 1e-7 and r["dinf"] <= 1e-7
    h.close()


@pytest.mark.parametrize("name,tol", [("cfg1", 1e-7), ("cfg1", 1e-9), ("normmin", 1e-8), ("random_sdp", 1e-8),
                                      ("band_wide", 1e-8)])
def test_solve_matches_mc_oracle(name, tol):
    """The whole trajectory against the matrix-completion oracle (same method,
    same E, same step rules): iteration count, objective, and z to 1e-6."""
    prob = CASES[name]()
    P = oracle.Params(gap_tol=tol, feas_tol=tol)
    ref = oracle.mc_pdipm(prob, P)
    assert ref["status"] == "optimal"
    h = _create(prob, gap_tol=tol, feas_tol=tol)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    assert r["iters"] == ref["iters"]
    obj, robj = (r["pobj"] + r["dobj"]) / 2, (ref["pobj"] + ref["dobj"]) / 2
    assert abs(obj - robj) <= 1e-7 * max(1.0, abs(robj))
    _, _, z = h.sdpc_get_solution()
    assert np.abs(host(z) - ref["z"]).max() <= 1e-6 * max(1.0, np.abs(ref["z"]).max())
    h.close()


@pytest.mark.parametrize("name", ["band_ragged", "normmin"])
def test_update_slots_in_memory_match_pool(name):
    """The one-wave factorisation keeps pending updates in an LDS pool or, beyond the
    pool's LDS budget, in device memory: the same arithmetic in the same order, so
    the whole solve is bit for bit the same either way."""
    prob = CASES[name]()
    out = []
    for pool in (32 * 1024, 0):
        h = _create(prob, pool_lds_bytes=pool)
        r = h.sdpc_solve()
        assert r["status"] == 0, r
        X, Y, z = h.sdpc_get_solution()
        out.append((r["iters"], host(X), host(Y), host(z)))
        h.close()
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1:], out[1][1:]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("bw", [16, 24])
@pytest.mark.parametrize("pool", [32 * 1024, 0])
def test_tall_trailing_updates_match_oracle(bw, pool):
    """Bandwidth 40 in storage blocks of 16 or 24 columns: every panel has up to 40 rows
    below its diagonal block, so the one-wave factorisation updates the ancestors with
    four 16-row tiles of L21 (ten tile pairs), and 16-column blocks take the 16-wide
    elimination; with pool = 0 the pending updates live in device memory.  One SCM
    evaluation (N, B) and one iteration (direction, both step lengths, the dual step's
    candidates) against the oracle."""
    prob = sdpgen.maxcut_band(200, 40, 0.9, 6)
    from paper_1310_6919_amd.sdpc import sdpc_analyze
    info = sdpc_analyze(prob, block_width=bw)[0]
    # some block has more than 32 rows below its own columns, and every block fits a wave
    assert info["max_block_rows"] - bw > 32 and info["max_block_rows"] <= 64
    rng = np.random.default_rng(17)
    Xfull, Y = _state(prob, rng)
    h = _create(prob, block_width=bw, pool_lds_bytes=pool)
    B = h.sdpc_scm(dev(to_E(h, Xfull)), dev(to_E(h, Y)))
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols)
    E = ch.E_mask()
    Xh = oracle.maxdet_complete(ch, np.where(E, Xfull, 0.0))
    Bref = oracle.dense_scm(oracle.scm.problem_mats(prob), Xh, np.linalg.inv(Y))
    assert rel_err(np.tril(host(B)), np.tril(Bref)) <= 1e-10
    N, _ = h.sdpc_get_factors()
    iE, jE, perm = h.sdpc_get_pattern()
    pos = np.empty(prob.n, dtype=int)
    pos[perm] = np.arange(prob.n)
    ok = iE >= 0
    Nref = np.linalg.cholesky(Y[np.ix_(perm, perm)])
    pi, pj = pos[iE[ok]], pos[jE[ok]]
    assert rel_err(host(N)[ok], Nref[np.maximum(pi, pj), np.minimum(pi, pj)]) <= 1e-11
    z = rng.standard_normal(prob.m) * 0.1
    h.sdpc_set_state(dev(to_E(h, Xfull)), dev(to_E(h, Y)), dev(z))
    h.sdpc_step()
    dz, dX, dY, (ap, ad) = h.sdpc_get_direction()
    A = oracle.pdipm.permuted_mats(prob, ch)
    ref = oracle.mc_direction(ch, A, prob.b, np.where(E, Xfull, 0.0), Y, z)
    assert rel_err(host(dz), ref["dz"]) <= 1e-9
    assert rel_err(from_E(h, host(dY)), ref["dY"]) <= 1e-9
    assert rel_err(from_E(h, host(dX)), ref["dX"]) <= 1e-9
    assert abs(ap - ref["alpha_p"]) <= 1e-9 * max(1.0, ref["alpha_p"])
    assert ref["alpha_d"] * (1 - 1e-4) <= ad <= ref["alpha_d"] * (1 + 1e-12)
    h.close()


def test_solve_one_column_blocks_match_wide_blocks():
    """Storage blocks of one column (3000 of them) leave the block walk of the
    inverse-by-solves kernel without room for its descriptor table in LDS, so it
    takes the generic kernel; the solve must agree with the default 32-column
    blocks."""
    prob = sdpgen.maxcut_band(3000, 3, 0.7, 3)
    from paper_1310_6919_amd.sdpc import sdpc_analyze
    info = sdpc_analyze(prob, block_width=1)[0]
    assert info["nblocks"] == 3000
    res = []
    for bw in (1, 32):
        h = _create(prob, block_width=bw)
        r = h.sdpc_solve()
        assert r["status"] == 0, r
        res.append(r)
        h.close()
    o1, o32 = [(r["pobj"] + r["dobj"]) / 2 for r in res]
    assert abs(o1 - o32) <= 1e-7 * max(1.0, abs(o32))


def test_solve_cycles_closed_form():
    for n in (5, 8, 13):
        e = sdpgen.cycle_graph(n)
        prob = sdpgen.maxcut(n, e, np.ones(len(e)))
        h = _create(prob, gap_tol=1e-9, feas_tol=1e-9)
        r = h.sdpc_solve()
        val = oracle.cycle_sdp_value(n)
        assert abs(-(r["pobj"] + r["dobj"]) / 2 - val) <= 1e-7 * val
        h.close()


def test_solve_normmin_sigma_max():
    prob = sdpgen.normmin(150, 10, 12, 2)
    h = _create(prob, gap_tol=1e-9, feas_tol=1e-9)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    _, _, z = h.sdpc_get_solution()
    z = host(z)
    F = prob.meta["F"]
    Fy = F[0] + np.einsum("i,ijk->jk", z[1:], F[1:])
    smax = np.linalg.svd(Fy, compute_uv=False)[0]
    assert abs(z[0] - smax) <= 1e-7 * smax
    h.close()


# ----------------------------------------------------------------- full sizes
# The bench workload (max-cut on a band graph, n = m = 4000, bandwidth 20) and the
# norm-minimisation SDP (n = 2010, m = 64) at their real sizes, in the launch
# configuration the bench uses (default parameters).


def test_scm_central_point_full_size():
    """X = mu Y^{-1} on E at n = m = 4000: then X^ = mu Y^{-1} and, for max-cut,
    B = mu (Y^{-1} o Y^{-1}) entry by entry (the whole lower triangle)."""
    prob = sdpgen.maxcut_band(4000, 20, 0.5, 0)
    rng = np.random.default_rng(21)
    rows, cols = aggregate_pattern(prob)
    Y = sdpgen.random_pd_on_pattern(prob.n, rows, cols, rng)
    mu = 0.05
    Yi = np.linalg.inv(Y)
    h = _create(prob)
    B = h.sdpc_scm(dev(to_E(h, mu * Yi)), dev(to_E(h, Y)), factor=True)
    Bl = np.tril(host(B))
    ref = np.tril(mu * Yi * Yi)
    # with factor=True the lower triangle holds R; rebuild B = R R^T on a sample of rows
    sel = np.sort(rng.choice(prob.n, 64, replace=False))
    Rs = Bl[sel]
    Bs = Rs @ Bl.T
    full_ref = mu * Yi * Yi
    assert rel_err(Bs, full_ref[sel]) <= 1e-10
    h.close()
    h = _create(prob)
    B = h.sdpc_scm(dev(to_E(h, mu * Yi)), dev(to_E(h, Y)))
    assert rel_err(np.tril(host(B)), ref) <= 1e-10
    h.close()


def test_solve_bench_workload_matches_golden():
    """Objective at gap 1e-7 (the bench's stopping rule) within 1e-7 of the dense
    oracle's optimum, and z at gap 1e-9 within 1e-6 of the oracle's z (both from
    tests/golden/oracle_cfg2.json, written by tests/golden/make_golden.py)."""
    prob = sdpgen.maxcut_band(4000, 20, 0.5, 0)
    g = golden("cfg2")
    ref_obj = (g["pobj"] + g["dobj"]) / 2
    h = _create(prob)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    obj = (r["pobj"] + r["dobj"]) / 2
    assert abs(obj - ref_obj) <= 1e-7 * max(1.0, abs(ref_obj))
    assert r["rel_gap"] <= 1e-7 and r["pinf"] <= 1e-7 and r["dinf"] <= 1e-7
    h.close()
    h = _create(prob, gap_tol=1e-9, feas_tol=1e-9)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    _, _, z = h.sdpc_get_solution()
    gz = np.asarray(g["z"])
    assert np.abs(host(z) - gz).max() <= 1e-6 * max(1.0, np.abs(gz).max())
    h.close()


def test_solve_normmin_full_size_matches_golden():
    """Norm minimisation, p = 2000, q = 10, 63 coefficients (n = 2010, m = 64):
    objective within 1e-7 and z within 1e-6 of the dense oracle at gap 1e-10."""
    prob = sdpgen.normmin(2000, 10, 63, 0)
    g = golden("cfg3")
    ref_obj = (g["pobj"] + g["dobj"]) / 2
    h = _create(prob, gap_tol=1e-9, feas_tol=1e-9)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    obj = (r["pobj"] + r["dobj"]) / 2
    assert abs(obj - ref_obj) <= 1e-7 * max(1.0, abs(ref_obj))
    _, _, z = h.sdpc_get_solution()
    gz = np.asarray(g["z"])
    assert np.abs(host(z) - gz).max() <= 1e-6 * max(1.0, np.abs(gz).max())
    h.close()


# ----------------------------------------------------------------- lattice max-cut workloads
def test_lattice_solve_matches_mc_oracle():
    """A small lattice in the short-side-first elimination order (a caller-given
    order): the whole trajectory against the matrix-completion oracle in the same
    order, and the optimum against the closed form (minus the total weight)."""
    p, q = 12, 10
    prob = sdpgen.maxcut_lattice(p, q, 4)
    order = sdpgen.lattice_short_first_order(p, q)
    total = prob.meta["weights"].sum()
    ref = oracle.mc_pdipm(prob, oracle.Params(), order=order)
    assert ref["status"] == "optimal"
    h = _create(prob, user_perm=order)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    assert r["iters"] == ref["iters"]
    obj = (r["pobj"] + r["dobj"]) / 2
    assert abs(obj - (ref["pobj"] + ref["dobj"]) / 2) <= 1e-7 * total
    assert abs(obj + total) <= 2e-7 * total
    _, _, z = h.sdpc_get_solution()
    assert np.abs(host(z) - ref["z"]).max() <= 1e-6 * max(1.0, np.abs(ref["z"]).max())
    h.close()
    # the natural order (the paper's numbering: a band of width p) reaches the same optimum
    h = _create(prob)
    r2 = h.sdpc_solve()
    assert r2["status"] == 0, r2
    assert abs((r2["pobj"] + r2["dobj"]) / 2 + total) <= 2e-7 * total
    h.close()


@pytest.mark.parametrize("p", [400, 1200])
def test_lattice_full_size_closed_form(p):
    """MaxCut400 and MaxCut1200 sizes (n = m = 4000 and 12000, q = 10): the solve
    to gap 1e-7 lands on minus the total weight, the optimum of a bipartite graph."""
    prob = sdpgen.maxcut_lattice(p, 10, 0)
    total = prob.meta["weights"].sum()
    h = _create(prob, user_perm=sdpgen.lattice_short_first_order(p, 10))
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    assert r["rel_gap"] <= 1e-7 and r["pinf"] <= 1e-7 and r["dinf"] <= 1e-7
    assert abs((r["pobj"] + r["dobj"]) / 2 + total) <= 2e-7 * total
    h.close()


def test_lattice_min_degree_order_solve():
    """The minimum-degree order (ordering = 1) gives the lattice a bushy elimination
    tree of many small storage blocks instead of a band: the whole trajectory against
    the matrix-completion oracle in its own minimum-degree order (the same fill, so
    the same E), and the optimum against the closed form."""
    from oracle.symbolic import aggregate_pattern as agg, min_degree_order
    p, q = 30, 10
    prob = sdpgen.maxcut_lattice(p, q, 5)
    total = prob.meta["weights"].sum()
    rows, cols = agg(prob)
    ref = oracle.mc_pdipm(prob, oracle.Params(), order=min_degree_order(prob.n, rows, cols))
    assert ref["status"] == "optimal"
    from paper_1310_6919_amd.sdpc import sdpc_analyze
    info = sdpc_analyze(prob, ordering=1)[0]
    assert info["nblocks"] > prob.n // 8   # far more blocks than the band order's n / 32
    h = _create(prob, ordering=1)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    assert r["iters"] == ref["iters"]
    obj = (r["pobj"] + r["dobj"]) / 2
    assert abs(obj - (ref["pobj"] + ref["dobj"]) / 2) <= 1e-7 * total
    assert abs(obj + total) <= 2e-7 * total
    _, _, z = h.sdpc_get_solution()
    assert np.abs(host(z) - ref["z"]).max() <= 1e-6 * max(1.0, np.abs(ref["z"]).max())
    h.close()


def test_ktree_batch_instance_matches_mc_oracle():
    """An instance of the 256-instance k-tree max-cut batch (n = 89, k = 12: a bushy
    elimination tree) in its reverse insertion order, a perfect elimination order:
    the whole trajectory against the matrix-completion oracle in the same order."""
    prob = sdpgen.maxcut_ktree_batch(256, 0)[2]
    order = np.arange(prob.n)[::-1].astype(np.int32)
    ref = oracle.mc_pdipm(prob, oracle.Params(), order=order)
    assert ref["status"] == "optimal"
    h = _create(prob, user_perm=order)
    r = h.sdpc_solve()
    assert r["status"] == 0, r
    assert r["iters"] == ref["iters"]
    obj, robj = (r["pobj"] + r["dobj"]) / 2, (ref["pobj"] + ref["dobj"]) / 2
    assert abs(obj - robj) <= 1e-7 * max(1.0, abs(robj))
    _, _, z = h.sdpc_get_solution()
    assert np.abs(host(z) - ref["z"]).max() <= 1e-6 * max(1.0, np.abs(ref["z"]).max())
    h.close()
