"""GPU: the adjoint of the central-point solve (sdpc_center, sdpc_adjoint and the
torch.autograd binding) on the band-16 max-cut differentiation workload
(n = 2000, every in-band edge, weights U[0.5, 1.5], seed 0; loss
L = <G_L, X> + |z|^2 with G_L ~ N(0,1) on the band).

The central point is taken at the mu of a solve stopped at gap 1e-8; every
perturbed solve is re-centred at that same mu, so the adjoint and the central
differences (h = 1e-6) differentiate the same smooth map.  Bars: 1e-4 relative
per edge (1e-7 absolute for tiny gradients) against the differences, and 1e-8
relative against the oracle's dense evaluation of the same formulas at the
library's own central point.
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle.adjoint import adjoint as oracle_adjoint
from oracle.symbolic import aggregate_pattern, chordal_structure
from tests.gpu_common import dev, from_E, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_6919_amd import load
    load()


GAP = dict(gap_tol=1e-8, feas_tol=1e-8)


def _a0_from_w(prob, w):
    """A_0 = -(Diag(W e) - W)/4 as the values of prob's A_0 triplets (diagonal then
    edges, the generator's packing), differentiable in w."""
    edges = torch.as_tensor(prob.meta["edges"], device=w.device)
    deg = torch.zeros(prob.n, dtype=w.dtype, device=w.device)
    deg = deg.index_add(0, edges[:, 0], w).index_add(0, edges[:, 1], w)
    return torch.cat([-deg / 4.0, w / 4.0])


def _loss_terms(h, prob, gl):
    """Coefficients c_s of <G_L, X> = sum_s c_s Xbar_E[s] (G_L given as lower triplets)."""
    iE, jE, _ = h.sdpc_get_pattern()
    key = {(int(a), int(b)): s for s, (a, b) in enumerate(zip(iE, jE)) if a >= 0}
    gr, gc, gv = gl
    c = np.zeros(len(iE))
    for a, b, v in zip(gr, gc, gv):
        s = key.get((int(a), int(b)), key.get((int(b), int(a))))
        c[s] += v if a == b else 2 * v
    return torch.as_tensor(c, device="cuda")


@pytest.fixture(scope="module")
def case():
    prob, gl, sel = sdpgen.maxcut_adjoint_case(2000, 16, 0, nedges=20)
    from paper_1310_6919_amd import sdpc_create
    h = sdpc_create(prob, **GAP)
    r = h.sdpc_solve()
    assert r["status"] == 0
    mu = r["mu"]
    c = _loss_terms(h, prob, gl)
    h.close()
    return prob, gl, sel, mu, c


def _forward(prob, w, mu, c):
    from paper_1310_6919_amd.autograd import CentralSDP
    a0 = _a0_from_w(prob, w)
    b = torch.as_tensor(prob.b, device="cuda")
    X_E, z = CentralSDP.apply(a0, b, prob, mu, GAP)
    return (c * X_E).sum() + (z * z).sum()


def _central_loss(prob, w, mu, c):
    """The same loss without autograd: solve, centre at mu, evaluate, release."""
    from paper_1310_6919_amd import sdpc_create
    p2 = sdpgen.maxcut(prob.n, prob.meta["edges"], w)
    h = sdpc_create(p2, **GAP)
    assert h.sdpc_solve()["status"] == 0
    h.sdpc_center(mu)
    X_E, _, z = h.sdpc_get_solution()
    val = float((c * X_E).sum() + (z * z).sum())
    h.close()
    return val


def test_center_converges(case):
    prob, gl, sel, mu, c = case
    from paper_1310_6919_amd import sdpc_create
    h = sdpc_create(prob, **GAP)
    h.sdpc_solve()
    steps, rel = h.sdpc_center(mu)
    assert rel <= 1e-14 and steps < 60
    X_E, Y_E, _ = h.sdpc_get_solution()
    # X^ Y = mu I: its diagonal equals mu (the solve's own end point is only
    # near the path, within a factor of a few of its mu)
    Xh = host(h.sdpc_complete_dense())
    Y = from_E(h, host(Y_E))
    assert np.abs(np.einsum("ij,ji->i", Xh, Y) - mu).max() <= 1e-3 * mu
    h.close()


def test_adjoint_matches_central_differences(case):
    prob, gl, sel, mu, c = case
    w0 = torch.as_tensor(prob.meta["weights"], device="cuda").clone().requires_grad_(True)
    L = _forward(prob, w0, mu, c)
    L.backward()
    grad = host(w0.grad)
    hstep = 1e-6
    for e in sel:
        vals = []
        for s in (+1, -1):
            w = np.array(prob.meta["weights"], dtype=np.float64, copy=True)
            w[e] += s * hstep
            vals.append(_central_loss(prob, w, mu, c))
        fd = (vals[0] - vals[1]) / (2 * hstep)
        assert abs(fd - grad[e]) <= max(1e-4 * abs(grad[e]), 1e-7), (int(e), fd, grad[e])


@pytest.mark.parametrize("gap", [1e-4, 1e-8])
def test_adjoint_matches_dense_oracle_formula(case, gap):
    """The library's dL/db and dL/dA_0 against the oracle's dense evaluation of the same
    formulas at the library's own central point.  At the mu of a gap-1e-4 solve B is
    well conditioned and the bar is 1e-9; at the differentiation workload's mu (gap
    1e-8) the solve for lambda loses cond(B) times the unit roundoff, and the bar is
    derived from it: 4 cond(B) 2^-53 (the central differences above check that
    point's gradient independently)."""
    prob, gl, sel, _, c = case
    from paper_1310_6919_amd import sdpc_create
    h = sdpc_create(prob, gap_tol=gap, feas_tol=1e-8)
    r = h.sdpc_solve()
    assert r["status"] == 0
    h.sdpc_center(r["mu"])
    X_E, Y_E, z = h.sdpc_get_solution()
    gr, gc, gv = gl
    GL = np.zeros((prob.n, prob.n))
    GL[gr, gc] = gv
    GL[gc, gr] = gv
    gb, gC = h.sdpc_adjoint(dev(_gl_E(h, GL)), 2 * z)
    # the oracle at the library's central point: completion, dense inverse, formulas
    _, _, perm = h.sdpc_get_pattern()
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols, perm)
    Xbar = from_E(h, host(X_E))
    Xh = ch.unpermute(oracle.maxdet_complete(ch, ch.permute(Xbar)))
    Y = from_E(h, host(Y_E))
    lam, Gam = oracle_adjoint(prob, Xh, Y, host(z), GL, 2 * host(z))
    if gap >= 1e-4:
        bar = 1e-9
    else:
        B = oracle.dense_scm(oracle.scm.problem_mats(prob), Xh, np.linalg.inv(Y))
        bar = max(1e-9, 4 * np.linalg.cond(B) * 2.0 ** -53)
        assert bar <= 1e-3   # the derived bar must still say something
    assert np.abs(host(gb) - lam).max() <= bar * np.abs(lam).max()
    iE, jE, _ = h.sdpc_get_pattern()
    ok = iE >= 0
    assert np.abs(host(gC)[ok] - Gam[iE[ok], jE[ok]]).max() <= bar * np.abs(Gam).max()
    assert np.all(host(gC)[~ok] == 0)
    h.close()


def _gl_E(h, GL):
    iE, jE, _ = h.sdpc_get_pattern()
    v = np.zeros(len(iE))
    ok = iE >= 0
    v[ok] = GL[iE[ok], jE[ok]]
    return v
