"""Pins for the oracle's derivative of the central solution (oracle/adjoint.py).

The formulas are checked against central differences of the mu-central map
itself: each perturbed problem is solved by the dense oracle and re-centred at
the same mu, and the loss L = <G_L, X> + |z|^2 is differenced.  A wrong sign,
a missing term (the h(G_L) part of lambda, the z part, the symmetrisation), or
a transposed product all change the gradient by O(1) and fail here.

The central point is taken at the mu of a solve stopped at gap 1e-6: the map is
smooth at any mu > 0, and there B keeps a condition number that lets the FP64
solve for lambda resolve the 1e-6 bar (at mu ~ 1e-10 it does not).
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle.adjoint import adjoint, center


def _solve_central(prob, mu=None):
    res = oracle.dense_pdipm(prob, oracle.Params(gap_tol=1e-6, feas_tol=1e-9))
    X, Y, z = res["X"], res["Y"], res["z"]
    if mu is None:
        mu = float(np.sum(X * Y)) / prob.n
    X, Y, z, rel = center(prob, X, Y, z, mu)
    assert rel <= 1e-13
    return X, Y, z, mu


def _loss(GL, X, z):
    return float(np.sum(GL * X) + z @ z)


def _case(n=10, bw=3, seed=0):
    prob, (gr, gc, gv), _ = sdpgen.maxcut_adjoint_case(n, bw, seed, nedges=4)
    GL = np.zeros((n, n))
    GL[gr, gc] = gv
    GL[gc, gr] = gv
    return prob, GL


def test_center_reaches_the_central_point():
    prob, _ = _case()
    X, Y, z, mu = _solve_central(prob)
    assert np.abs(X @ Y - mu * np.eye(prob.n)).max() <= 1e-12 * max(1.0, np.abs(X @ Y).max())
    A = oracle.scm.problem_mats(prob)
    assert np.abs(np.array([np.sum(A[k].toarray() * X) for k in range(1, prob.m + 1)]) - prob.b).max() <= 1e-12
    G = A[0].toarray() - sum(z[k - 1] * A[k].toarray() for k in range(1, prob.m + 1)) - Y
    assert np.abs(G).max() <= 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_central_differences_in_the_weights(seed):
    prob, GL = _case(seed=seed)
    X, Y, z, mu = _solve_central(prob)
    lam, Gam = adjoint(prob, X, Y, z, GL, 2 * z)
    edges, w = prob.meta["edges"], prob.meta["weights"]
    h = 1e-5
    for e in range(0, len(w), 7):
        i, j = edges[e]
        grad = -(Gam[i, i] + Gam[j, j] - 2 * Gam[i, j]) / 4.0
        vals = []
        for s in (+1, -1):
            w2 = w.copy()
            w2[e] += s * h
            p2 = sdpgen.maxcut(prob.n, edges, w2)
            X2, _, z2, _ = _solve_central(p2, mu)
            vals.append(_loss(GL, X2, z2))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - grad) <= 1e-6 * max(1.0, abs(grad)), (e, fd, grad)


def test_adjoint_matches_central_differences_in_b_and_general_A0():
    # a general SDP with multi-entry constraints: dL/db_k and dL/d[A_0]_ij
    prob = sdpgen.random_sparse_sdp(8, 5, 3)
    rng = np.random.default_rng(4)
    GL = rng.standard_normal((8, 8))
    GL = GL + GL.T
    X, Y, z, mu = _solve_central(prob)
    lam, Gam = adjoint(prob, X, Y, z, GL, 2 * z)
    h = 1e-5
    for k in range(0, prob.m, 2):
        vals = []
        for s in (+1, -1):
            p2 = sdpgen.Problem(prob.n, prob.m, prob.ptr, prob.row, prob.col, prob.val, prob.b.copy())
            p2.b[k] += s * h
            X2, _, z2, _ = _solve_central(p2, mu)
            vals.append(_loss(GL, X2, z2))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - lam[k]) <= 1e-6 * max(1.0, abs(lam[k])), (k, fd, lam[k])
    r0, c0, _ = prob.triplets(0)
    for t in range(min(4, len(r0))):
        i, j = int(r0[t]), int(c0[t])
        vals = []
        for s in (+1, -1):
            v2 = prob.val.copy()
            v2[int(prob.ptr[0]) + t] += s * h
            p2 = sdpgen.Problem(prob.n, prob.m, prob.ptr, prob.row, prob.col, v2, prob.b)
            X2, _, z2, _ = _solve_central(p2, mu)
            vals.append(_loss(GL, X2, z2))
        fd = (vals[0] - vals[1]) / (2 * h)
        grad = Gam[i, i] if i == j else 2 * Gam[i, j]   # the triplet moves both symmetric entries
        assert abs(fd - grad) <= 1e-6 * max(1.0, abs(grad)), (t, fd, grad)
