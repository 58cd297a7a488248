"""Pins for the oracle's Schur complement matrix (eq. SCM) and SCE right-hand
side.

Independent facts used:
  * Kronecker identity B = Avec^T (Y^{-1} kron X) Avec (brute force, tiny n);
  * literal trace definition tr(A_p X A_q Y^{-1}) with dense matrices;
  * iteration 0 (X = Y = lambda I): B_pq = A_p . A_q (Gram matrix), which is
    I for max-cut and has closed-form entries for norm minimisation;
  * max-cut: B = X o Y^{-1} (Hadamard product, A_k = e_k e_k^T);
  * central point X = mu Y^{-1}: B_pq = mu A_p . (Y^{-1} A_q Y^{-1});
  * B symmetric positive definite for independent A_k;
  * the direction built from g satisfies the linearised equations
    A_k . dX = b_k - A_k . X and dY + sum dz_k A_k = G, and
    dX~ Y + X dY = beta mu I - X Y (the HKM linearisation).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import sdpgen
from oracle.scm import dense_scm, problem_mats, scm_kron, scm_rhs


def _rand_state(n, rng):
    return sdpgen.random_pd_dense(n, rng, 5.0), sdpgen.random_pd_dense(n, rng, 5.0)


@pytest.mark.parametrize("seed", range(4))
def test_scm_kron_and_trace(seed):
    rng = np.random.default_rng(seed)
    prob = sdpgen.random_sparse_sdp(7, 5, seed=seed)
    A = problem_mats(prob)
    X, Y = _rand_state(prob.n, rng)
    Yi = np.linalg.inv(Y)
    B = dense_scm(A, X, Yi)
    Ad = [prob.dense(k) for k in range(1, prob.m + 1)]
    Bk = scm_kron(Ad, X, Yi)
    Bt = np.array([[np.trace(ap @ X @ aq @ Yi) for aq in Ad] for ap in Ad])
    assert np.allclose(B, Bk, rtol=1e-12, atol=1e-12)
    assert np.allclose(B, Bt, rtol=1e-12, atol=1e-12)
    assert np.allclose(B, B.T, rtol=1e-12, atol=1e-13)
    assert np.linalg.eigvalsh(B)[0] > 0


def test_scm_iteration0_gram():
    lam = 100.0
    prob = sdpgen.normmin(p=30, q=4, ny=5, seed=0)
    A = problem_mats(prob)
    n = prob.n
    B = dense_scm(A, lam * np.eye(n), np.eye(n) / lam)
    F = prob.meta["F"]
    # B_tt = n, B_{t,y_i} = 0, B_{y_i,y_j} = 2 <F_i, F_j>
    assert np.isclose(B[0, 0], n, rtol=1e-14)
    assert np.allclose(B[0, 1:], 0.0, atol=1e-14)
    G = 2.0 * np.einsum("iab,jab->ij", F[1:], F[1:])
    assert np.allclose(B[1:, 1:], G, rtol=1e-13, atol=1e-15)
    mc = sdpgen.maxcut_cycle_chords(20, 0)
    Bm = dense_scm(problem_mats(mc), lam * np.eye(20), np.eye(20) / lam)
    assert np.allclose(Bm, np.eye(20), rtol=1e-14, atol=0)


def test_scm_maxcut_hadamard():
    rng = np.random.default_rng(2)
    prob = sdpgen.maxcut_cycle_chords(24, 1)
    X, Y = _rand_state(24, rng)
    Yi = np.linalg.inv(Y)
    B = dense_scm(problem_mats(prob), X, Yi)
    assert np.allclose(B, X * Yi.T, rtol=1e-13, atol=1e-15)


def test_scm_central_point():
    rng = np.random.default_rng(4)
    prob = sdpgen.random_sparse_sdp(9, 6, seed=3)
    A = problem_mats(prob)
    _, Y = _rand_state(9, rng)
    Yi = np.linalg.inv(Y)
    mu = 0.25
    B = dense_scm(A, mu * Yi, Yi)
    Ad = [prob.dense(k) for k in range(1, prob.m + 1)]
    expect = np.array([[mu * np.sum(ap * (Yi @ aq @ Yi)) for aq in Ad] for ap in Ad])
    assert np.allclose(B, expect, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_rhs_linearised_equations(seed):
    rng = np.random.default_rng(seed)
    prob = sdpgen.random_sparse_sdp(8, 5, seed=10 + seed)
    A = problem_mats(prob)
    Ad = [prob.dense(k) for k in range(prob.m + 1)]
    n, m = prob.n, prob.m
    X, Y = _rand_state(n, rng)
    z = rng.standard_normal(m)
    Yi = np.linalg.inv(Y)
    G = Ad[0] - sum(zk * a for zk, a in zip(z, Ad[1:])) - Y
    mu = np.sum(X * Y) / n
    beta = 0.3
    B = dense_scm(A, X, Yi)
    g = scm_rhs(A, prob.b, X, Yi, G, beta, mu)
    dz = np.linalg.solve(B, g)
    dY = G - sum(d * a for d, a in zip(dz, Ad[1:]))
    dXt = beta * mu * Yi - X - X @ dY @ Yi
    dX = (dXt + dXt.T) / 2
    lhs = np.array([np.sum(a * dX) for a in Ad[1:]])
    rhs = prob.b - np.array([np.sum(a * X) for a in Ad[1:]])
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-10)
    assert np.allclose(dY + sum(d * a for d, a in zip(dz, Ad[1:])), G, atol=1e-12)
    assert np.allclose(dXt @ Y + X @ dY, beta * mu * np.eye(n) - X @ Y, rtol=1e-10, atol=1e-9)
    # a wrong sign on the G term must break the linearised primal equations
    g_bad = scm_rhs(A, prob.b, X, Yi, -G, beta, mu)
    dz_b = np.linalg.solve(B, g_bad)
    dY_b = G - sum(d * a for d, a in zip(dz_b, Ad[1:]))
    dX_b = beta * mu * Yi - X - X @ dY_b @ Yi
    lhs_b = np.array([np.sum(a * (dX_b + dX_b.T) / 2) for a in Ad[1:]])
    assert not np.allclose(lhs_b, rhs, rtol=1e-6, atol=1e-6)
