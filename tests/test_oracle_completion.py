"""Pins for the oracle's max-determinant completion and Algorithm 1.

What fixes them, independently of the code under test:
  * the completion agrees with the given entries on E, is positive definite,
    and its inverse vanishes off E (the characterisation in Section 3.1);
  * brute force: det X^ is a local maximum over the free entries;
  * a different clique sequence (one clique per vertex) gives the same matrix;
  * Algorithm 1 reproduces chol(inv(X^)) (textbook definition), and the
    closed forms of the validity proof (Section 3.1): the block form of Lhat
    from M (first clique) and N (second clique), and the explicit inverse;
  * special cases: one clique (Lhat = chol(X^{-1})), diagonal E
    (Lhat = diag(X_ii^{-1/2})), the central point X = mu Y^{-1} on E
    (Lhat = N / sqrt(mu) with Y = N N^T).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import sdpgen
from oracle.completion import algorithm1, completion_by_vertex, lhat_textbook, maxdet_complete
from oracle.symbolic import aggregate_pattern, chordal_structure


def _random_case(seed, n=16, p=0.2):
    rng = np.random.default_rng(seed)
    e = sdpgen.random_graph(n, p, rng)
    prob = sdpgen.maxcut(n, e, np.ones(len(e)))
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(n, rows, cols, rng.permutation(n))
    Xfull = sdpgen.random_pd_dense(n, rng, cond=20.0)
    Xbar = np.where(ch.E_mask(), Xfull, 0.0)
    return ch, Xbar, rng


@pytest.mark.parametrize("seed", range(5))
def test_completion_characterisation(seed):
    ch, Xbar, _ = _random_case(seed)
    E = ch.E_mask()
    Xh = maxdet_complete(ch, Xbar)
    assert np.allclose(Xh, Xh.T, atol=0)
    assert np.array_equal(Xh[E], Xbar[E])
    assert np.linalg.eigvalsh(Xh)[0] > 0
    Xi = np.linalg.inv(Xh)
    assert np.abs(Xi[~E]).max() <= 1e-10 * np.abs(Xi).max()
    Xv = completion_by_vertex(ch, Xbar)
    assert np.allclose(Xv, Xh, rtol=1e-11, atol=1e-11)


def test_completion_is_det_maximal():
    ch, Xbar, rng = _random_case(11, n=10, p=0.25)
    E = ch.E_mask()
    Xh = maxdet_complete(ch, Xbar)
    ld0 = np.linalg.slogdet(Xh)[1]
    free = np.argwhere(np.triu(~E, 1))
    assert len(free) > 0
    for _ in range(200):
        D = np.zeros_like(Xh)
        d = rng.standard_normal(len(free)) * 1e-3
        D[free[:, 0], free[:, 1]] = d
        D = D + D.T
        s, ld = np.linalg.slogdet(Xh + D)
        assert s > 0 and ld < ld0


def test_two_clique_closed_form():
    # X = [[X_SS X_SU ?], [X_US X_UU X_UT], [? X_TU X_TT]]; the unknown block
    # is X_SU X_UU^{-1} X_UT (Section 3.1, validity proof)
    rng = np.random.default_rng(5)
    s, u, t = 3, 2, 4
    n = s + u + t
    Xfull = sdpgen.random_pd_dense(n, rng, cond=8.0)
    S, U, T = np.arange(s), np.arange(s, s + u), np.arange(s + u, n)
    rows, cols = np.tril_indices(n)
    keep = ~(np.isin(rows, T) & np.isin(cols, S))
    ch = chordal_structure(n, rows[keep], cols[keep])
    assert ch.ell >= 2
    Xbar = np.where(ch.E_mask(), Xfull, 0.0)
    Xh = maxdet_complete(ch, Xbar)
    expect = Xfull[np.ix_(S, U)] @ np.linalg.solve(Xfull[np.ix_(U, U)], Xfull[np.ix_(U, T)])
    assert np.allclose(Xh[np.ix_(S, T)], expect, rtol=1e-12, atol=1e-13)
    # block form of Lhat (eq. widehatL) and its explicit inverse
    C1 = np.concatenate([S, U])
    C2 = np.concatenate([U, T])
    Mfull = np.linalg.cholesky(np.linalg.inv(Xfull[np.ix_(C1, C1)]))
    Nfull = np.linalg.cholesky(np.linalg.inv(Xfull[np.ix_(C2, C2)]))
    M_SS, M_US = Mfull[:s, :s], Mfull[s:, :s]
    N_UU, N_TU, N_TT = Nfull[:u, :u], Nfull[u:, :u], Nfull[u:, u:]
    L = np.zeros((n, n))
    L[np.ix_(S, S)] = M_SS
    L[np.ix_(U, S)] = M_US
    L[np.ix_(U, U)] = N_UU
    L[np.ix_(T, U)] = N_TU
    L[np.ix_(T, T)] = N_TT
    Lh = algorithm1(ch, Xbar)
    assert np.allclose(Lh, L, rtol=1e-12, atol=1e-13)
    inv = lambda a: np.linalg.inv(a)
    Li = np.zeros((n, n))
    Li[np.ix_(S, S)] = inv(M_SS)
    Li[np.ix_(U, S)] = -inv(N_UU) @ M_US @ inv(M_SS)
    Li[np.ix_(U, U)] = inv(N_UU)
    Li[np.ix_(T, S)] = inv(N_TT) @ N_TU @ inv(N_UU) @ M_US @ inv(M_SS)
    Li[np.ix_(T, U)] = -inv(N_TT) @ N_TU @ inv(N_UU)
    Li[np.ix_(T, T)] = inv(N_TT)
    assert np.allclose(np.linalg.inv(Lh), Li, rtol=1e-11, atol=1e-12)
    assert np.allclose(Li.T @ Li, Xh, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_algorithm1_matches_textbook(seed):
    ch, Xbar, _ = _random_case(100 + seed, n=18)
    Xh = maxdet_complete(ch, Xbar)
    Lh = algorithm1(ch, Xbar)
    assert np.allclose(Lh, lhat_textbook(Xh), rtol=1e-10, atol=1e-12)
    assert np.array_equal(Lh != 0, np.tril(ch.E_mask()) & (Lh != 0))
    assert np.allclose(Lh.T @ Xh @ Lh, np.eye(ch.n), atol=1e-10)


def test_algorithm1_single_clique_and_diagonal():
    rng = np.random.default_rng(3)
    n = 7
    X = sdpgen.random_pd_dense(n, rng)
    rows, cols = np.tril_indices(n)
    ch = chordal_structure(n, rows, cols)
    assert ch.ell == 1
    assert np.allclose(algorithm1(ch, X), np.linalg.cholesky(np.linalg.inv(X)), rtol=1e-12)
    chd = chordal_structure(n, np.arange(n), np.arange(n))
    Xd = np.where(np.eye(n, dtype=bool), X, 0.0)
    assert np.allclose(algorithm1(chd, Xd), np.diag(np.diag(X) ** -0.5), rtol=1e-15)


def test_algorithm1_central_point():
    # X = mu Y^{-1} on E with Y supported on the aggregate pattern: the
    # completion is mu Y^{-1} itself, so Lhat = N / sqrt(mu)
    rng = np.random.default_rng(9)
    n = 40
    prob = sdpgen.maxcut_band(n, bw=4, p=0.6, seed=4)
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(n, rows, cols)
    Y = sdpgen.random_pd_on_pattern(n, rows, cols, rng)
    mu = 0.37
    Xbar = np.where(ch.E_mask(), mu * np.linalg.inv(Y), 0.0)
    Lh = algorithm1(ch, Xbar)
    N = np.linalg.cholesky(Y)
    assert np.allclose(Lh, N / np.sqrt(mu), rtol=1e-10, atol=1e-12)
    assert np.allclose(maxdet_complete(ch, Xbar), mu * np.linalg.inv(Y), rtol=1e-10, atol=1e-12)


# ------------------------------------------------ the earlier factorisation X^ = L^T D L
# Pins of sparse_factors (Section 2.1, eqs. sparse_fact, orig_L, orig_D): its product must
# be the max-determinant completion, which maxdet_complete reaches by a different formula
# (the two-clique completion of the validity proof); L^{-1} keeps the sparsity of E (the
# property the earlier solver's substitutions rely on); a three-vertex path worked by hand.
@pytest.mark.parametrize("seed", range(5))
def test_sparse_factors_reproduce_completion(seed):
    from oracle.completion import sparse_factors
    ch, Xbar, _ = _random_case(seed)
    L, D = sparse_factors(ch, Xbar)
    Xh = maxdet_complete(ch, Xbar)
    assert np.abs(L.T @ D @ L - Xh).max() <= 1e-10 * np.abs(Xh).max()
    assert np.array_equal(np.triu(L, 1), np.zeros_like(L)) and np.array_equal(np.diag(L), np.ones(ch.n))
    Li = np.linalg.inv(L)
    E = ch.E_mask()
    assert np.abs(Li[~E]).max() <= 1e-12 * np.abs(Li).max()
    # D is block diagonal over the supernodes S_r and positive definite
    for r, C in enumerate(ch.cliques):
        S = C[:int(ch.nS[r])]
        others = np.setdiff1d(np.arange(ch.n), S)
        assert np.abs(D[np.ix_(S, others)]).max(initial=0.0) == 0.0
        assert np.linalg.eigvalsh(D[np.ix_(S, S)])[0] > 0
    # and its inverse is Lhat Lhat^T of Algorithm 1
    Lh = algorithm1(ch, Xbar)
    assert np.abs(Li @ np.linalg.inv(D) @ Li.T - Lh @ Lh.T).max() <= 1e-10 * np.abs(Lh @ Lh.T).max()


def test_sparse_factors_three_vertex_path_by_hand():
    from oracle.completion import sparse_factors
    # path 0 - 1 - 2: cliques {0, 1} (S = {0}, U = {1}) and {1, 2} (S = {1, 2})
    ch = chordal_structure(3, np.array([0, 1, 1, 2, 2]), np.array([0, 0, 1, 1, 2]))
    assert [list(C) for C in ch.cliques] == [[0, 1], [1, 2]] and list(ch.nS) == [1, 2]
    x11, x21, x22, x32, x33 = 3.0, 1.0, 2.0, -0.5, 4.0
    Xbar = np.array([[x11, x21, 0.0], [x21, x22, x32], [0.0, x32, x33]])
    L, D = sparse_factors(ch, Xbar)
    assert np.allclose(L, [[1, 0, 0], [x21 / x22, 1, 0], [0, 0, 1]], rtol=0, atol=1e-15)
    assert np.allclose(D, [[x11 - x21 ** 2 / x22, 0, 0], [0, x22, x32], [0, x32, x33]], rtol=0, atol=1e-15)
    Xh = L.T @ D @ L
    assert abs(Xh[2, 0] - x32 * x21 / x22) <= 1e-15   # the classic max-det fill of a path
    assert np.allclose(Xh[np.triu_indices(3)][[0, 1, 3, 4, 5]], [x11, x21, x22, x32, x33], atol=1e-15)
