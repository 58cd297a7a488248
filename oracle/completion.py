"""Oracle: max-determinant completion and Algorithm 1.

All matrices are dense n x n in the permuted index space of a Chordal
structure; only entries on the extended pattern E of the partial matrix
Xbar are read.

maxdet_complete   Section 3.1, validity proof of Algorithm 1: for two cliques
                  S+U and U+T the max-determinant completion fills the
                  unknown block with X_SU X_UU^{-1} X_UT.  Applied along the
                  clique sequence from the last clique back to the first, the
                  union of the later cliques plays the role of U+T (the
                  running-intersection induction the proof refers to).
completion_by_vertex
                  The same with one clique per vertex, {j} + struct(j); a
                  different clique sequence that must give the same matrix.
algorithm1        Lhat of Algorithm 1 (Section 3.1): on the rows C_r, the
                  columns S_r of Lhat are the leading |S_r| columns of the
                  lower-triangular Cholesky factor of (Xbar(C_r, C_r))^{-1}.
                  Algorithm 1 reaches that factor without an inverse, from a
                  factorisation of the block in reversed order; here the
                  inverse of the clique block is formed and factorised
                  directly, so the two share no arithmetic.
lhat_textbook     chol(inv(X^)), the definition Algorithm 1 must reproduce.
sparse_factors    the earlier factorisation X^ = L^T D L (Section 2.1,
                  eqs. sparse_fact, orig_L and orig_D): one elementary lower
                  factor L_r per clique with X_UU^{-1} X_US in rows U_r,
                  columns S_r; L = L_{l-1} ... L_1 multiplied out densely; D the
                  block diagonal of the Schur complements X_SS - X_SU X_UU^{-1}
                  X_US (X_SS itself for the last clique).
"""
from __future__ import annotations

import numpy as np

from .symbolic import Chordal


def _complete(n, blocks, Xbar):
    Xh = np.zeros((n, n))
    done = np.zeros(n, dtype=bool)
    for C, k in reversed(blocks):
        S, U = C[:k], C[k:]
        Xh[np.ix_(C, C)] = Xbar[np.ix_(C, C)]
        T = np.nonzero(done)[0]
        T = T[~np.isin(T, U)]
        if len(T) and len(U):
            W = Xbar[np.ix_(S, U)] @ np.linalg.solve(Xbar[np.ix_(U, U)], Xh[np.ix_(U, T)])
            Xh[np.ix_(S, T)] = W
            Xh[np.ix_(T, S)] = W.T
        done[C] = True
    return Xh


def maxdet_complete(ch: Chordal, Xbar: np.ndarray) -> np.ndarray:
    """Max-determinant positive definite completion X^ of Xbar (known on E)."""
    return _complete(ch.n, [(ch.cliques[r], int(ch.nS[r])) for r in range(ch.ell)], Xbar)


def completion_by_vertex(ch: Chordal, Xbar: np.ndarray) -> np.ndarray:
    return _complete(ch.n, [(ch.struct[j], 1) for j in range(ch.n)], Xbar)


def algorithm1(ch: Chordal, Xbar: np.ndarray) -> np.ndarray:
    """Lhat with Lhat Lhat^T = X^{-1}, clique by clique (Algorithm 1).
    Returns a dense lower-triangular n x n matrix (zero outside E)."""
    Lhat = np.zeros((ch.n, ch.n))
    for r, C in enumerate(ch.cliques):
        k = int(ch.nS[r])
        K = np.linalg.cholesky(np.linalg.inv(Xbar[np.ix_(C, C)]))   # K K^T = Xbar(C, C)^{-1}
        Lhat[np.ix_(C, C[:k])] = K[:, :k]
    return Lhat


def lhat_textbook(Xhat: np.ndarray) -> np.ndarray:
    return np.linalg.cholesky(np.linalg.inv(Xhat))


def sparse_factors(ch: Chordal, Xbar: np.ndarray):
    """(L, D) with X^ = L^T D L, from their definitions (Section 2.1)."""
    n = ch.n
    L = np.eye(n)
    D = np.zeros((n, n))
    for r, C in enumerate(ch.cliques):
        k = int(ch.nS[r])
        S, U = C[:k], C[k:]
        Lr = np.eye(n)
        if len(U):
            XUU = Xbar[np.ix_(U, U)]
            Lr[np.ix_(U, S)] = np.linalg.solve(XUU, Xbar[np.ix_(U, S)])
            D[np.ix_(S, S)] = Xbar[np.ix_(S, S)] - Xbar[np.ix_(S, U)] @ np.linalg.solve(XUU, Xbar[np.ix_(U, S)])
        else:
            D[np.ix_(S, S)] = Xbar[np.ix_(S, S)]
        L = Lr @ L   # L = L_r ... L_1 after clique r
    return L, D
