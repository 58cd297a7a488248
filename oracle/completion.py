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
algorithm1        Algorithm 1 (Steps 1-3): per clique, Cholesky factor M_r of
                  the block with reversed row/column order, L_r = P_r M_r^{-T}
                  P_r^T, first |S_r| columns of L_r into Lhat(C_r, S_r).
lhat_textbook     chol(inv(X^)), the definition Algorithm 1 must reproduce.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

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
    """Lhat with Lhat Lhat^T = X^{-1}, computed clique by clique (Algorithm 1).
    Returns a dense lower-triangular n x n matrix (zero outside E)."""
    n = ch.n
    Lhat = np.zeros((n, n))                                   # Step 1
    for r in range(ch.ell):                                    # Step 2
        C = ch.cliques[r]
        c = len(C)
        P = np.eye(c)[::-1]                                    # Step 2-1: [P]_ij = 1 iff i + j = c + 1
        M = np.linalg.cholesky(P @ Xbar[np.ix_(C, C)] @ P.T)   # Step 2-2
        Minv_T = sla.solve_triangular(M, np.eye(c), lower=True).T
        Lr = P @ Minv_T @ P.T                                  # Step 2-3
        k = int(ch.nS[r])
        Lhat[np.ix_(C, C[:k])] = Lr[:, :k]                     # Step 3
    return Lhat


def lhat_textbook(Xhat: np.ndarray) -> np.ndarray:
    return np.linalg.cholesky(np.linalg.inv(Xhat))
