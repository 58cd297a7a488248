"""Oracle: Schur complement matrix and the right-hand side of the SCE.

dense_scm  eq. SCM: B_qp = (X A_q Y^{-1}) . A_p; B is symmetric, so column q
           is B_pq = sum over (a,b) in supp A_p of [A_p]_ab (X A_q Y^{-1})_ab.
           For each q, P_q = X[:, R_q] A_q[R_q, K_q] (R_q / K_q are the
           nonzero rows / columns of A_q) and (X A_q Y^{-1})_ab =
           P_q[a, :] . Y^{-1}[K_q, b] is evaluated only on the union support
           of A_1..A_m.  B is exactly the matrix eq. SCM defines; nothing is
           dropped, only zero products are skipped.
scm_kron   The same matrix through the identity
           vec(X A Y^{-1}) = (Y^{-1} kron X) vec(A) (X, Y symmetric):
           B = Avec^T (Y^{-1} kron X) Avec.  Tiny n only; used as a pin.
scm_rhs    Right-hand side g of the SCE (eq. SCE).  The printed g_k and G
           are garbled (no primal residual, and G lacks -Y).  Reading used:
               G   = A_0 - sum_k z_k A_k - Y            (dual residual)
               g_k = (b_k - A_k . X) - A_k . (beta mu Y^{-1} - X - X G Y^{-1})
                   =  b_k - beta mu A_k . Y^{-1} + A_k . (X G Y^{-1}),
           the unique g for which dY = G - sum dz_k A_k and the eq. dX
           direction satisfy A_k . dX = b_k - A_k . X.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .symbolic import sym_sparse


def _union_support(mats):
    acc = None
    for a in mats:
        s = (a != 0).astype(np.int8)
        acc = s if acc is None else acc + s
    acc = sp.coo_matrix(acc)
    return acc.row.astype(np.int64), acc.col.astype(np.int64)


def dense_scm(A, Xhat: np.ndarray, Yinv: np.ndarray, chunk: int = 4096, cols=None) -> np.ndarray:
    """A: list of full symmetric scipy matrices A_0..A_m (A[0] unused).  cols: if
    given, only these columns q (0-based) of B are evaluated; the others stay 0."""
    m = len(A) - 1
    n = Xhat.shape[0]
    Ak = A[1:]
    Sa, Sb = _union_support(Ak)
    # Amat[p, s] = [A_p]_{Sa[s], Sb[s]}
    Amat = sp.vstack([sp.csr_matrix(a[Sa, Sb]) for a in Ak]).tocsr()
    B = np.zeros((m, m))
    for q, a in enumerate(Ak):
        if cols is not None and q not in cols:
            continue
        a = sp.csc_matrix(a)
        Kq = np.nonzero(np.diff(a.indptr))[0]
        Rq = np.unique(a.indices)
        if len(Kq) == 0:
            continue
        sub = a[Rq][:, Kq]                              # |R_q| x |K_q|
        Pq = np.asarray((sub.T @ Xhat[Rq, :]).T)        # = X[:, R_q] A_q[R_q, K_q]
        if len(Sa) > 8 * n:
            # many support entries: form X A_q Y^{-1} whole, then read it on S
            T = (Pq @ Yinv[Kq, :])[Sa, Sb]
        else:
            T = np.empty(len(Sa))
            for s0 in range(0, len(Sa), chunk):
                ia = Sa[s0:s0 + chunk]
                ib = Sb[s0:s0 + chunk]
                T[s0:s0 + chunk] = np.einsum("ij,ji->i", Pq[ia, :], Yinv[np.ix_(Kq, ib)])
        B[:, q] = Amat @ T
    return B


def scm_kron(A_dense, X: np.ndarray, Yinv: np.ndarray) -> np.ndarray:
    """A_dense: list of dense symmetric A_1..A_m."""
    Avec = np.stack([a.reshape(-1, order="F") for a in A_dense], axis=1)
    return Avec.T @ np.kron(Yinv, X) @ Avec


def scm_rhs(A, b, Xhat, Yinv, G, beta, mu) -> np.ndarray:
    M = Xhat @ G @ Yinv
    g = np.empty(len(A) - 1)
    for k in range(1, len(A)):
        a = sp.coo_matrix(A[k])
        g[k - 1] = (b[k - 1] - beta * mu * float(np.sum(a.data * Yinv[a.row, a.col]))
                    + float(np.sum(a.data * M[a.row, a.col])))
    return g


def problem_mats(prob):
    return [sym_sparse(prob, k) for k in range(prob.m + 1)]
