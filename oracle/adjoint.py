"""Oracle: derivatives of a central solution (test infrastructure only).

The paper does not differentiate its solution; these routines fix what the
library's adjoint must compute, in plain dense FP64.

For fixed mu > 0 the point of the central path of Section 2.2,
    A(X) = b,   sum_k z_k A_k + Y = A_0,   X = mu Y^{-1},
is a smooth function of (b, A_0).  Differentiating the three equations gives
dY = dA_0 - sum_k dz_k A_k and dX = -X dY Y^{-1} (with X = mu Y^{-1}), and
A(dX) = db then reads B dz = db + h(dA_0) with the Schur complement matrix
B_pq = A_p . (X A_q Y^{-1}) of eq. SCM and h_p(M) = A_p . (X M Y^{-1}).  For a
loss L(X, z) with gradients G_L (w.r.t. X) and v (w.r.t. z), back-substitution
through that system gives
    lambda  = B^{-1} (h(G_L) + v)
    dL/db   = lambda
    dL/dA_0 = sym(X (sum_k lambda_k A_k - G_L) Y^{-1})
(dL = <dL/dA_0, dA_0> in the Frobenius product of symmetric matrices).

center   Newton steps of Step 2 of Section 2.2 with the centring target beta mu
         replaced by a fixed mu: full steps while X + dX and Y + dY stay
         positive definite, otherwise the usual gamma times the longest step.
adjoint  the formulas above, dense.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .pdipm import Params, _Ops, _inv_spd, dense_state_metrics, step_length_dense
from .scm import dense_scm, problem_mats, scm_rhs


def center(prob, X, Y, z, mu, steps=60, tol=1e-14, params: Params = Params()):
    """Dense Newton steps toward the mu-central point from (X, Y, z); returns the
    new (X, Y, z) and the last relative step of z."""
    A = problem_mats(prob)
    ops = _Ops(A)
    n, b = prob.n, prob.b
    X, Y, z = X.copy(), Y.copy(), z.copy()
    rel = np.inf
    for _ in range(steps):
        st = dense_state_metrics(ops, b, X, Y, z)
        Yinv = _inv_spd(Y)
        B = dense_scm(A, X, Yinv)
        g = scm_rhs(A, b, X, Yinv, st["G"], 1.0, mu)
        dz = sla.cho_solve(sla.cho_factor(B, lower=True), g)
        dY = st["G"] - ops.combine(dz, n)
        dXt = mu * Yinv - X - X @ dY @ Yinv
        dX = (dXt + dXt.T) / 2.0
        ap = step_length_dense(X, dX)
        ad = step_length_dense(Y, dY)
        sp_ = 1.0 if ap >= 1.0 else params.gamma * ap
        sd_ = 1.0 if ad >= 1.0 else params.gamma * ad
        X = X + sp_ * dX
        Y = Y + sd_ * dY
        z = z + sd_ * dz
        rel = float(np.abs(sd_ * dz).max() / max(1.0, np.abs(z).max()))
        if rel <= tol:
            break
    return X, Y, z, rel


def adjoint(prob, X, Y, z, GL, dLdz):
    """(dL/db, dL/dA_0) at a central point (X, Y, z) for the loss gradients GL
    (symmetric n x n, w.r.t. X) and dLdz (length m)."""
    A = problem_mats(prob)
    ops = _Ops(A)
    n = prob.n
    Yinv = _inv_spd(Y)
    B = dense_scm(A, X, Yinv)
    T = X @ GL @ Yinv
    h = np.array([float(A[k].multiply(T).sum()) for k in range(1, prob.m + 1)])
    lam = sla.cho_solve(sla.cho_factor(B, lower=True), h + dLdz)
    M = ops.combine(lam, n) - GL
    Gam = X @ M @ Yinv
    return lam, (Gam + Gam.T) / 2.0
