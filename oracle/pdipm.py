"""Oracle primal-dual interior-point methods (dense HKM, and its matrix-
completion variant).

Section 2.2, basic framework:
  Step 0  X = Y = lambda0 I, z = 0; 0 < beta, gamma < 1.
  Step 1  stop when the (relative) gap and both infeasibilities are small.
  Step 2  HKM direction: B dz = g (eq. SCE), dY = G - sum dz_k A_k,
          dX~ = beta mu Y^{-1} - X - X dY Y^{-1}, dX = (dX~ + dX~^T)/2 (eq. dX).
  Step 3  alpha = max{alpha in (0,1] : X + alpha dX psd}, likewise for Y
          (eq. primal_length).
  Step 4  X += gamma alpha_p dX, Y += gamma alpha_d dY, z += gamma alpha_d dz.

Readings where the paper is silent or garbled (one choice, used by the GPU
library as well):
  * G = A_0 - sum z_k A_k - Y and g as in scm.scm_rhs (the printed G and g
    are garbled);
  * lambda0 = 100, beta = 0.1 once both infeasibilities are <= feas_tol and
    0.2 before, gamma = 0.9, at most 100 iterations;
  * pobj = A_0 . X, dobj = b . z, relgap = |pobj - dobj| / max(1, (|pobj| +
    |dobj|)/2), pinf = max_k |b_k - A_k . X| / (1 + max_k |b_k|),
    dinf = max_ij |G_ij| / (1 + max_ij |[A_0]_ij|); stop when all three are
    <= their tolerances;
  * the largest step is found from the smallest eigenvalue of
    R^{-1} dX R^{-T} with X = R R^T: alpha = min(1, -1/lambda_min) when
    lambda_min < 0, else 1.

mc_pdipm keeps X only on the extended pattern E (as the matrix-completion
method does): X^ is the max-determinant completion of that partial matrix,
the direction is eq. dX with X^ in place of X (eq. newdX2 evaluates the same
columns through Lhat and N), dX is kept on E only, and alpha_p is taken
clique by clique (eq. primal_length2).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .completion import maxdet_complete
from .scm import dense_scm, problem_mats, scm_rhs
from .symbolic import Chordal, aggregate_pattern, chordal_structure


@dataclasses.dataclass
class Params:
    gap_tol: float = 1e-7
    feas_tol: float = 1e-7
    beta_feas: float = 0.1
    beta_infeas: float = 0.2
    gamma: float = 0.9
    lambda0: float = 100.0
    max_iter: int = 100


class _Ops:
    """Vectorised A(X) and sum_k z_k A_k over all constraint triplets."""

    def __init__(self, A):
        self.A = A
        self.m = len(A) - 1
        rows, cols, vals, ks = [], [], [], []
        for k in range(1, len(A)):
            a = sp.coo_matrix(A[k])
            rows.append(a.row)
            cols.append(a.col)
            vals.append(a.data)
            ks.append(np.full(len(a.data), k - 1))
        self.r = np.concatenate(rows)
        self.c = np.concatenate(cols)
        self.v = np.concatenate(vals)
        self.k = np.concatenate(ks)
        self.A0 = A[0].toarray()
        self.A0max = float(np.abs(self.A0).max()) if self.A0.size else 0.0

    def apply(self, X):                      # [A_k . X]_k
        return np.bincount(self.k, weights=self.v * X[self.r, self.c], minlength=self.m)

    def combine(self, y, n):                 # sum_k y_k A_k, dense
        out = np.zeros((n, n))
        np.add.at(out, (self.r, self.c), self.v * y[self.k])
        return out


def dense_state_metrics(ops: _Ops, b, X, Y, z):
    n = X.shape[0]
    pobj = float(np.sum(ops.A0 * X))
    dobj = float(b @ z)
    r = b - ops.apply(X)
    G = ops.A0 - ops.combine(z, n) - Y
    relgap = abs(pobj - dobj) / max(1.0, (abs(pobj) + abs(dobj)) / 2.0)
    pinf = float(np.abs(r).max()) / (1.0 + float(np.abs(b).max())) if len(b) else 0.0
    dinf = float(np.abs(G).max()) / (1.0 + ops.A0max)
    return dict(pobj=pobj, dobj=dobj, relgap=relgap, pinf=pinf, dinf=dinf, G=G, r=r)


def _alpha_from_lmin(lmin: float) -> float:
    return 1.0 if lmin >= -1.0 else -1.0 / lmin


def step_length_dense(X: np.ndarray, dX: np.ndarray) -> float:
    R = np.linalg.cholesky(X)
    W = sla.solve_triangular(R, dX, lower=True)
    M = sla.solve_triangular(R, W.T, lower=True)
    M = (M + M.T) / 2.0
    lmin = float(sla.eigh(M, eigvals_only=True, subset_by_index=[0, 0])[0])
    return _alpha_from_lmin(lmin)


def step_length_cliques(ch: Chordal, Xbar: np.ndarray, dX: np.ndarray):
    """eq. primal_length2: min over cliques of the largest step keeping the
    clique block psd.  Returns (alpha, per-clique alphas)."""
    al = np.empty(ch.ell)
    for r, C in enumerate(ch.cliques):
        ix = np.ix_(C, C)
        R = np.linalg.cholesky(Xbar[ix])
        W = sla.solve_triangular(R, dX[ix], lower=True)
        M = sla.solve_triangular(R, W.T, lower=True)
        lmin = float(np.linalg.eigvalsh((M + M.T) / 2.0)[0])
        al[r] = _alpha_from_lmin(lmin)
    return float(al.min()) if len(al) else 1.0, al


def _inv_spd(Y):
    c = sla.cho_factor(Y, lower=True)
    return sla.cho_solve(c, np.eye(Y.shape[0]))


def dense_pdipm(prob, params: Params = Params(), verbose: bool = False, max_iter=None):
    n, m = prob.n, prob.m
    A = problem_mats(prob)
    ops = _Ops(A)
    b = prob.b
    X = params.lambda0 * np.eye(n)
    Y = params.lambda0 * np.eye(n)
    z = np.zeros(m)
    hist = []
    status = "maxiter"
    limit = params.max_iter if max_iter is None else max_iter
    it = 0
    t_all = time.perf_counter()
    for it in range(limit + 1):
        t0 = time.perf_counter()
        st = dense_state_metrics(ops, b, X, Y, z)
        rec = dict(it=it, pobj=st["pobj"], dobj=st["dobj"], relgap=st["relgap"],
                   pinf=st["pinf"], dinf=st["dinf"])
        if st["relgap"] <= params.gap_tol and st["pinf"] <= params.feas_tol \
                and st["dinf"] <= params.feas_tol:
            status = "optimal"
            hist.append(rec)
            break
        if it == limit:
            hist.append(rec)
            break
        mu = float(np.sum(X * Y)) / n
        feas = st["pinf"] <= params.feas_tol and st["dinf"] <= params.feas_tol
        beta = params.beta_feas if feas else params.beta_infeas
        t1 = time.perf_counter()
        Yinv = _inv_spd(Y)
        B = dense_scm(A, X, Yinv)
        cB = sla.cho_factor(B, lower=True)
        t2 = time.perf_counter()
        g = scm_rhs(A, b, X, Yinv, st["G"], beta, mu)
        dz = sla.cho_solve(cB, g)
        dY = st["G"] - ops.combine(dz, n)
        dXt = beta * mu * Yinv - X - X @ dY @ Yinv
        dX = (dXt + dXt.T) / 2.0
        ap = step_length_dense(X, dX)
        ad = step_length_dense(Y, dY)
        X = X + params.gamma * ap * dX
        Y = Y + params.gamma * ad * dY
        z = z + params.gamma * ad * dz
        t3 = time.perf_counter()
        rec.update(mu=mu, beta=beta, alpha_p=ap, alpha_d=ad, t_scm=t2 - t1, t_iter=t3 - t0)
        hist.append(rec)
        if verbose:
            print({k: (round(v, 10) if isinstance(v, float) else v) for k, v in rec.items()},
                  flush=True)
    st = dense_state_metrics(ops, b, X, Y, z)
    return dict(status=status, iters=it, X=X, Y=Y, z=z, pobj=st["pobj"], dobj=st["dobj"],
                relgap=st["relgap"], pinf=st["pinf"], dinf=st["dinf"], history=hist,
                seconds=time.perf_counter() - t_all)


# --------------------------------------------------------------------------
# matrix-completion variant (X known on E only)
# --------------------------------------------------------------------------

def permuted_mats(prob, ch: Chordal):
    P = sp.csr_matrix((np.ones(prob.n), (np.arange(prob.n), ch.order)), shape=(prob.n, prob.n))
    return [sp.csr_matrix(P @ a @ P.T) for a in problem_mats(prob)]


def mc_direction(ch: Chordal, A, b, Xbar, Y, z, params: Params = Params()):
    """One Step 2 + Step 3 of the matrix-completion method at (Xbar on E, Y, z),
    all in the permuted index space.  Returns the direction, the step lengths
    and the intermediate quantities."""
    ops = _Ops(A)
    n = ch.n
    Emask = ch.E_mask()
    st = dense_state_metrics(ops, b, Xbar, Y, z)
    mu = float(np.sum(Xbar * Y)) / n
    feas = st["pinf"] <= params.feas_tol and st["dinf"] <= params.feas_tol
    beta = params.beta_feas if feas else params.beta_infeas
    Xhat = maxdet_complete(ch, Xbar)
    Yinv = _inv_spd(Y)
    B = dense_scm(A, Xhat, Yinv)
    g = scm_rhs(A, b, Xhat, Yinv, st["G"], beta, mu)
    dz = sla.cho_solve(sla.cho_factor(B, lower=True), g)
    dY = st["G"] - ops.combine(dz, n)
    dXt = beta * mu * Yinv - Xhat - Xhat @ dY @ Yinv
    dX = np.where(Emask, (dXt + dXt.T) / 2.0, 0.0)
    ap, _ = step_length_cliques(ch, Xbar, dX)
    ad = step_length_dense(Y, dY)
    return dict(Xhat=Xhat, Yinv=Yinv, B=B, g=g, dz=dz, dY=dY, dX=dX, alpha_p=ap,
                alpha_d=ad, mu=mu, beta=beta, metrics=st)


def mc_pdipm(prob, params: Params = Params(), order=None, verbose: bool = False,
             max_iter=None):
    """Matrix-completion PDIPM.  Returns the state in ORIGINAL indices: Xbar
    (zero off E), its completion, Y, z."""
    rows, cols = aggregate_pattern(prob)
    ch = chordal_structure(prob.n, rows, cols, order)
    A = permuted_mats(prob, ch)
    ops = _Ops(A)
    n, m, b = prob.n, prob.m, prob.b
    Xbar = params.lambda0 * np.eye(n)
    Y = params.lambda0 * np.eye(n)
    z = np.zeros(m)
    hist = []
    status = "maxiter"
    limit = params.max_iter if max_iter is None else max_iter
    it = 0
    for it in range(limit + 1):
        st = dense_state_metrics(ops, b, Xbar, Y, z)
        rec = dict(it=it, pobj=st["pobj"], dobj=st["dobj"], relgap=st["relgap"],
                   pinf=st["pinf"], dinf=st["dinf"])
        hist.append(rec)
        if st["relgap"] <= params.gap_tol and st["pinf"] <= params.feas_tol \
                and st["dinf"] <= params.feas_tol:
            status = "optimal"
            break
        if it == limit:
            break
        d = mc_direction(ch, A, b, Xbar, Y, z, params)
        rec.update(mu=d["mu"], beta=d["beta"], alpha_p=d["alpha_p"], alpha_d=d["alpha_d"])
        Xbar = Xbar + params.gamma * d["alpha_p"] * d["dX"]
        Y = Y + params.gamma * d["alpha_d"] * d["dY"]
        z = z + params.gamma * d["alpha_d"] * d["dz"]
        if verbose:
            print(rec, flush=True)
    st = dense_state_metrics(ops, b, Xbar, Y, z)
    Xhat = maxdet_complete(ch, Xbar)
    return dict(status=status, iters=it, Xbar=ch.unpermute(Xbar), Xhat=ch.unpermute(Xhat),
                Y=ch.unpermute(Y), z=z, pobj=st["pobj"], dobj=st["dobj"],
                relgap=st["relgap"], pinf=st["pinf"], dinf=st["dinf"], history=hist,
                chordal=ch)
