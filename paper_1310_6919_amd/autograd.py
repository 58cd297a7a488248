"""torch.autograd binding of the library's central-point solve and its adjoint.

CentralSDP.apply(a0, b, problem, mu) solves the SDP whose objective matrix A_0
has the lower-triangle triplet values `a0` (the triplet positions and A_1..A_m
are those of `problem`) and right-hand side `b`, centres the final iterate at
the mu-central point (sdpc_center), and returns (Xbar on E, z): the E-vector in
the library's storage order and the dual vector.  backward calls sdpc_adjoint.

Marshalling only: the solve, the centring and the derivative run in the
library's kernels; this module maps gradients between E-slots and triplets.
The loss must depend on X only through the aggregate sparsity pattern (where
the completion X^ equals Xbar), e.g. L = <G_L, X> with G_L on that pattern.
"""
from __future__ import annotations

import numpy as np
import torch

from .sdpc import sdpc_create


class _Instance:
    """A problem with replaced A_0 values and b (duck-typed like sdpgen.Problem)."""

    def __init__(self, base, a0, b):
        self.n, self.m = base.n, base.m
        self.ptr, self.row, self.col = base.ptr, base.row, base.col
        self.val = np.array(base.val, dtype=np.float64, copy=True)
        self.val[int(base.ptr[0]):int(base.ptr[1])] = a0
        self.b = np.asarray(b, dtype=np.float64)


def _slot_maps(h, problem):
    """E-slot weights (1 on the diagonal, 2 off it, 0 on padding) and the slot of
    every A_0 triplet."""
    iE, jE, _ = h.sdpc_get_pattern()
    ok = iE >= 0
    wE = np.where(ok, np.where(iE == jE, 1.0, 2.0), 0.0)
    key = {}
    for s in np.nonzero(ok)[0]:
        a, c = int(iE[s]), int(jE[s])
        key[(max(a, c), min(a, c))] = int(s)
    s0, s1 = int(problem.ptr[0]), int(problem.ptr[1])
    r, c = problem.row[s0:s1], problem.col[s0:s1]
    a0_slot = np.array([key[(int(max(a, b)), int(min(a, b)))] for a, b in zip(r, c)], dtype=np.int64)
    a0_diag = (r == c)
    return wE, a0_slot, a0_diag


class CentralSDP(torch.autograd.Function):

    @staticmethod
    def forward(ctx, a0, b, problem, mu, params=None):
        params = dict(params or {})
        inst = _Instance(problem, a0.detach().cpu().numpy(), b.detach().cpu().numpy())
        h = sdpc_create(inst, **params)
        r = h.sdpc_solve()
        if r["status"] != 0:
            raise RuntimeError(f"CentralSDP: solve failed: {r}")
        h.sdpc_center(mu)
        X_E, _, z = h.sdpc_get_solution()
        wE, a0_slot, a0_diag = _slot_maps(h, problem)
        ctx.h = h
        ctx.maps = (wE, a0_slot, a0_diag)
        return X_E, z

    @staticmethod
    def backward(ctx, gX, gz):
        h = ctx.h
        wE, a0_slot, a0_diag = ctx.maps
        dev = h.device
        w = torch.as_tensor(wE, device=dev)
        # L = sum_s gX_s X_s = <G_L, X> with G_L(i, j) = gX_s / wE_s on slot s
        GL = torch.where(w > 0, (gX if gX is not None else torch.zeros_like(w)) / torch.clamp(w, min=1.0),
                         torch.zeros_like(w)).contiguous()
        dz = None if gz is None else gz.contiguous()
        gb, gC = h.sdpc_adjoint(GL, dz)
        # a triplet (i, j) of A_0 moves both symmetric entries: 2 dL/dA_0(i, j) off the diagonal
        sl = torch.as_tensor(a0_slot, device=dev)
        scale = torch.as_tensor(np.where(a0_diag, 1.0, 2.0), device=dev)
        ga0 = gC[sl] * scale
        h.close()
        ctx.h = None
        return ga0, gb, None, None, None
