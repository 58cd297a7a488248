"""Helpers shared by the GPU parity tests (marshalling only, no arithmetic of
the method)."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def to_E(h, dense):
    """Dense symmetric matrix (original indices) -> E-vector in the library's layout."""
    iE, jE, _ = h.sdpc_get_pattern()
    v = np.zeros(len(iE))
    ok = iE >= 0
    v[ok] = dense[iE[ok], jE[ok]]
    return v


def from_E(h, vec):
    """E-vector -> dense symmetric matrix on E (original indices), zero elsewhere."""
    iE, jE, _ = h.sdpc_get_pattern()
    out = np.zeros((h.n, h.n))
    ok = iE >= 0
    out[iE[ok], jE[ok]] = vec[ok]
    out[jE[ok], iE[ok]] = vec[ok]
    return out


def golden(name):
    with open(os.path.join(GOLDEN, f"oracle_{name}.json")) as f:
        return json.load(f)


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(1e-300, np.abs(b).max()))
