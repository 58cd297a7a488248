"""Oracle checkers: values fixed by combinatorics or closed forms.

brute_force_maxcut  maximum cut weight over all 2^(n-1) bipartitions.
cycle_sdp_value     the max-cut SDP value of the unit-weight cycle C_n,
                    (n/4) lambda_max(L(C_n)) = (n/2)(1 - cos(2 pi floor(n/2) / n)),
                    valid because C_n is vertex transitive (a uniform dual is
                    optimal).
"""
from __future__ import annotations

import numpy as np


def brute_force_maxcut(n: int, edges: np.ndarray, w: np.ndarray) -> float:
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.asarray(w, dtype=np.float64)
    if n <= 1 or len(edges) == 0:
        return 0.0
    masks = np.arange(1 << (n - 1), dtype=np.int64)       # vertex n-1 fixed on side 0
    best = 0.0
    for s0 in range(0, len(masks), 1 << 16):
        mk = masks[s0:s0 + (1 << 16)]
        side_i = (mk[:, None] >> edges[None, :, 0]) & 1
        side_j = (mk[:, None] >> edges[None, :, 1]) & 1
        cut = ((side_i != side_j) * w[None, :]).sum(1)
        best = max(best, float(cut.max()))
    return best


def cycle_sdp_value(n: int) -> float:
    return (n / 2.0) * (1.0 - np.cos(2.0 * np.pi * (n // 2) / n))
