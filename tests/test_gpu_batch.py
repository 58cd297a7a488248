"""GPU: the batched solver (sdpc_batch_solve) on instances of the k-tree max-cut
batch (n uniform in [50, 800], random k-trees with k in [3, 12], 30% of the
edges dropped, weights U[0,1], seed 0), each in the reverse insertion order of
its k-tree.

Every instance must be solved; each objective must match the plain solver's on
the same instance (1e-7 relative: the tuned block width changes only rounding),
and a seeded sample of instances must match the matrix-completion oracle in the
same elimination order (objective 1e-7, z 1e-6, iteration count within one).
"""
import numpy as np
import pytest

import oracle
import sdpgen
from tests.gpu_common import host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_6919_amd import load
    load()


def _rev(p):
    return np.arange(p.n)[::-1].astype(np.int32)


@pytest.fixture(scope="module")
def batch():
    from paper_1310_6919_amd.sdpc import sdpc_batch_solve
    probs = sdpgen.maxcut_ktree_batch(256, 0)[:40]
    res, zs, opt = sdpc_batch_solve(probs, [{"user_perm": _rev(p)} for p in probs], workers=6, autotune=True)
    return probs, res, zs, opt


def test_batch_solves_every_instance_like_the_plain_solver(batch):
    from paper_1310_6919_amd import sdpc_create
    probs, res, zs, opt = batch
    assert all(r["status"] == 0 for r in res)
    assert any(w > 0 for w in opt["tuned_width"])
    for p, r, z in zip(probs, res, zs):
        h = sdpc_create(p, user_perm=_rev(p))
        r0 = h.sdpc_solve()
        _, _, z0 = h.sdpc_get_solution()
        h.close()
        o, o0 = (r["pobj"] + r["dobj"]) / 2, (r0["pobj"] + r0["dobj"]) / 2
        assert abs(o - o0) <= 1e-7 * max(1.0, abs(o0)), (p.name, o, o0)
        assert np.abs(host(z) - host(z0)).max() <= 1e-5 * max(1.0, np.abs(host(z0)).max())


def test_batch_sample_matches_mc_oracle(batch):
    probs, res, zs, opt = batch
    rng = np.random.default_rng(5)
    small = [i for i, p in enumerate(probs) if p.n <= 320]
    for i in rng.choice(small, size=min(8, len(small)), replace=False):
        p = probs[i]
        ref = oracle.mc_pdipm(p, oracle.Params(), order=_rev(p))
        assert ref["status"] == "optimal"
        r = res[i]
        assert abs(r["iters"] - ref["iters"]) <= 1, (p.name, r["iters"], ref["iters"])
        o, ro = (r["pobj"] + r["dobj"]) / 2, (ref["pobj"] + ref["dobj"]) / 2
        assert abs(o - ro) <= 1e-7 * max(1.0, abs(ro)), (p.name, o, ro)
        assert np.abs(host(zs[i]) - ref["z"]).max() <= 1e-6 * max(1.0, np.abs(ref["z"]).max()), p.name
