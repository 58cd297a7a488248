"""GPU: the handle-free dense Cholesky on the fixed per-GPU workspace
(sdpc_potrf_static, for callers that cannot allocate device memory) against
the handle's sdpc_potrf on the same inputs, through the C ABI.

Both run the same kernels, so their factors must agree bit for bit; each is
also held to LAPACK's factor (1e-12 times the condition number, as for
sdpc_potrf).  Two calls in a row, the second on a smaller matrix, check that
the workspace left by the first call does not leak into the second.
"""
import ctypes as C

import numpy as np
import pytest

import sdpgen
from tests.gpu_common import dev, host, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_6919_amd import load
    load()


def _colmajor(A):
    return dev(A.T.copy()).T


def test_static_potrf_matches_handle_potrf_twice():
    from paper_1310_6919_amd import sdpc_create
    from paper_1310_6919_amd.sdpc import sdpc_potrf_static
    # handle sized for m <= 300, with the per-block Cholesky the static entry point runs
    h = sdpc_create(sdpgen.maxcut_band(300, 3, 1.0, 0), chol_kernel=1)
    rng = np.random.default_rng(2024)
    for m in (300, 130):   # the second call is smaller than the first
        A = sdpgen.random_pd_dense(m, rng, cond=1e3)
        marker = np.triu(np.full((m, m), 7.0), 1)
        Bh = _colmajor(A + marker)
        Bs = _colmajor(A + marker)
        h.sdpc_potrf(Bh, m)
        sdpc_potrf_static(Bs, m)
        torch.cuda.synchronize()
        Rh, Rs = host(Bh), host(Bs)
        assert np.array_equal(np.tril(Rs), np.tril(Rh)), f"m={m}: static and handle factors differ"
        assert np.array_equal(np.triu(Rs, 1), np.triu(A, 1) + marker)   # strict upper untouched
        assert rel_err(np.tril(Rs), np.linalg.cholesky(A)) <= 1e-12 * 1e3
    h.close()


def test_static_potrf_async_info_and_not_pd():
    from paper_1310_6919_amd import SdpcError
    from paper_1310_6919_amd.sdpc import SDPC_E_NOT_PD, sdpc_potrf_static
    rng = np.random.default_rng(7)
    m = 200
    A = sdpgen.random_pd_dense(m, rng, cond=50.0)
    B = _colmajor(A)
    info = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    sdpc_potrf_static(B, m, info=info)   # asynchronous: the outcome arrives in info
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert rel_err(np.tril(host(B)), np.linalg.cholesky(A)) <= 1e-12 * 50
    # a failed pivot: reported through info, and as SDPC_E_NOT_PD by the synchronous form
    piv = 97
    A = np.eye(m)
    A[piv, piv] = -1.0
    info.fill_(99)
    sdpc_potrf_static(_colmajor(A), m, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == piv + 1
    with pytest.raises(SdpcError) as e:
        sdpc_potrf_static(_colmajor(A), m)
    assert e.value.status == SDPC_E_NOT_PD and f"pivot {piv}" in str(e.value)


def test_static_potrf_rejects_oversize():
    from paper_1310_6919_amd import load
    from paper_1310_6919_amd.sdpc import SDPC_E_ARG
    lib = load()
    B = torch.zeros(4, dtype=torch.float64, device="cuda")
    st = lib.sdpc_potrf_static(C.c_void_p(B.data_ptr()), 65536, 65536, None,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == SDPC_E_ARG
    assert b"exceeds the limit of 65535" in lib.sdpc_last_error(None)
