"""Thin ctypes binding of libsdpc.so (include/sdpc.h), same names as the C ABI.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device buffers are torch tensors (float64 / int32 on a HIP
device); the stream handed to sdpc_create is torch's current stream.  The
library must be built (paper_1310_6919_amd.build); loading fails loudly
otherwise, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libsdpc.so")

SDPC_OK, SDPC_E_ARG, SDPC_E_PATTERN, SDPC_E_NOT_PD, SDPC_E_HIP, SDPC_E_MAXITER, \
    SDPC_E_STAGNATION, SDPC_E_NUMERIC, SDPC_E_OOM = 0, -1, -2, -3, -4, -5, -6, -7, -8

EXPORTS = ["sdpc_default_params", "sdpc_analyze", "sdpc_create", "sdpc_solve", "sdpc_reset", "sdpc_step", "sdpc_scm",
           "sdpc_potrf", "sdpc_get_pattern", "sdpc_get_cliques", "sdpc_get_solution", "sdpc_set_state",
           "sdpc_get_factors", "sdpc_get_dense", "sdpc_complete_dense", "sdpc_get_direction", "sdpc_get_scm_timing",
           "sdpc_default_batch_options", "sdpc_batch_solve", "sdpc_center", "sdpc_adjoint", "sdpc_potrf_static", "sdpc_status_string", "sdpc_last_error", "sdpc_destroy"]


class sdpc_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("ptr", C.POINTER(C.c_int64)),
                ("row", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double))]


class sdpc_params(C.Structure):
    _fields_ = [("gap_tol", C.c_double), ("feas_tol", C.c_double), ("beta_feas", C.c_double),
                ("beta_infeas", C.c_double), ("gamma", C.c_double), ("lambda0", C.c_double),
                ("max_iter", C.c_int32), ("ordering", C.c_int32), ("block_width", C.c_int32),
                ("verbose", C.c_int32), ("pool_lds_bytes", C.c_int32), ("solve_kernel", C.c_int32),
                ("factorization", C.c_int32), ("merge_siblings", C.c_int32), ("dual_points", C.c_int32),
                ("chol_kernel", C.c_int32), ("user_perm", C.POINTER(C.c_int32))]


class sdpc_analysis(C.Structure):
    _fields_ = [("nslot", C.c_int64), ("nnzE", C.c_int64), ("ncliques", C.c_int32), ("nblocks", C.c_int32),
                ("max_clique", C.c_int32), ("max_block_rows", C.c_int32), ("max_block_cols", C.c_int32),
                ("nfwd", C.c_int32), ("nbwd", C.c_int32), ("hadamard", C.c_int32), ("sum_clique", C.c_int64),
                ("limit_clique", C.c_int32), ("limit_panel", C.c_int32), ("limit_m", C.c_int32),
                ("pad_", C.c_int32), ("device_bytes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class sdpc_batch_options(C.Structure):
    _fields_ = [("workers", C.c_int32), ("autotune", C.c_int32), ("tuned_width", C.c_int32 * 9),
                ("dual_points", C.c_int32), ("tune_ms", C.c_double), ("create_ms", C.c_double),
                ("solve_ms", C.c_double), ("total_ms", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["tuned_width"] = list(self.tuned_width)
        return d


class sdpc_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("pobj", C.c_double), ("dobj", C.c_double),
                ("rel_gap", C.c_double), ("pinf", C.c_double), ("dinf", C.c_double), ("mu", C.c_double),
                ("alpha_p", C.c_double), ("alpha_d", C.c_double), ("beta", C.c_double),
                ("t_scm_ms", C.c_double), ("t_chol_ms", C.c_double), ("t_pmatrix_ms", C.c_double),
                ("t_total_ms", C.c_double), ("t_potrf_ms", C.c_double), ("n_potrf", C.c_int32),
                ("pad_", C.c_int32), ("device_bytes", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load libsdpc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_1310_6919_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, VP, I32, I64, D = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "sdpc_default_params": (sdpc_params, []),
        "sdpc_analyze": (I32, [P(sdpc_problem), P(sdpc_params), P(sdpc_analysis), VP, VP, VP, VP]),
        "sdpc_create": (I32, [P(sdpc_problem), P(sdpc_params), VP, P(VP)]),
        "sdpc_solve": (I32, [VP, P(sdpc_result)]),
        "sdpc_reset": (I32, [VP]),
        "sdpc_step": (I32, [VP, P(sdpc_result)]),
        "sdpc_scm": (I32, [VP, VP, VP, VP, I64, I32]),
        "sdpc_potrf": (I32, [VP, VP, I64, I32]),
        "sdpc_get_pattern": (I32, [VP, P(I64), VP, VP, VP, P(I32)]),
        "sdpc_get_cliques": (I32, [VP, VP, VP, VP]),
        "sdpc_get_solution": (I32, [VP, VP, VP, VP]),
        "sdpc_set_state": (I32, [VP, VP, VP, VP]),
        "sdpc_get_factors": (I32, [VP, VP, VP]),
        "sdpc_get_dense": (I32, [VP, VP, VP]),
        "sdpc_complete_dense": (I32, [VP, VP]),
        "sdpc_get_direction": (I32, [VP, VP, VP, VP, P(D)]),
        "sdpc_get_scm_timing": (I32, [VP, P(D)]),
        "sdpc_default_batch_options": (sdpc_batch_options, []),
        "sdpc_batch_solve": (I32, [I32, VP, VP, P(sdpc_batch_options), VP, VP]),
        "sdpc_center": (I32, [VP, D, I32, D, P(I32), P(D)]),
        "sdpc_adjoint": (I32, [VP, VP, VP, VP, VP]),
        "sdpc_potrf_static": (I32, [VP, I64, I32, VP, VP]),
        "sdpc_status_string": (C.c_char_p, [I32]),
        "sdpc_last_error": (C.c_char_p, [VP]),
        "sdpc_destroy": (None, [VP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SdpcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _np(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


def sdpc_default_params(**kw) -> sdpc_params:
    p = load().sdpc_default_params()
    for k, v in kw.items():
        if k == "user_perm":
            continue
        setattr(p, k, v)
    return p


def _problem_struct(prob, keep):
    arrs = [_np(prob.ptr, np.int64), _np(prob.row, np.int32), _np(prob.col, np.int32),
            _np(prob.val, np.float64), _np(prob.b, np.float64)]
    keep.extend(arrs)
    ptr, row, col, val, b = arrs
    return sdpc_problem(int(prob.n), int(prob.m), ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                        row.ctypes.data_as(C.POINTER(C.c_int32)), col.ctypes.data_as(C.POINTER(C.c_int32)),
                        val.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double)))


def _params_struct(params, keep):
    prm = sdpc_default_params(**params)
    if params.get("user_perm") is not None:
        up = _np(params["user_perm"], np.int32)
        keep.append(up)
        prm.user_perm = up.ctypes.data_as(C.POINTER(C.c_int32))
        prm.ordering = 2
    return prm


def sdpc_analyze(prob, **params):
    """Host-only symbolic phase: (info dict, perm, cliques, nS); no device is touched."""
    lib = load()
    keep = []
    cp = _problem_struct(prob, keep)
    prm = _params_struct(params, keep)
    info = sdpc_analysis()
    st = lib.sdpc_analyze(C.byref(cp), C.byref(prm), C.byref(info), None, None, None, None)
    if st != SDPC_OK:
        raise SdpcError(st, "sdpc_analyze: " + lib.sdpc_status_string(st).decode())
    perm = np.empty(int(prob.n), np.int32)
    cptr = np.empty(info.ncliques + 1, np.int64)
    cidx = np.empty(int(info.sum_clique), np.int32)
    nS = np.empty(info.ncliques, np.int32)
    st = lib.sdpc_analyze(C.byref(cp), C.byref(prm), C.byref(info), perm.ctypes.data_as(C.c_void_p),
                          cptr.ctypes.data_as(C.c_void_p), cidx.ctypes.data_as(C.c_void_p),
                          nS.ctypes.data_as(C.c_void_p))
    if st != SDPC_OK:
        raise SdpcError(st, "sdpc_analyze: " + lib.sdpc_status_string(st).decode())
    cliques = [cidx[cptr[r]:cptr[r + 1]] for r in range(info.ncliques)]
    return info.as_dict(), perm, cliques, nS


class Handle:
    """Owns an sdpc_handle and the host copies its create call reads."""

    def __init__(self, prob, stream=None, **params):
        import torch
        lib = load()
        self.lib = lib
        self.n, self.m = int(prob.n), int(prob.m)
        self._keep = []
        cp = _problem_struct(prob, self._keep)
        prm = _params_struct(params, self._keep)
        self.params = prm
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        st = lib.sdpc_create(C.byref(cp), C.byref(prm), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != SDPC_OK:
            raise SdpcError(st, "sdpc_create: " + lib.sdpc_status_string(st).decode())
        self.h = h
        self.device = torch.device("cuda", torch.cuda.current_device())
        n_ = C.c_int64()
        ncl = C.c_int32()
        self._check(lib.sdpc_get_pattern(h, C.byref(n_), None, None, None, C.byref(ncl)), "sdpc_get_pattern")
        self.nslot = int(n_.value)
        self.ncliques = int(ncl.value)

    # -- helpers
    def _check(self, st, what):
        if st != SDPC_OK:
            raise SdpcError(st, f"{what}: {self.lib.sdpc_last_error(self.h).decode()}")

    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.sdpc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, one method per entry point
    def sdpc_solve(self):
        r = sdpc_result()
        st = self.lib.sdpc_solve(self.h, C.byref(r))
        d = r.as_dict()
        d["status"] = int(st)
        if st not in (SDPC_OK, SDPC_E_MAXITER, SDPC_E_STAGNATION):
            self._check(st, "sdpc_solve")
        return d

    def sdpc_reset(self):
        self._check(self.lib.sdpc_reset(self.h), "sdpc_reset")

    def sdpc_step(self):
        r = sdpc_result()
        st = self.lib.sdpc_step(self.h, C.byref(r))
        self._check(st, "sdpc_step")
        return r.as_dict()

    @staticmethod
    def _ld(B, m):
        """Leading dimension of a column-major (stride(0) == 1) matrix view."""
        if B.dim() != 2 or B.dtype.itemsize != 8 or (B.shape[0] > 1 and B.stride(0) != 1):
            raise ValueError("B must be a 2-D float64 column-major view (e.g. torch.empty(m, m).T)")
        return max(B.stride(1), m, 1) if B.shape[1] > 1 else max(m, 1)

    def sdpc_scm(self, Xbar_E, Y_E, B=None, factor=False):
        """B (m x m, column-major view): lower triangle <- SCM (or its Cholesky factor)."""
        if B is None:
            B = self._empty(self.m, self.m).zero_().T
        self._check(self.lib.sdpc_scm(self.h, _ptr(Xbar_E), _ptr(Y_E), _ptr(B), self._ld(B, self.m),
                                      int(bool(factor))), "sdpc_scm")
        return B

    def sdpc_potrf(self, B, m=None):
        m = self.m if m is None else m
        self._check(self.lib.sdpc_potrf(self.h, _ptr(B), self._ld(B, m), m), "sdpc_potrf")
        return B

    def sdpc_get_pattern(self):
        iE = np.empty(self.nslot, np.int32)
        jE = np.empty(self.nslot, np.int32)
        perm = np.empty(self.n, np.int32)
        n_ = C.c_int64()
        self._check(self.lib.sdpc_get_pattern(self.h, C.byref(n_), iE.ctypes.data_as(C.c_void_p),
                                              jE.ctypes.data_as(C.c_void_p), perm.ctypes.data_as(C.c_void_p),
                                              None), "sdpc_get_pattern")
        return iE, jE, perm

    def sdpc_get_cliques(self):
        cptr = np.empty(self.ncliques + 1, np.int64)
        nS = np.empty(self.ncliques, np.int32)
        self._check(self.lib.sdpc_get_cliques(self.h, cptr.ctypes.data_as(C.c_void_p), None,
                                              nS.ctypes.data_as(C.c_void_p)), "sdpc_get_cliques")
        cidx = np.empty(int(cptr[-1]), np.int32)
        self._check(self.lib.sdpc_get_cliques(self.h, None, cidx.ctypes.data_as(C.c_void_p), None),
                    "sdpc_get_cliques")
        return [cidx[cptr[r]:cptr[r + 1]] for r in range(self.ncliques)], nS

    def sdpc_get_solution(self):
        X, Y, z = self._empty(self.nslot), self._empty(self.nslot), self._empty(self.m)
        self._check(self.lib.sdpc_get_solution(self.h, _ptr(X), _ptr(Y), _ptr(z)), "sdpc_get_solution")
        return X, Y, z

    def sdpc_set_state(self, X_E, Y_E, z):
        self._check(self.lib.sdpc_set_state(self.h, _ptr(X_E), _ptr(Y_E), _ptr(z)), "sdpc_set_state")

    def sdpc_get_factors(self):
        N, L = self._empty(self.nslot), self._empty(self.nslot)
        self._check(self.lib.sdpc_get_factors(self.h, _ptr(N), _ptr(L)), "sdpc_get_factors")
        return N, L

    def sdpc_get_dense(self):
        Xh, Yi = self._empty(self.n, self.n), self._empty(self.n, self.n)
        self._check(self.lib.sdpc_get_dense(self.h, _ptr(Xh), _ptr(Yi)), "sdpc_get_dense")
        return Xh.T, Yi.T   # stored column-major

    def sdpc_complete_dense(self, out=True):
        """Max-determinant completion of the current Xbar, n x n in original indices."""
        Xh = self._empty(self.n, self.n) if out else None
        self._check(self.lib.sdpc_complete_dense(self.h, _ptr(Xh)), "sdpc_complete_dense")
        return None if Xh is None else Xh.T   # stored column-major (symmetric anyway)

    def sdpc_get_direction(self):
        dz, dX, dY = self._empty(self.m), self._empty(self.nslot), self._empty(self.nslot)
        al = (C.c_double * 2)()
        self._check(self.lib.sdpc_get_direction(self.h, _ptr(dz), _ptr(dX), _ptr(dY), al), "sdpc_get_direction")
        return dz, dX, dY, (al[0], al[1])

    def sdpc_center(self, mu, max_steps=60, tol=1e-14):
        """Newton steps toward the mu-central point; returns (steps, last relative z step)."""
        k = C.c_int32()
        rel = C.c_double()
        self._check(self.lib.sdpc_center(self.h, float(mu), int(max_steps), float(tol), C.byref(k), C.byref(rel)),
                    "sdpc_center")
        return int(k.value), float(rel.value)

    def sdpc_adjoint(self, GL_E, dLdz=None):
        """(dL/db, dL/dA_0 as an E-vector) at the current (central) iterate."""
        gb, gC = self._empty(self.m), self._empty(self.nslot)
        self._check(self.lib.sdpc_adjoint(self.h, _ptr(GL_E), _ptr(dLdz), _ptr(gb), _ptr(gC)), "sdpc_adjoint")
        return gb, gC

    def sdpc_get_scm_timing(self):
        ms = (C.c_double * 5)()
        self._check(self.lib.sdpc_get_scm_timing(self.h, ms), "sdpc_get_scm_timing")
        return list(ms)


def sdpc_potrf_static(B, m=None, info=None, stream=None):
    """Handle-free dense Cholesky on a fixed per-GPU workspace (no device allocation).

    B: column-major float64 view (lower triangle overwritten by R).  info: optional
    int32 device tensor of one element; when given the call is asynchronous and
    info receives 0 or 1 + the failing pivot."""
    import torch
    lib = load()
    m = B.shape[0] if m is None else m
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib.sdpc_potrf_static(_ptr(B), Handle._ld(B, m), int(m), _ptr(info), C.c_void_p(stream.cuda_stream))
    if st != SDPC_OK:
        raise SdpcError(st, "sdpc_potrf_static: " + lib.sdpc_last_error(None).decode())
    return B


def sdpc_batch_solve(probs, params=None, workers=8, autotune=True, want_z=True, dual_points=None):
    """Solve many SDPs at once (sdpc_batch_solve).  params: None, one dict for all,
    or a list of dicts (e.g. per-instance user_perm).  Returns (results, z list,
    options dict); raises SdpcError if an instance fails."""
    import torch
    lib = load()
    count = len(probs)
    keep = []
    probs_arr = (sdpc_problem * max(count, 1))()
    prm_arr = (sdpc_params * max(count, 1))()
    for i, p in enumerate(probs):
        probs_arr[i] = _problem_struct(p, keep)
        pd = params[i] if isinstance(params, (list, tuple)) else (params or {})
        prm_arr[i] = _params_struct(pd, keep)
    opt = lib.sdpc_default_batch_options()
    opt.workers = int(workers)
    opt.autotune = int(bool(autotune))
    if dual_points is not None:
        opt.dual_points = int(dual_points)
    res = (sdpc_result * max(count, 1))()
    zs = [torch.empty(int(p.m), dtype=torch.float64, device="cuda") for p in probs] if want_z else None
    zp = (C.c_void_p * max(count, 1))(*([z.data_ptr() for z in zs] if zs else [None] * count)) if want_z else None
    torch.cuda.synchronize()
    st = lib.sdpc_batch_solve(count, probs_arr, prm_arr, C.byref(opt), res, zp)
    out = []
    for i in range(count):
        d = res[i].as_dict()
        out.append(d)
    if st != SDPC_OK:
        raise SdpcError(st, "sdpc_batch_solve: " + lib.sdpc_last_error(None).decode())
    return out, zs, opt.as_dict()


def sdpc_create(prob, stream=None, **params) -> Handle:
    return Handle(prob, stream=stream, **params)
