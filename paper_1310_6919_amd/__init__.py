"""MI355X-native hot path of the matrix-completion primal-dual interior-point
method (Yamashita & Nakata, SDPA-C 7): the Schur complement matrix through the
Cholesky factor of the inverse of the max-determinant completion and the
sparse Cholesky factor of Y, its dense FP64 Cholesky, and the rest of each
iteration, behind the C ABI of include/sdpc.h.
"""
from .sdpc import (EXPORTS, Handle, SdpcError, load, sdpc_analyze, sdpc_create,  # noqa: F401
                   sdpc_default_params, LIB_PATH)
