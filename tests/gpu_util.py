"""Helpers shared by the GPU tests (inputs and comparisons only)."""
import numpy as np
import scipy.sparse as sp


def full_from_upper(A):
    U = sp.csr_matrix((A.val.astype(np.float64), A.col, A.row_ptr), shape=(A.n, A.n))
    return (U + U.T - sp.diags(U.diagonal())).tocsr()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))
