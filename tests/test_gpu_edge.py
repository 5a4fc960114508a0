"""Edge cases and error paths through the C ABI (sizes at the limits, degenerate partitions)."""
import numpy as np
import pytest
import torch

import levelgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2407_08901_amd as P
    P.lib()
    return P


def _lam(A, k):
    return np.linalg.eigvalsh(oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n).toarray())[:k]


class _Upper:
    """An upper CSR built here (row_ptr, col, val, level_offsets, n, nnz)."""

    def __init__(self, n, rows, cols, vals, level_offsets):
        order = np.lexsort((cols, rows))
        rows, cols, vals = rows[order], cols[order], vals[order]
        self.n = n
        self.row_ptr = np.zeros(n + 1, np.int64)
        np.add.at(self.row_ptr, rows + 1, 1)
        self.row_ptr = np.cumsum(self.row_ptr)
        self.col = cols.astype(np.int32)
        self.val = vals.astype(np.float32)
        self.level_offsets = np.asarray(level_offsets, np.int64)
        self.nnz = len(cols)


def _solve(P, A, ns, k, **kw):
    rp, col, val = P.upload(A)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(**kw))
    out = P.sppc_solve(ctx)
    P.sppc_destroy(ctx)
    return out


@pytest.mark.parametrize("k", [1, 16])
def test_k_at_its_limits(P, k):
    A = levelgen.generate((60, 600, 5000), 40, 61) if k == 16 else levelgen.WORKLOADS[0].generate()
    print("case edge k=%d n=%d" % (k, A.n), flush=True)
    ev, Z, rrn, st, status = _solve(P, A, 1, k)
    assert status == P.SPPC_OK and max(rrn) < 1e-6
    lam = _lam(A, k)
    assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-10


def test_tiny_ragged_levels(P):
    A = levelgen.generate((5, 7, 11), 4, 3)
    print("case edge tiny n=%d" % A.n, flush=True)
    ev, Z, rrn, st, status = _solve(P, A, 1, 2)
    assert status == P.SPPC_OK
    lam = _lam(A, 2)
    assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-10


def test_small_space_is_everything(P):
    # n0 = n: H0 = H and V = 0, so the zeroth order is exact (converged at p = 0)
    A = levelgen.generate((40, 300), 20, 8)
    print("case edge n0=n", flush=True)
    ev, Z, rrn, st, status = _solve(P, A, 2, 3)
    assert status == P.SPPC_OK and st["iterations"] == 0
    lam = _lam(A, 3)
    assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-10


def test_decoupled_small_space(P):
    # no entries between the small space and the rest: V Psi^(0) = 0, converged at p = 0 with the
    # lowest eigenvalues those of H0hat (they lie below the other levels here)
    B = levelgen.generate((50, 400, 3000), 30, 9)
    rows = np.repeat(np.arange(B.n), np.diff(B.row_ptr))
    keep = ~((rows < 50) & (B.col >= 50))
    A = _Upper(B.n, rows[keep], B.col[keep].astype(np.int64), B.val[keep], B.level_offsets)
    print("case edge decoupled", flush=True)
    ev, Z, rrn, st, status = _solve(P, A, 1, 4)
    assert status == P.SPPC_OK and st["iterations"] == 0
    lam = _lam(A, 4)
    assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-10


def _setup_status(P, A, ns, k, **kw):
    rp, col, val = P.upload(A)
    try:
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(**kw))
    except P.SPPCError as e:
        return e.status
    P.sppc_destroy(ctx)
    return P.SPPC_OK


def test_singular_zeroth_order_is_refused(P):
    # H0hat = diag(-2, 0, 1): the second wanted E^(0) is zero (eq. sm_first divides by it)
    n = 9
    rows = np.array([0, 1, 2] + list(range(3, n)) + [0, 2], np.int64)
    cols = np.array([0, 1, 2] + list(range(3, n)) + [5, 7], np.int64)
    vals = np.array([-2.0, 0.0, 1.0] + [10.0 + i for i in range(3, n)] + [0.3, 0.2])
    A = _Upper(n, rows, cols, vals, [0, 3, n])
    print("case edge singular E0", flush=True)
    assert _setup_status(P, A, 1, 2) == P.SPPC_E_SINGULAR_E0


def test_invalid_inputs_are_refused(P):
    A = levelgen.generate((20, 90, 300), 14, 4)
    print("case edge invalid inputs", flush=True)
    assert _setup_status(P, A, 1, 0) == P.SPPC_E_ARG                      # k = 0
    assert _setup_status(P, A, 1, 21) == P.SPPC_E_ARG                     # k > n0
    assert _setup_status(P, A, 4, 2) == P.SPPC_E_ARG                      # more small levels than levels
    assert _setup_status(P, A, 1, 2, m_max=3) == P.SPPC_E_ARG             # m_max < 2k
    assert _setup_status(P, A, 1, 2, panel_width=70000) == P.SPPC_E_ARG
    assert _setup_status(P, A, 1, 2, precond=9) == P.SPPC_E_ARG
    assert _setup_status(P, A, 1, 2, precond_tol=1.5) == P.SPPC_E_ARG
    bad = _Upper(A.n, np.repeat(np.arange(A.n), np.diff(A.row_ptr)), A.col.astype(np.int64), A.val,
                 [0, 20, 110, 409])                                        # offsets do not end at n
    assert _setup_status(P, bad, 1, 2) == P.SPPC_E_ARG
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    lower = _Upper(A.n, np.append(rows, 30), np.append(A.col, 5).astype(np.int64), np.append(A.val, 0.1),
                   A.level_offsets)                                        # an entry below the diagonal
    assert _setup_status(P, lower, 1, 2) == P.SPPC_E_ARG
    nanv = _Upper(A.n, rows, A.col.astype(np.int64), np.where(np.arange(A.nnz) == 7, np.nan, A.val),
                  A.level_offsets)
    assert _setup_status(P, nanv, 1, 2) == P.SPPC_E_NAN


def test_invalid_calls_on_a_context(P):
    A = levelgen.generate((20, 90, 300), 14, 4)
    print("case edge invalid calls", flush=True)
    rp, col, val = P.upload(A)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, 2, P.sppc_default_opts())
    X = torch.zeros((A.n, 40), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(P.SPPCError) as e:
        P.sppc_spmm(ctx, X, Y)                                             # b = 40 > 32
    assert e.value.status == P.SPPC_E_ARG
    with pytest.raises(P.SPPCError) as e:
        P.sppc_correct(ctx, 17)
    assert e.value.status == P.SPPC_E_ARG
    w = np.zeros(P.SPPC_MPNN_NPARAM, np.float32)
    R = torch.zeros((A.n, 33), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SPPCError) as e:
        P.sppc_mpnn_eval(ctx, w, R, R.clone(), [0.0] * 33)                 # S = 33 > 32
    assert e.value.status == P.SPPC_E_ARG
    with pytest.raises(P.SPPCError) as e:
        P.sppc_correct(ctx, P.SPPC_CORR_MPNN)                              # no weights set
    assert e.value.status == P.SPPC_E_ARG
    # the context still works after refused calls
    ev, Z, rrn, st, status = P.sppc_solve(ctx)
    assert status == P.SPPC_OK
    P.sppc_destroy(ctx)
