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


def test_basis_that_fills_the_whole_space(P):
    # n = 285, k = 14, solved to 1e-9: the 15 perturbative steps alone fill 224 columns, and the
    # continuation brings the basis to all n directions.  The last blocks are then dependent on the
    # basis and on each other; the Cholesky-QR must drop what only rounding keeps apart (the oracle's
    # pivoted Householder QR does), or the basis loses orthogonality and the solve breaks down.
    A = levelgen.generate((33, 252), 79, 275309)
    print("case edge full basis n=%d" % A.n, flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:14]
    r = oracle.sppc(H, 33, 14, oracle.Options(tol=1e-9))
    assert r.converged and r.Q.shape[1] == A.n
    for prec in (P.SPPC_PREC_FP64, P.SPPC_PREC_MIXED):
        rp, col, val = P.upload(A)
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, 14, P.sppc_default_opts(tol=1e-9, precision=prec))
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK and st["basis_size"] <= A.n, (status, st["basis_size"])
        ev = np.array(ev)
        Zh = Z.cpu().numpy()
        assert np.max(np.abs(Zh.T @ Zh - np.eye(14))) < 1e-12
        assert np.max(np.linalg.norm(H @ Zh - Zh * ev[None, :], axis=0) / np.abs(ev)) < 1e-9
        assert np.max(np.abs(ev - lam) / np.abs(lam)) < 1e-12


@pytest.mark.parametrize("shape", [((9, 26, 80, 239, 715), 20, 485638, 11), ((8, 28, 104, 376), 21, 873697, 12)],
                         ids=["n0=35-k11", "n0=36-k12"])
def test_zeroth_order_filter_block_near_the_small_space(P, shape):
    # two small levels of 35 and 36 rows with k = 11 and 12: the float64 form deflates 28 eigenpairs of
    # H0hat, so the filtered block (32 columns) nearly fills the small space.  The filter amplifies
    # its lowest directions by up to ~7e10, so some columns come out almost parallel; the block is
    # orthonormalised on its own there (no basis to stay orthogonal to) and keeps them
    sizes, d, seed, k = shape
    A = levelgen.generate(sizes, d, seed)
    print("case edge zeroth-order block n0=%d k=%d" % (sizes[0] + sizes[1], k), flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:k]
    rp, col, val = P.upload(A)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, 2, k, P.sppc_default_opts())
    ev, Z, rrn, st, status = P.sppc_solve(ctx)
    P.sppc_destroy(ctx)
    assert status == P.SPPC_OK
    assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-10


@pytest.mark.parametrize("sizes,d,seed", [((8, 100, 900), 20, 71), ((16, 150, 1500), 30, 72)], ids=["n0=8", "n0=16"])
def test_k_equals_the_small_space(P, sizes, d, seed):
    # k = n0: every eigenpair of H0hat is a wanted zeroth order, and the small solves deflate all of
    # them (n_deflate = n0), so the CG works on an empty complement
    A = levelgen.generate(sizes, d, seed)
    k = sizes[0]
    print("case edge k=n0=%d" % k, flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:k]
    ref = oracle.sppc(H, k, k, oracle.Options())
    assert ref.converged and np.max(np.abs(ref.theta - lam) / np.abs(lam)) < 1e-10
    rp, col, val = P.upload(A)
    for kw, bound in ((dict(), 1e-10), (dict(precision=P.SPPC_PREC_MIXED), 1e-8),
                      (dict(precond=P.SPPC_CORR_RMMDIIS), 1e-10),
                      (dict(precision=P.SPPC_PREC_MIXED, precond=P.SPPC_CORR_RMMDIIS), 1e-8)):
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, k, P.sppc_default_opts(**kw))
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK and max(rrn) < 1e-6, kw
        assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < bound, kw


def test_one_row_small_space(P):
    # n0 = 1, k = 1: H0hat is the scalar H[0][0], the zeroth order the first unit vector
    A = levelgen.generate((1, 50, 400), 12, 73)
    print("case edge n0=1", flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:1]
    rp, col, val = P.upload(A)
    for kw in (dict(), dict(precision=P.SPPC_PREC_MIXED), dict(precond=P.SPPC_CORR_RMMDIIS)):
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, 1, P.sppc_default_opts(**kw))
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK and max(rrn) < 1e-6, kw
        assert abs(ev[0] - lam[0]) / abs(lam[0]) < 1e-8, kw


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
    assert _setup_status(P, A, 1, 2, auto_switch=2) == P.SPPC_E_ARG
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


def test_no_convergence_returns_the_best_pairs(P):
    # pure SPPC stopped at p = 3 (cfg 0 needs far more): SPPC_E_NOCONV, and what is written is the
    # final check's pairs, as the oracle computes them at the same point, with their true residuals
    w = levelgen.WORKLOADS[0]
    A = w.generate()
    print("case edge no convergence", flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    ref = oracle.sppc(H, w.n0, w.k, oracle.Options(continuation=False, maxiter=3))
    assert not ref.converged
    ev, Z, rrn, st, status = _solve(P, A, w.n_small_levels, w.k, p_switch=0, maxiter=3)
    assert status == P.SPPC_E_NOCONV and st["converged"] == 0 and st["iterations"] == 3
    assert np.max(np.abs(np.array(ev) - ref.theta) / np.abs(ref.theta)) < 1e-10
    Zh = Z.cpu().numpy()
    assert np.max(np.abs(Zh.T @ Zh - np.eye(w.k))) < 1e-12
    R = H @ Zh - Zh * np.array(ev)[None, :]
    true = np.linalg.norm(R, axis=0) / np.abs(ev)
    assert np.allclose(rrn, true, rtol=1e-8) and np.allclose(rrn, ref.rrn, rtol=1e-6)
    assert min(rrn) > 1e-6


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


def _structures():
    """Upper CSRs whose mirror is unusual: no strict-upper entries at all, rows without any entry
    (and without the diagonal), one row coupled to every later column, one column coupled to every
    earlier row (a mirrored row of n - 1 entries), and n above 2^16 (three radix passes)."""
    rng = np.random.default_rng(5)
    out = []
    n = 300
    d = np.arange(n, dtype=np.int64)
    dv = 10.0 * (d >= 20) + rng.uniform(-1, 1, n)
    out.append(("diagonal only", _Upper(n, d, d, dv, [0, 20, n])))
    r = rng.integers(0, n, 2000)
    c = rng.integers(0, n, 2000)
    r, c = np.minimum(r, c), np.maximum(r, c)
    empty = (r % 7 == 3) | (c % 7 == 3)       # rows/columns 3, 10, 17, ... stay empty
    keepd = (d % 7 != 3) | (d < 20)
    rows = np.concatenate([d[keepd], r[~empty]])
    cols = np.concatenate([d[keepd], c[~empty]])
    pairs = np.unique(np.stack([rows, cols], 1), axis=0)
    vals = np.where(pairs[:, 0] == pairs[:, 1], 10.0 * (pairs[:, 0] >= 20), 0.0) + rng.normal(0, 0.5, len(pairs))
    out.append(("empty rows", _Upper(n, pairs[:, 0], pairs[:, 1], vals, [0, 20, n])))
    n = 3000
    d = np.arange(n, dtype=np.int64)
    rows = np.concatenate([d, np.zeros(n - 1, np.int64), np.arange(1, n - 1)])
    cols = np.concatenate([d, np.arange(1, n), np.full(n - 2, n - 1)])
    pairs = np.unique(np.stack([rows, cols], 1), axis=0)
    vals = np.where(pairs[:, 0] == pairs[:, 1], 10.0 * (pairs[:, 0] >= 30) + 1.0 + 0.01 * pairs[:, 0], 0.01)
    out.append(("dense row and column", _Upper(n, pairs[:, 0], pairs[:, 1], vals, [0, 30, n])))
    B = levelgen.generate((100, 1000, 70000), 8, 12)
    out.append(("n = 71,100", B))
    return out


@pytest.mark.parametrize("panel", [0, 1000])
def test_mirror_of_unusual_structures(P, panel):
    # the device copy of both triangles, through the block product, against the oracle's product
    # from the upper triangle (the row-wise CSR kernel, and the panel stream with 1000 columns)
    for name, A in _structures():
        print("case edge mirror %s panel=%d" % (name, panel), flush=True)
        rp, col, val = P.upload(A)
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, 2, P.sppc_default_opts(panel_width=panel))
        X = np.random.default_rng(A.n).standard_normal((A.n, 3))
        Y = torch.empty((A.n, 3), dtype=torch.float64, device="cuda")
        P.sppc_spmm(ctx, torch.from_numpy(X).cuda(), Y)
        torch.cuda.synchronize()
        P.sppc_destroy(ctx)
        ref = oracle.product_from_upper(A.row_ptr, A.col, A.val, A.n, X)
        scale = oracle.product_from_upper(A.row_ptr, A.col, np.abs(A.val), A.n, np.abs(X))
        assert np.max(np.abs(Y.cpu().numpy() - ref) / np.maximum(scale, 1e-300)) < 1e-14, name


def test_cached_memory_is_reused_and_released(P):
    # with the (opt-in) cache enabled, contexts of two sizes interleaved: the cache hands blocks of one
    # size back to the next context of that size (stale contents must not matter), and releasing the
    # cache keeps live contexts intact; disabling it frees what it holds
    As = [levelgen.generate((20, 90, 300), 14, 4), levelgen.generate((30, 200, 900), 16, 5)]
    ref = [_lam(A, 2) for A in As]
    print("case edge memory cache", flush=True)
    assert P.sppc_set_memory_cache(1 << 30) == 0   # off by default
    for rep in range(3):
        for i, A in enumerate(As):
            ev, Z, rrn, st, status = _solve(P, A, 1, 2)
            assert status == P.SPPC_OK
            assert np.max(np.abs(np.array(ev) - ref[i]) / np.abs(ref[i])) < 1e-10
    rp, col, val = P.upload(As[0])
    ctx = P.sppc_setup(rp, col, val, As[0].level_offsets, 1, 2, P.sppc_default_opts())
    assert P.sppc_release_cached_memory() > 0
    ev, Z, rrn, st, status = P.sppc_solve(ctx)
    P.sppc_destroy(ctx)
    assert status == P.SPPC_OK
    assert np.max(np.abs(np.array(ev) - ref[0]) / np.abs(ref[0])) < 1e-10
    assert P.sppc_set_memory_cache(0) == 1 << 30
    assert P.sppc_release_cached_memory() == 0


def test_bad_shifts_are_refused(P):
    w = levelgen.WORKLOADS[0]
    A = w.generate()
    print("case edge shifts", flush=True)
    rp, col, val = P.upload(A)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, w.n_small_levels, w.k, P.sppc_default_opts())
    D = min(3 * w.k, 28, w.n0)  # the float64 form's default n_deflate
    top = P.sppc_get(ctx, 0, D)[-1]
    for bad, code in (([top + 1.0] * w.k, P.SPPC_E_ARG), ([float("nan")] * w.k, P.SPPC_E_ARG),
                      ([0.0] * w.k, P.SPPC_E_ARG)):  # E^(0) < 0 here: zero lies above E_D^(0)
        with pytest.raises(P.SPPCError) as e:
            P.sppc_correct(ctx, P.SPPC_CORR_PERTURBATIVE, shifts=bad)
        assert e.value.status == code
    with pytest.raises(P.SPPCError) as e:
        P.sppc_correct(ctx, P.SPPC_CORR_JACOBI, shifts=[top] * w.k)
    assert e.value.status == P.SPPC_E_ARG
    # the context still works after the refusals
    P.sppc_correct(ctx, P.SPPC_CORR_PERTURBATIVE)
    th, rr, added = P.sppc_rayleigh_ritz(ctx)
    assert added == w.k
    P.sppc_destroy(ctx)


@pytest.mark.parametrize("pw", [0, 1000])
def test_values_that_float32_cannot_hold(P, pw):
    """float64 values that are not float32-exact: the library keeps float64 values for the float64
    products and a rounded float32 copy for the mixed form's products.  Products with float64 X use
    the exact values (1e-14), products with float32 X the rounded ones (each value and each product
    rounded once: 2 * 2^-24); plain and mixed solves reach the dense eigenvalues of the exact H
    (1e-10, 1e-8) with the true residual (float64 H, recomputed here) below the tolerance.  With
    pw = 1000 the products run over the column-panel copy, which then holds float64 values (and the
    rounded float32 ones in the mixed form)."""
    A = levelgen.WORKLOADS[0].generate()
    rng = np.random.default_rng(33)
    v64 = A.val.astype(np.float64) * (1.0 + 1e-7 * rng.standard_normal(A.val.size))
    assert np.any(v64.astype(np.float32).astype(np.float64) != v64)
    print("case edge float64 values n=%d panel width %d" % (A.n, pw), flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, v64, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:4]
    rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, np.int64)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(A.col, np.int32)).cuda()
    val = torch.from_numpy(v64).cuda()
    X = rng.standard_normal((A.n, 8))
    scale = abs(H) @ np.abs(X)
    for prec, bound in ((P.SPPC_PREC_FP64, 1e-10), (P.SPPC_PREC_MIXED, 1e-8)):
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, 4, P.sppc_default_opts(precision=prec, panel_width=pw))
        Y = torch.empty((A.n, 8), dtype=torch.float64, device="cuda")
        P.sppc_spmm(ctx, torch.from_numpy(X).cuda(), Y)
        torch.cuda.synchronize()
        assert np.max(np.abs(Y.cpu().numpy() - H @ X) / scale) < 1e-14
        if prec == P.SPPC_PREC_MIXED:
            X32 = X.astype(np.float32)
            P.sppc_spmm(ctx, torch.from_numpy(X32).cuda(), Y)
            torch.cuda.synchronize()
            ref = H @ X32.astype(np.float64)
            assert np.max(np.abs(Y.cpu().numpy() - ref) / scale) < 2.01 * 2.0 ** -24
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK
        assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < bound
        Zc = Z.cpu().numpy()
        R = H @ Zc - Zc * np.array(ev)[None, :]
        assert np.max(np.linalg.norm(R, axis=0) / np.abs(ev)) < 1e-6
