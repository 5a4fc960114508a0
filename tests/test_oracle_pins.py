"""Pins of the CPU oracle against facts fixed by the paper and by linear algebra.

Each test checks the oracle against something other than itself: closed forms
that follow from the splitting (eq. first_PC), the perturbation series of
H(c) = H0 + cV (eq. Hc, eq. exp), the Krylov space the method must reproduce
when the small space is as small as the block, dense brute force on tiny
inputs, and eigenvalue bounds for Rayleigh-Ritz pairs.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import levelgen
import oracle
from oracle import core as osp


def _H(sizes, d, seed):
    A = levelgen.generate(sizes, d, seed)
    return oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n), A


@pytest.fixture(scope="module")
def cfg0():
    w = levelgen.WORKLOADS[0]
    A = w.generate()
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam, X = np.linalg.eigh(H.toarray())
    return H, w.n0, w.k, lam, X


@pytest.fixture(scope="module")
def cfg0_run(cfg0):
    H, n0, k, lam, _ = cfg0
    return oracle.sppc(H, n0, k, oracle.Options())


# --- P2: at p = 0 the projected matrix is diag(E^(0)) because V11 = 0 (eq. split2)
def test_p0_projected_matrix_is_diag_E0(cfg0_run):
    T0 = cfg0_run.history[0]["T0"]
    assert np.allclose(T0, np.diag(cfg0_run.E0), rtol=0, atol=1e-14 * np.abs(cfg0_run.E0).max())


# --- P3: E^(1) = 0 and Psi^(1) = (H Psi^(0) - E^(0) Psi^(0)) / E^(0) (eq. first_PC)
def test_first_order_closed_form():
    H, A = _H((30, 120, 400), 24, 5)
    n0, k = 30, 3
    E, Psi = oracle.rs_corrections(H, n0, k, 2)
    assert np.max(np.abs(E[1])) < 1e-14
    Psi0 = Psi[0]
    E0 = E[0]
    expect = (H @ Psi0 - Psi0 * E0[None, :]) / E0[None, :]
    assert np.max(np.abs(Psi[1] - expect)) < 1e-14 * np.max(np.abs(expect))


# --- P4: E^(2) = ||V21 psi||^2 / E^(0) (eq. exp_seq with eq. first_PC)
def test_second_order_energy_closed_form():
    H, A = _H((30, 120, 400), 24, 6)
    n0, k = 30, 3
    E, Psi = oracle.rs_corrections(H, n0, k, 2)
    Hd = H.toarray()
    V21 = Hd[n0:, :n0]
    w, U = np.linalg.eigh(Hd[:n0, :n0])
    e2 = np.sum((V21 @ U[:, :k]) ** 2, axis=0) / w[:k]
    assert np.allclose(E[2], e2, rtol=1e-13, atol=0)


# --- P5: the energy series of H(c) = H0 + cV is reproduced order by order (eq. Hc, eq. exp)
def _series_slopes(H, n0, k, P, c):
    E, _ = oracle.rs_corrections(H, n0, k, P)
    Hd = H.toarray()
    H0 = np.zeros_like(Hd)
    H0[:n0, :n0] = Hd[:n0, :n0]
    V = Hd - H0
    out = []
    for cc in (c, c / 2):
        exact = np.linalg.eigvalsh(H0 + cc * V)[:k]
        partial = sum(cc ** p * E[p] for p in range(P + 1))
        out.append(np.abs(exact - partial))
    return out[0] / out[1]


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_perturbation_series_order(P):
    H, _ = _H((12, 60, 150), 10, 3)
    ratio = _series_slopes(H, 12, 2, P, 0.04)
    # the truncation error must scale like c^(P+1)
    assert np.all(ratio > 2 ** (P + 1) * 0.75) and np.all(ratio < 2 ** (P + 1) * 1.33), ratio


def test_series_pin_catches_a_dropped_sum_term(monkeypatch):
    """Plant a mistake in the oracle (drop the sum over lower orders): the series pin must fail.

    The sum first changes Psi^(3) (its l = 0 term is projected out), hence E^(4): P = 5 sees it.
    """
    def broken(VPsi_prev, E_hist, Psi_hist, p):
        return -VPsi_prev.copy()
    monkeypatch.setattr(osp, "correction_rhs", broken)
    H, _ = _H((12, 60, 150), 10, 3)
    ratio = _series_slopes(H, 12, 2, 5, 0.04)
    assert not (np.all(ratio > 2 ** 6 * 0.75) and np.all(ratio < 2 ** 6 * 1.33))


# --- P13: the block shortcut (eqs. bl_diag, sm_first, sm_lin_proj) equals the dense
#          full-space minimum-norm solve of eq. exp_seq with psi_k projected out
def test_block_split_equals_dense_pseudoinverse():
    H, _ = _H((20, 80, 200), 16, 9)
    n0, k, P = 20, 3, 4
    E, Psi = oracle.rs_corrections(H, n0, k, P)
    Hd = H.toarray()
    n = Hd.shape[0]
    H0 = np.zeros_like(Hd)
    H0[:n0, :n0] = Hd[:n0, :n0]
    V = Hd - H0
    for kk in range(k):
        w, U = np.linalg.eigh(Hd[:n0, :n0])
        psi0 = np.zeros(n)
        psi0[:n0] = U[:, kk] * np.sign(U[np.argmax(np.abs(U[:, kk])), kk])
        Ek = w[kk]
        A = np.linalg.pinv(H0 - Ek * np.eye(n), rcond=1e-12)
        Pj = np.eye(n) - np.outer(psi0, psi0)
        ps = [psi0]
        es = [Ek, psi0 @ V @ psi0]
        for p in range(1, P + 1):
            if p >= 2:
                es.append(ps[p - 1] @ V @ psi0)
            rhs = (es[1] * np.eye(n) - V) @ ps[p - 1]
            for l in range(0, p - 1):
                rhs = rhs + es[p - l] * ps[l]
            ps.append(A @ (Pj @ rhs))
            assert np.allclose(ps[p], Psi[p][:, kk], rtol=0, atol=1e-11 * np.abs(ps[p]).max())


# --- P6: with n0 = k the SPPC subspace is the block Krylov space K_{p+1}(H, Psi^(0))
@pytest.mark.parametrize("k", [1, 3])
def test_tiny_small_space_gives_block_krylov(k):
    H, _ = _H((k, 50, 160), 14, 21 + k)
    res = oracle.sppc(H, k, k, oracle.Options(continuation=False, maxiter=5, tol=1e-300,
                                               final_check=False))
    Hd = H.toarray()
    X = np.zeros((Hd.shape[0], k))
    X[:k, :k] = np.linalg.eigh(Hd[:k, :k])[1]
    blocks = [X]
    for p in range(1, 6):
        Y = Hd @ blocks[-1]
        B = np.hstack(blocks)
        for _ in range(2):
            Y = Y - B @ (B.T @ Y)
        Y, _ = np.linalg.qr(Y)
        blocks.append(Y)
        Qk = np.hstack(blocks)
        ritz = np.linalg.eigvalsh(Qk.T @ Hd @ Qk)[:k]
        th = res.history[p]["theta"]
        assert np.allclose(th, ritz, rtol=1e-12, atol=0), (p, th, ritz)


# --- P7: 2 x 2 with n0 = 1 is exact after one correction
def test_two_by_two_closed_form():
    a, b, d = -1.3, 0.7, 2.9
    H = sp.csr_matrix(np.array([[a, b], [b, d]]))
    res = oracle.sppc(H, 1, 1, oracle.Options(tol=1e-300, maxiter=1, continuation=False,
                                              final_check=False))
    exact = (a + d) / 2 - np.sqrt(((a - d) / 2) ** 2 + b ** 2)
    assert abs(res.history[1]["theta"][0] - exact) < 1e-15 * 4


# --- P1: Rayleigh-Ritz bounds: theta_i >= lambda_i, monotone in p (nested subspaces)
def test_interlacing_and_monotone(cfg0, cfg0_run):
    lam = cfg0[3][:cfg0[2]]
    prev = None
    for h in cfg0_run.history:
        th = h["theta"]
        assert np.all(th >= lam - 1e-13 * np.abs(lam))
        if prev is not None:
            assert np.all(th <= prev + 1e-13 * np.abs(prev))
        prev = th


def test_full_space_is_exact():
    H, _ = _H((6, 12, 20), 8, 4)
    n = H.shape[0]
    res = oracle.sppc(H, 6, 2, oracle.Options(tol=1e-300, maxiter=60, continuation=False,
                                              final_check=False))
    assert res.history[-1]["m"] == n
    lam = np.linalg.eigvalsh(H.toarray())[:2]
    assert np.allclose(res.history[-1]["theta"], lam, rtol=1e-13, atol=0)


# --- P9: orthonormal basis
def test_basis_orthonormal(cfg0_run):
    Q = cfg0_run.Q
    assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) < 1e-12


# --- P10: decoupled blocks (V12 = 0) or n0 = n converge at p = 0
def test_decoupled_converges_at_p0():
    H, _ = _H((20, 60, 100), 12, 8)
    Hd = H.toarray()
    Hd[:20, 20:] = 0.0
    Hd[20:, :20] = 0.0
    Hd[20:, 20:] += 20.0 * np.eye(Hd.shape[0] - 20)   # keep the wanted pairs in the small block
    res = oracle.sppc(sp.csr_matrix(Hd), 20, 3, oracle.Options())
    assert res.history[-1]["p"] == 0 and np.all(res.rrn < 1e-13)
    H2, _ = _H((40,), 10, 8)
    res2 = oracle.sppc(H2, 40, 3, oracle.Options())
    assert res2.history[-1]["p"] == 0 and np.all(res2.rrn < 1e-12)


# --- P11: converged pairs obey the residual and Kato-Temple bounds and equal eigh's
def test_converged_pairs_bounds(cfg0, cfg0_run):
    H, n0, k, lam, X = cfg0
    res = cfg0_run
    assert res.converged
    for i in range(k):
        r = np.linalg.norm(H @ res.Z[:, i] - res.theta[i] * res.Z[:, i])
        assert abs(res.theta[i] - lam[i]) <= r
        a = lam[i - 1] if i > 0 else -np.inf
        b = lam[i + 1]
        assert res.theta[i] - r * r / (b - res.theta[i]) <= lam[i] + 1e-14
        if np.isfinite(a):
            assert lam[i] <= res.theta[i] + r * r / (res.theta[i] - a) + 1e-14
        assert abs(res.theta[i] - lam[i]) / abs(lam[i]) < 1e-10
        assert res.rrn[i] < 1e-6


# --- P12: k products with H per SPPC step (Sec. IV.B-C)
def test_spmv_accounting(cfg0_run):
    k = len(cfg0_run.theta)
    for h in cfg0_run.history:
        if h["phase"] == "sppc":
            assert h["n_spmv"] == k * (h["p"] + 1)


# --- P14: stagnation of pure SPPC (Sec. VI): angles decay, residual stalls above 1e-6
def test_stagnation_pattern(cfg0):
    H, n0, k, lam, _ = cfg0
    res = oracle.sppc(H, n0, k, oracle.Options(continuation=False, maxiter=30, final_check=False))
    ang = [np.min(h["angles"]) for h in res.history[1:]]
    assert ang[14] < 1e-5 and ang[14] < ang[4] * 1e-3
    assert not res.converged and res.history[-1]["rrn"].max() > 1e-6
    assert res.history[15]["rrn"].max() < res.history[0]["rrn"].max() * 1e-2


# --- zero E^(0) is refused (eq. sm_first divides by it)
def test_zero_E0_refused():
    Hd = np.diag([0.0, 1.0, 5.0, 6.0])
    Hd[0, 2] = Hd[2, 0] = 0.3
    with pytest.raises(ZeroDivisionError):
        oracle.sppc(sp.csr_matrix(Hd), 2, 1, oracle.Options())


# ---------------------------------------------------------------- small-space preconditioner
def test_small_space_correction_vanishes_for_rayleigh_quotient_when_the_small_space_is_everything():
    # with n0 = n the preconditioner is (H - theta)^-1 and (H - theta)^-1 (H z - theta z) = z, so
    # the projected correction -(I - z z^T) z is exactly zero (Rayleigh quotient iteration)
    A = levelgen.generate((30, 60), 12, 5)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    rng = np.random.default_rng(0)
    z = rng.standard_normal(A.n)
    z /= np.linalg.norm(z)
    theta = float(z @ (H @ z))
    r = H @ z - theta * z
    t = oracle.small_space_correction(H, A.n, theta, r, z)
    # |t| ~ eps * cond(H - theta) * |z|, cond ~ 1e2 here
    assert np.linalg.norm(t) < 1e-12


def test_small_space_correction_is_the_diagonal_step_off_the_small_space():
    # decoupled H (no entries between the first n0 rows and the rest) and z supported off the
    # small space: the small-space rows of r vanish, the step is the diagonal one
    A = levelgen.generate((20, 80), 10, 6)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n).tolil()
    n0 = 20
    H[:n0, n0:] = 0.0
    H[n0:, :n0] = 0.0
    H = H.tocsr()
    rng = np.random.default_rng(1)
    z = np.zeros(A.n)
    z[n0:] = rng.standard_normal(A.n - n0)
    z /= np.linalg.norm(z)
    theta = float(z @ (H @ z))
    r = H @ z - theta * z
    t = oracle.small_space_correction(H, n0, theta, r, z)
    ref = oracle.jacobi_correction(H.diagonal(), theta, r, z)
    assert np.allclose(t, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_product_from_upper_matches_the_dense_symmetric_matrix():
    # the block product from the upper triangle equals the product with the full symmetric matrix
    # written out entry by entry (brute force on a small ragged case, diagonal entries present
    # and absent)
    rng = np.random.default_rng(11)
    n = 37
    rows, cols, vals = [], [], []
    for i in range(n):
        js = sorted(set([i] * (i % 3 != 0) + list(rng.integers(i, n, size=4))))
        for j in js:
            rows.append(i)
            cols.append(j)
            vals.append(rng.standard_normal())
    rp = np.zeros(n + 1, dtype=np.int64)
    for i in rows:
        rp[i + 1] += 1
    rp = np.cumsum(rp)
    Hd = np.zeros((n, n))
    for i, j, v in zip(rows, cols, vals):
        Hd[i, j] = v
        Hd[j, i] = v
    X = rng.standard_normal((n, 5))
    Y = oracle.product_from_upper(rp, np.array(cols), np.array(vals), n, X)
    assert np.max(np.abs(Y - Hd @ X)) < 1e-13
    # single rows from the definition: every row, a repeated row, and unsorted order
    rows = np.concatenate([np.arange(n), [5, 5, 36, 0]])[::-1]
    Yr = oracle.product_rows_from_upper(rp, np.array(cols, dtype=np.int32), np.array(vals), n, X, rows)
    assert np.max(np.abs(Yr - (Hd @ X)[rows])) < 1e-13
    # the full matrix the oracle solves: every entry of symmetric_from_upper equals the matrix
    # written out entry by entry (a doubled or a missing diagonal, or a dropped mirror, fails)
    Hs = oracle.symmetric_from_upper(rp, np.array(cols, dtype=np.int32), np.array(vals), n).toarray()
    assert np.array_equal(Hs, Hd)
    # the ragged case has rows with and without a stored diagonal entry
    assert any(Hd[i, i] == 0.0 for i in range(n)) and any(Hd[i, i] != 0.0 for i in range(n))


def test_symmetric_from_upper_hand_case():
    # 3 x 3 upper triangle [[2, -1, 0.5], [., 0 (absent), 4], [., ., -3]] written by hand
    rp = np.array([0, 3, 4, 5], dtype=np.int64)
    col = np.array([0, 1, 2, 2, 2], dtype=np.int32)
    val = np.array([2.0, -1.0, 0.5, 4.0, -3.0])
    H = oracle.symmetric_from_upper(rp, col, val, 3).toarray()
    want = np.array([[2.0, -1.0, 0.5], [-1.0, 0.0, 4.0], [0.5, 4.0, -3.0]])
    assert np.array_equal(H, want)
    X = np.array([[1.0], [2.0], [-1.0]])
    assert np.array_equal(oracle.product_from_upper(rp, col, val, 3, X), want @ X)


# --- the diagonal step of the continuation (Sec. V names a diagonal preconditioner): a 5 x 5 case
# computed by hand, with one denominator clamped up to +floor, one clamped down to -floor and the
# projection against the Ritz vector
def test_jacobi_correction_hand_case():
    d = np.array([1.0, 2.0, 3.004, 2.99, -1.0])
    theta = 3.0                      # floor = 1e-2 * max(1, |theta|) = 0.03
    r = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    z = np.array([0.6, 0.8, 0.0, 0.0, 0.0])
    # d - theta = [-2, -1, 0.004, -0.01, -4] -> clamped [-2, -1, 0.03, -0.03, -4]
    # M r = [-0.5, -2, 100, -400/3, -1.25];  z . M r = -1.9
    # (I - z z^T) M r = [0.64, -0.48, 100, -400/3, -1.25];  t = -that
    want = np.array([-0.64, 0.48, -100.0, 400.0 / 3.0, 1.25])
    t = oracle.jacobi_correction(d, theta, r, z)
    assert np.allclose(t, want, rtol=1e-14, atol=1e-14)
    # |theta| < 1: the floor is 1e-2 (not 1e-2 |theta|); d - theta = 0.005 -> +0.01
    t = oracle.jacobi_correction(np.array([-0.495, 1.5]), -0.5, np.array([1.0, 1.0]), np.array([0.0, 1.0]))
    assert np.allclose(t, [-100.0, 0.0], rtol=1e-14, atol=1e-14)
    # the RMM-DIIS step uses the same clamped diagonal, without the projection
    assert np.allclose(oracle.core.diag_precond(d, theta, r), [-0.5, -2.0, 100.0, -400.0 / 3.0, -1.25],
                       rtol=1e-14, atol=1e-14)


# ------------------------------------------------------------------ RMM-DIIS (the hybrid's continuation)

def test_diis_coefficients_are_the_constrained_minimiser():
    # two residuals: the minimiser of |a1 r1 + a2 r2| with a1 + a2 = 1 in closed form, and for
    # three a brute-force scan of the constraint plane
    rng = np.random.default_rng(21)
    R = rng.standard_normal((50, 2))
    A = R.T @ R
    a = oracle.core.diis_coefficients(A)
    t = (A[1, 1] - A[0, 1]) / (A[0, 0] + A[1, 1] - 2 * A[0, 1])
    assert abs(a.sum() - 1.0) < 1e-14 and abs(a[0] - t) < 1e-12
    R = rng.standard_normal((50, 3))
    A = R.T @ R
    a = oracle.core.diis_coefficients(A)
    f = a @ A @ a
    g = np.linspace(-3, 3, 241)
    best = min((x * x * A[0, 0] + y * y * A[1, 1] + (1 - x - y) ** 2 * A[2, 2] + 2 * x * y * A[0, 1]
                + 2 * x * (1 - x - y) * A[0, 2] + 2 * y * (1 - x - y) * A[1, 2]) for x in g for y in g)
    assert abs(a.sum() - 1.0) < 1e-14 and f <= best + 1e-12


def test_rmm_diis_step_minimises_the_residual_along_the_direction():
    # one iteration from x0: the new iterate is x0 + lam t (normalised) with t the preconditioned
    # residual and lam minimising |R0 + lam (H - theta0) t| (checked against a fine scan of lam)
    rng = np.random.default_rng(4)
    n = 40
    Hd = np.diag(np.arange(n, dtype=float)) + 0.05 * (lambda B: B + B.T)(rng.standard_normal((n, n)))
    H = sp.csr_matrix(Hd)
    x0 = np.zeros(n); x0[0] = 1.0; x0 += 0.05 * rng.standard_normal(n)
    x0 /= np.linalg.norm(x0)
    th0 = x0 @ Hd @ x0
    R0 = Hd @ x0 - th0 * x0
    t = oracle.core.diag_precond(Hd.diagonal(), th0, R0)
    u = Hd @ t - th0 * t
    lams = np.linspace(-3, 3, 60001)
    res = [np.linalg.norm(R0 + l * u) for l in lams]
    lam_scan = lams[int(np.argmin(res))]
    th, x, hx, rrn, prods, its = oracle.core.rmm_diis(H, Hd.diagonal(), x0, Hd @ x0, 0.0, 1)
    xn = x0 + (-(R0 @ u) / (u @ u)) * t
    assert prods == 1 and abs(-(R0 @ u) / (u @ u) - lam_scan) < 2e-4
    # with two iterates in the history the returned vector is their DIIS combination; after one
    # iteration (max_iter = 1) it is the combination of x0 and the new iterate
    assert abs(abs(x @ (xn / np.linalg.norm(xn))) - 1.0) < 0.05


def test_rmm_diis_converges_to_the_eigenpair_it_starts_near():
    # a diagonally dominant matrix (the diagonal preconditioner is good): from a perturbed
    # eigenvector RMM-DIIS reaches that eigenpair to 1e-12, one product per iteration
    rng = np.random.default_rng(8)
    n = 300
    B = sp.random(n, n, density=0.03, random_state=np.random.RandomState(3))
    Hs = (sp.diags(np.linspace(1.0, 30.0, n)) + 0.1 * (B + B.T)).tocsr()
    w, U = np.linalg.eigh(Hs.toarray())
    for j in (0, 3):
        x0 = U[:, j] + 1e-3 * rng.standard_normal(n)
        th, x, hx, rrn, prods, its = oracle.core.rmm_diis(Hs, Hs.diagonal(), x0, Hs @ x0, 1e-12, 200)
        assert rrn < 1e-12 and prods == its
        assert abs(th - w[j]) < 1e-11 * abs(w[j]) and abs(abs(x @ U[:, j]) - 1.0) < 1e-12


def test_hybrid_sppc_rmm_diis_reaches_the_eigenvalues():
    # SPPC + RMM-DIIS (sweeps of 4 iterations, Rayleigh-Ritz between sweeps) on a small
    # level-structured matrix: the same eigenvalues as dense eigh within the Kato-Temple bound
    A = levelgen.generate((100, 1000, 7000), 60, 13)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:3]
    r = oracle.sppc(H, 100, 3, oracle.Options(tol=1e-9, rmm_diis=True, max_cont=400))
    assert r.converged and any(h["phase"] == "rmmdiis" for h in r.history)
    assert np.max(np.abs(r.theta - lam) / np.abs(lam)) < 1e-12


def test_rmm_stagnation_rule():
    # the largest residual after each sweep (top[0]: at the switch) must halve within three sweeps
    f = oracle.core.rmm_stagnated
    assert not f([1.0, 0.9, 0.8])                 # fewer than three sweeps
    assert f([1.0, 0.9, 0.8, 0.5])                # exactly half is not below half
    assert not f([1.0, 0.9, 0.8, 0.49])
    assert f([1.0, 0.1, 0.09, 0.08, 0.06])        # against three sweeps back, not the switch


def test_hybrid_hands_over_where_rmm_diis_stagnates():
    # Pair 4 of this five-level matrix is interior (three eigenvalues below its Ritz value, and one
    # diagonal entry): the minimal-residual step along its diagonally preconditioned residual turns
    # orthogonal to that residual once a sweep restarts the DIIS history, and RMM-DIIS alone holds it
    # near 2e-6 for all 200 iterations.  The sweeps stagnate, the Davidson continuation takes over
    # from the refined Ritz vectors and reaches the eigenvalues of ARPACK's Lanczos (shift-free,
    # smallest algebraic) to the Kato-Temple bound.
    from scipy.sparse.linalg import eigsh
    A = levelgen.generate((7, 61, 509, 3001, 7919), 30, 505)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.sort(eigsh(H, k=4, which="SA", tol=1e-14, v0=np.ones(A.n))[0])
    r = oracle.sppc(H, int(A.level_offsets[2]), 4, oracle.Options(tol=1e-6, rmm_diis=True, max_cont=200))
    phases = [h["phase"] for h in r.history]
    assert r.converged and "cont" in phases
    i = phases.index("cont")
    assert "rmmdiis" in phases[:i] and set(phases[i:]) == {"cont"}
    top = [max(h["rrn"]) for h in r.history if h["phase"] in ("sppc", "rmmdiis")][-(phases.count("rmmdiis") + 1):]
    assert oracle.core.rmm_stagnated(top) and not oracle.core.rmm_stagnated(top[:-1])
    assert top[-1] > 1e-6  # stalled above the tolerance
    assert np.max(np.abs(r.theta - lam) / np.abs(lam)) < 1e-12


# --- the stagnation diagnostic of Fig. 3: the recorded angle of each correction vector is the sine
# of its principal angle to the span of all earlier correction vectors (LAPACK-based
# scipy.linalg.subspace_angles on the raw vectors of the Rayleigh-Schrodinger recursion)
def test_recorded_angles_are_sines_of_principal_angles(cfg0):
    import scipy.linalg as sla
    H, n0, k, lam, _ = cfg0
    res = oracle.sppc(H, n0, k, oracle.Options(continuation=False, maxiter=8, final_check=False))
    _, Psi = oracle.rs_corrections(H, n0, k, 8)
    for p in (1, 3, 6, 8):
        prev = np.hstack(Psi[:p])
        want = [np.sin(sla.subspace_angles(Psi[p][:, [j]], prev)[0]) for j in range(k)]
        assert np.allclose(res.history[p]["angles"], want, rtol=1e-6, atol=1e-14), p


# --- the automatic switch (Sec. VII leaves it open; the rule is a reading): the run with it is the
# fixed-switch run up to the first step whose record meets the rule, then continues from there
# and still reaches the eigenvalues of dense eigh
@pytest.mark.parametrize("case", ["cfg0", "four_levels"])
def test_automatic_switch_stops_at_the_first_stagnated_step(cfg0, case):
    if case == "cfg0":
        H, n0, k, lam, _ = cfg0
    else:
        import scipy.sparse.linalg as spla
        H, A = _H((40, 400, 3000, 8000), 60, 5)
        n0, k = 440, 4
        lam = np.sort(spla.eigsh(H, k=k, which="SA", tol=1e-14)[0])
    full = oracle.sppc(H, n0, k, oracle.Options(continuation=False, maxiter=15, final_check=False))
    first = None
    for p in range(1, 16):
        top = [np.max(h["rrn"]) for h in full.history[:p + 1]]
        if np.min(full.history[p]["angles"]) < 1e-4 or (p >= 3 and top[p] >= 0.5 * top[p - 3]):
            first = p
            break
    assert first is not None and first < 15
    auto = oracle.sppc(H, n0, k, oracle.Options(auto_switch=True))
    steps = [h for h in auto.history if h["phase"] == "sppc"]
    assert steps[-1]["p"] == first
    for a, b in zip(steps, full.history[:first + 1]):
        assert np.array_equal(a["theta"], b["theta"]) and a["m"] == b["m"]
    assert auto.converged and np.max(auto.rrn) < 1e-6
    assert np.max(np.abs(auto.theta - lam[:k]) / np.abs(lam[:k])) < 1e-9


# ------------------------------------------------------------------ shifted small-space corrections
def test_shifted_small_solve_equals_the_dense_projected_solve():
    # the shifted form of eq. sm_lin_proj: x1 = P (H0hat - sigma)^-1 P b1 with P = I - psi_k psi_k^T
    # (H0hat - sigma commutes with P), by a dense LU solve instead of the spectral sum; sigma = E_k^(0)
    # is the paper's singular case, where the minimum-norm solution is the pseudo-inverse's
    rng = np.random.default_rng(31)
    A = levelgen.generate((40, 200), 16, 31)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    n0 = 40
    H0 = H[:n0, :n0].toarray()
    z = osp.zeroth_order(H0)
    b1 = rng.standard_normal(n0)
    for kk, sigma in ((0, z.w[0] - 0.3), (2, z.w[2] - 0.01), (1, z.w[0] + 0.2)):
        P_ = np.eye(n0) - np.outer(z.U[:, kk], z.U[:, kk])
        want = P_ @ np.linalg.solve(H0 - sigma * np.eye(n0), P_ @ b1)
        got = osp.small_solve(z, kk, b1, sigma)
        assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want)), (kk, sigma)
    kk = 1
    P_ = np.eye(n0) - np.outer(z.U[:, kk], z.U[:, kk])
    want = np.linalg.pinv(H0 - z.w[kk] * np.eye(n0), rcond=1e-12) @ (P_ @ b1)
    assert np.allclose(osp.small_solve(z, kk, b1), want, rtol=0, atol=1e-10 * np.max(np.abs(want)))
    assert np.array_equal(osp.small_solve(z, kk, b1), osp.small_solve(z, kk, b1, z.w[kk]))


def test_theta_shifted_variant_with_E0_shifts_is_the_paper_recursion(cfg0):
    # passing shifts equal to E^(0) reproduces the default recursion exactly
    H, n0, k, lam, _ = cfg0
    H0 = osp.small_space_matrix(H, n0)
    z = osp.zeroth_order(H0)
    Psi0 = np.zeros((H.shape[0], k))
    Psi0[:n0] = z.U[:, :k]
    VPsi0 = H @ Psi0 - osp.apply_H0(H0, Psi0)
    E_hist = [z.w[:k].copy(), np.zeros(k)]
    a = osp.correction_vectors(H, H0, z, k, E_hist[:1], [Psi0], VPsi0)
    b = osp.correction_vectors(H, H0, z, k, E_hist[:1], [Psi0], VPsi0, shifts=z.w[:k].copy())
    assert np.array_equal(a[1], b[1])


# ------------------------------------------------------------------ Alg. 1 (one pair alone)
def test_pair_zero_is_the_single_pair_run(cfg0):
    H, n0, k, lam, _ = cfg0
    o = oracle.Options(continuation=False, maxiter=8, tol=1e-300, final_check=False)
    a = oracle.sppc_pair(H, n0, 0, o)
    b = oracle.sppc(H, n0, 1, o)
    for ha, hb in zip(a.history, b.history):
        assert np.array_equal(ha["theta"], hb["theta"])


@pytest.mark.parametrize("kk", [1, 3])
def test_pair_subspace_brute_force(cfg0, kk):
    # Alg. 1's Ritz value after step P is the lowest eigenvalue of H on span{Psi_kk^(0..P)}, the
    # raw Rayleigh-Schroedinger corrections of eq. exp_seq for pair kk (column kk of the k-pair
    # recursion): one orthonormalisation and one dense eigensolve at the end, no per-step
    # Gram-Schmidt, QR or Rayleigh-Ritz
    H, n0, k, lam, _ = cfg0
    P = 6
    E, Psi = oracle.rs_corrections(H, n0, kk + 1, P)
    run = oracle.sppc_pair(H, n0, kk, oracle.Options(continuation=False, maxiter=P, tol=1e-300,
                                                      final_check=False))
    for p in range(P + 1):
        B = np.stack([Psi[l][:, kk] for l in range(p + 1)], axis=1)
        Q, _ = np.linalg.qr(B)
        want = np.linalg.eigvalsh(Q.T @ (H @ Q))[0]
        got = run.history[p]["theta"][0]
        assert abs(got - want) <= 1e-11 * abs(want), (p, got, want)
        assert got >= lam[0] - 1e-12 * abs(lam[0])   # a Ritz value bounds lambda_1 from above
    th = [h["theta"][0] for h in run.history]
    assert np.all(np.diff(th) <= 1e-12 * abs(th[0]))   # nested subspaces: non-increasing


def test_pair_is_exact_when_the_small_space_is_everything():
    A = levelgen.generate((30, 50), 12, 12)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())
    r = oracle.sppc_pair(H, A.n, 2, oracle.Options(continuation=False, maxiter=3))
    assert r.history[0]["rrn"][0] < 1e-12 and abs(r.theta[0] - lam[2]) < 1e-12 * abs(lam[2])
