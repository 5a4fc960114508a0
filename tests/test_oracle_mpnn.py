"""Pins of the float64 reference of the learned preconditioner."""
import numpy as np

import levelgen
import oracle
from oracle import mpnn


def _setup(seed=3):
    A = levelgen.generate((20, 90, 300), 14, seed)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    Aoff, d = mpnn.offdiag(H)
    lev = mpnn.level_feature(A.level_offsets, 1)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(A.n)
    x /= np.linalg.norm(x)
    theta = float(x @ (H @ x))
    r = H @ x - theta * x
    e = rng.standard_normal(A.n)
    e -= x * (x @ e)
    w = rng.standard_normal(mpnn.NPARAM) * 0.3
    return H, Aoff, d, lev, theta, r, x, e, w


def test_zero_network_is_jacobi():
    H, Aoff, d, lev, theta, r, x, e, w = _setup()
    t = mpnn.correction(np.zeros(mpnn.NPARAM), Aoff, d, lev, theta, r, x)
    ref = oracle.jacobi_correction(d, theta, r, x)
    assert np.allclose(t, ref, rtol=0, atol=1e-15 * np.abs(ref).max())


def test_gradient_matches_central_differences():
    H, Aoff, d, lev, theta, r, x, e, w = _setup()
    L, g = mpnn.loss_and_grad(w, Aoff, d, lev, theta, r, x, e)
    h = 1e-6
    num = np.empty_like(g)
    for i in range(mpnn.NPARAM):
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        lp, _ = mpnn.loss_and_grad(wp, Aoff, d, lev, theta, r, x, e)
        lm, _ = mpnn.loss_and_grad(wm, Aoff, d, lev, theta, r, x, e)
        num[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(num - g)) < 1e-6 * max(1.0, np.abs(g).max())


def test_gradient_with_basis_projection_matches_central_differences():
    H, Aoff, d, lev, theta, r, x, e, w = _setup(7)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(np.column_stack([x, rng.standard_normal((x.size, 6))]))
    e = e - Q @ (Q.T @ e)
    L, g = mpnn.loss_and_grad(w, Aoff, d, lev, theta, r, x, e, Q)
    h = 1e-6
    idx = rng.choice(mpnn.NPARAM, 60, replace=False)
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        num = (mpnn.loss_and_grad(wp, Aoff, d, lev, theta, r, x, e, Q)[0] -
               mpnn.loss_and_grad(wm, Aoff, d, lev, theta, r, x, e, Q)[0]) / (2 * h)
        assert abs(num - g[i]) < 1e-6 * max(1.0, np.abs(g).max())


def test_loss_is_zero_for_the_target_direction_and_scale_free():
    H, Aoff, d, lev, theta, r, x, e, w = _setup()
    tp, _ = mpnn.forward(w, Aoff, d, lev, theta, r, x)
    assert abs(mpnn.loss(tp, 3.7 * tp)) < 1e-14
    assert abs(mpnn.loss(tp, -tp)) < 1e-14
    assert 0.0 <= mpnn.loss(tp, e) <= 1.0
    # the projected output is orthogonal to x
    assert abs(tp @ x) < 1e-12 * np.linalg.norm(tp)


def test_messages_use_only_offdiagonal_coupling():
    H, Aoff, d, lev, theta, r, x, e, w = _setup()
    assert np.allclose(Aoff.diagonal(), 0.0)
    assert abs(abs(Aoff).sum() - (abs(H).sum() - np.abs(d).sum())) < 1e-9


def test_level_feature_hand_cases():
    # three levels, one small: 0 | 1/2 | 1 (the same as level / (L - 1) there)
    assert np.array_equal(mpnn.level_feature([0, 2, 3, 5], 1), [0, 0, 0.5, 1, 1])
    # five levels, two small: 0 0 | 1/2 | 1 1
    assert np.array_equal(mpnn.level_feature([0, 1, 2, 3, 4, 6], 2), [0, 0, 0.5, 1, 1, 1])
