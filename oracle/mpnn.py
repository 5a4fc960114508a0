"""Float64 CPU reference of the learned preconditioner -- TEST INFRASTRUCTURE ONLY.

A 2-layer message-passing network over the graph of H corrects the diagonal (Jacobi)
step of the continuation (the diagonal preconditioner of Sec. V) for one Ritz pair
(theta, x) with residual r = H x - theta x:

  features per row      f = [ r / rms(r),  (d - theta) / (1 + |theta|),  lambda(level) ]
                        lambda = min(max(level - n_small_levels + 1, 0), 2) / 2 (level_feature)
  messages              g = A f,            A = H - diag(d)   (signed, symmetric)
  layer 1 (width 32)    h = tanh(f Ws^T + g Wn^T + b1)
  layer 2               o = h ws + A (h wn) + b2
  output                t = tJ (1 + o),     tJ = r / (d - theta)  (|denominator| clamped)
  projection            t~ = t - x (x^T t)

A zero network gives exactly the Jacobi correction.  The training loss of one sample is
1 - cos^2 between t~ and the target direction e (the exact correction, see the tests).
Parameters (289, float): Ws[32x3] | Wn[32x3] | b1[32] | ws[32] | wn[32] | b2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

HID = 32
NPARAM = 289


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    Ws = w[0:96].reshape(HID, 3)
    Wn = w[96:192].reshape(HID, 3)
    b1 = w[192:224]
    ws = w[224:256]
    wn = w[256:288]
    b2 = w[288]
    return Ws, Wn, b1, ws, wn, b2


def level_feature(level_offsets, n_small_levels: int) -> np.ndarray:
    """The level input of each row (a reading of "level id" that keeps one meaning for any number
    of levels): the row's level counted from the small space, clipped to 0..2 and halved -- 0 on the
    small-space levels, 1/2 on the first level outside them, 1 on every level beyond."""
    offs = np.asarray(level_offsets, dtype=np.int64)
    lvl = np.searchsorted(offs, np.arange(offs[-1]), side="right") - 1
    return np.clip(lvl - n_small_levels + 1, 0, 2) / 2.0


def offdiag(H: sp.csr_matrix):
    d = H.diagonal()
    return (H - sp.diags(d)).tocsr(), d


def jacobi_step(d, theta, r):
    den = d - theta
    floor = 1e-2 * max(1.0, abs(theta))
    den = np.where(np.abs(den) < floor, np.where(den >= 0, floor, -floor), den)
    return r / den


def project(t, x, Q=None):
    """t - x (x^T t), or, with a basis Q (orthonormal columns, x in its span), t - Q (Q^T t)."""
    if Q is None:
        return t - x * (x @ t)
    return t - Q @ (Q.T @ t)


def forward(w, A, d, lev, theta, r, x, Q=None):
    """Returns the projected output and the intermediate values used by the backward pass."""
    Ws, Wn, b1, ws, wn, b2 = unpack(w)
    n = r.shape[0]
    sr = np.sqrt(np.mean(r * r))
    sr = sr if sr > 0 else 1.0
    f = np.stack([r / sr, (d - theta) / (1.0 + abs(theta)), lev], axis=1)
    g = A @ f
    pre = f @ Ws.T + g @ Wn.T + b1[None, :]
    h = np.tanh(pre)
    u = h @ wn
    o = h @ ws + A @ u + b2
    tJ = jacobi_step(d, theta, r)
    t = tJ * (1.0 + o)
    t_proj = project(t, x, Q)
    cache = dict(f=f, g=g, h=h, u=u, o=o, tJ=tJ, t=t)
    return t_proj, cache


def loss(t_proj, e):
    c1 = t_proj @ e
    c2 = t_proj @ t_proj
    c3 = e @ e
    return 1.0 - c1 * c1 / (c2 * c3)


def loss_and_grad(w, A, d, lev, theta, r, x, e, Q=None):
    """Loss of one sample and its gradient with respect to the 289 parameters.

    With a basis Q the output is projected onto the complement of span(Q) (only that part
    enlarges the subspace) and compared with e = (I - Q Q^T) psi.
    """
    Ws, Wn, b1, ws, wn, b2 = unpack(w)
    tp, c = forward(w, A, d, lev, theta, r, x, Q)
    c1, c2, c3 = tp @ e, tp @ tp, e @ e
    L = 1.0 - c1 * c1 / (c2 * c3)
    dtp = -(2.0 * c1 / (c2 * c3)) * e + (2.0 * c1 * c1 / (c2 * c2 * c3)) * tp
    dt = project(dtp, x, Q)                        # through the (symmetric) projection
    do = dt * c["tJ"]                              # t = tJ (1 + o)
    du = A @ do                                    # o contains A u, A symmetric
    h = c["h"]
    dws = h.T @ do
    dwn = h.T @ du
    db2 = do.sum()
    dh = np.outer(do, ws) + np.outer(du, wn)
    dpre = dh * (1.0 - h * h)
    dWs = dpre.T @ c["f"]
    dWn = dpre.T @ c["g"]
    db1 = dpre.sum(axis=0)
    grad = np.concatenate([dWs.ravel(), dWn.ravel(), db1, dws, dwn, [db2]])
    return L, grad


def correction(w, A, d, lev, theta, r, z):
    """The continuation direction with the learned step: -(I - z z^T) tJ (1 + o)."""
    tp, _ = forward(w, A, d, lev, theta, r, z)
    return -tp
