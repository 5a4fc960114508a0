"""FP64 CPU oracle of SPPC -- test infrastructure only (see the package docstring).

Follows the paper step by step:

* split H = H0 + V with H0 = diag(H0hat, 0), V11 = 0          (Sec. II, eq. split2)
* zeroth order: eigenpairs of H0hat, zero-padded               (Alg. 2 step 1; eq. EP_small)
* p = 0: Rayleigh-Ritz on span(Psi^(0))                        (Alg. 2 steps 2-4)
* p >= 1, for each wanted pair k separately:
    E_k^(p) = Psi_k^(p-1)^T V Psi_k^(0)                        (eq. exp_seq, first line)
    b = -V Psi_k^(p-1) + sum_{l=0}^{p-2} E_k^(p-l) Psi_k^(l)   (eq. exp_seq2)
    x2 = -b2 / E_k^(0)                                         (eq. sm_first)
    (H0hat - E_k^(0)) x1 = b1 - (b1^T psi_k) psi_k             (eq. sm_lin_proj)
  then block Gram-Schmidt + QR of the new block, append to Q   (eqs. blkGS, QR, Qp)
  and Rayleigh-Ritz on the whole combined subspace             (eq. tilde_H, eq. comb_sub)
* convergence: ||H z - theta z|| / |theta| < tol for every pair (eq. rrn)

Everything is float64.  H-products are direct sparse products (the oracle does
not use the stored-HQ identity of Sec. IV.C, so that identity can be tested
against it).  The singular small system is solved exactly through the full
eigendecomposition of H0hat (minimum-norm solution orthogonal to psi_k).

Readings where the paper is silent (each one is listed with its reason in the
design notes of the repository):
  * the k lowest eigenpairs of H0hat are the zeroth order; |E_k^(0)| must be
    nonzero because eq. sm_first divides by it;
  * x1 is the minimum-norm solution, orthogonal to psi_k (intermediate
    normalisation, which the E^(p) formula presupposes); eigenvectors of H0hat
    whose eigenvalue equals E_k^(0) to 1e-12 relative are excluded as well;
  * classical Gram-Schmidt applied twice, then Householder QR; a new column
    whose remaining norm is <= tau_drop times its original norm is dropped;
  * T is symmetrised as (T + T^T)/2;
  * after p_switch SPPC steps without convergence (stagnation, Sec. V-VI), the
    subspace keeps growing with preconditioned residual blocks
    t_i = -(I - z_i z_i^T) M_i r_i for the unconverged pairs (a generalised
    Davidson continuation; M_i = diag(H) - theta_i with a clamped denominator
    is the diagonal preconditioner named in Sec. V);
  * a final explicit product H Z, Rayleigh-Ritz on span Z and the true
    residual certify the returned pairs;
  * the hybrid of Sec. V-VI refines each unconverged pair by RMM-DIIS in sweeps
    of 4 iterations with Rayleigh-Ritz on the refined vectors between sweeps;
    when the largest residual has not halved over three sweeps (rmm_stagnated)
    the refined Ritz vectors hand over to the Davidson continuation above;
  * optionally the switch comes early, once SPPC stagnates (sppc_stagnated;
    the paper leaves the detection open, Sec. VII);
  * Alg. 1 (sppc_pair): the same iteration for one pair alone, its zeroth order
    the kk-th eigenpair of H0hat and its approximation the lowest Ritz pair of
    the span of its own corrections;
  * optionally (Options.shift = "ritz") the small-space corrections use the Ritz
    value theta_k of the step before in place of E_k^(0) in eq. sm_first and
    eq. sm_lin_proj (the "(H11 - theta I) z = r" form), with the right-hand side
    of eq. exp_seq2 and E^(p) unchanged.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


# --------------------------------------------------------------------------- input


def symmetric_from_upper(row_ptr, col, val, n) -> sp.csr_matrix:
    """Full symmetric float64 CSR from the upper triangle (diagonal included)."""
    U = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)),
                      shape=(n, n))
    H = U + U.T - sp.diags(U.diagonal())
    H = H.tocsr()
    H.sort_indices()
    return H


def product_from_upper(row_ptr, col, val, n, X) -> np.ndarray:
    """Y = H X for the symmetric H given by its upper triangle (diagonal included): the block
    product with H that Sec. IV.C counts as the cost unit.  Y = U X + U^T X - diag(U) X, in
    float64, without forming the lower triangle."""
    U = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)),
                      shape=(n, n))
    X = np.asarray(X, dtype=np.float64)
    return U @ X + U.T @ X - U.diagonal()[:, None] * X


def product_rows_from_upper(row_ptr, col, val, n, X, rows) -> np.ndarray:
    """Rows `rows` of H X, each from its definition (H X)_i = sum_j H_ij X_j with H_ij = U_ij for
    j >= i and U_ji for j < i, in float64.  The entries of row i below the diagonal are the stored
    entries of column i, found by one pass over the column indices, so the cost is one pass over
    the matrix however many rows are asked for (the check of sampled rows at sizes where the full
    product is too slow on the CPU)."""
    rows, back = np.unique(np.asarray(rows, dtype=np.int64), return_inverse=True)
    row_ptr = np.asarray(row_ptr)
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((rows.size, X.shape[1]))
    for a, i in enumerate(rows):          # j >= i: row i of the upper triangle
        s, e = int(row_ptr[i]), int(row_ptr[i + 1])
        out[a] = np.asarray(val[s:e], dtype=np.float64) @ X[np.asarray(col[s:e], dtype=np.int64)]
    wanted = np.zeros(n, dtype=bool)       # j < i: stored entries (j, i) with j < i
    wanted[rows] = True
    slot = np.full(n, -1, dtype=np.int64)
    slot[rows] = np.arange(rows.size)
    hit = np.flatnonzero(wanted[col])
    owner = np.searchsorted(row_ptr, hit, side="right") - 1
    below = owner < np.asarray(col)[hit]
    hit, owner = hit[below], owner[below]
    np.add.at(out, slot[np.asarray(col)[hit]], np.asarray(val, dtype=np.float64)[hit][:, None] * X[owner])
    return out[back.ravel()]


def small_space_matrix(H: sp.csr_matrix, n0: int) -> np.ndarray:
    """H0hat: the leading n0 x n0 block of H, dense (eq. split2)."""
    return H[:n0, :n0].toarray()


def apply_H0(H0hat: np.ndarray, X: np.ndarray) -> np.ndarray:
    """H0 X with H0 = diag(H0hat, 0): [H0hat X1; 0] (eq. split2)."""
    n0 = H0hat.shape[0]
    Y = np.zeros_like(X)
    Y[:n0] = H0hat @ X[:n0]
    return Y


# --------------------------------------------------------------------------- zeroth order


@dataclass
class ZerothOrder:
    w: np.ndarray   # all eigenvalues of H0hat, ascending
    U: np.ndarray   # all eigenvectors (columns), signs fixed


def zeroth_order(H0hat: np.ndarray) -> ZerothOrder:
    """Full eigendecomposition of H0hat (Alg. 2 step 1, eq. EP_small).

    Sign convention: the entry of largest magnitude of each eigenvector is positive.
    """
    w, U = np.linalg.eigh(H0hat)
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return ZerothOrder(w, U * s)


def check_e0(z: ZerothOrder, k: int) -> None:
    """eq. sm_first divides by E_k^(0): it must be safely nonzero."""
    scale = max(1.0, float(np.max(np.abs(z.w))))
    if np.any(np.abs(z.w[:k]) < 1e-10 * scale):
        raise ZeroDivisionError("E^(0) is (numerically) zero: the complement block is singular")


# --------------------------------------------------------------------------- correction step


def small_solve(z: ZerothOrder, kk: int, b1: np.ndarray, shift: Optional[float] = None) -> np.ndarray:
    """Minimum-norm x1 of (H0hat - E_k^(0)) x1 = b1 - (b1^T psi_k) psi_k (eq. sm_lin_proj).

    Exact spectral form: x1 = sum_{j != k} u_j (u_j^T b1) / (w_j - E_k^(0)); eigenvalues
    equal to E_k^(0) to 1e-12 relative are treated as null directions too.  With `shift` the
    shift sigma replaces E_k^(0) in the denominators (the theta-shifted variant); psi_k is still
    projected out.
    """
    Ek = z.w[kk] if shift is None else float(shift)
    tol = 1e-12 * max(1.0, abs(Ek))
    mask = np.abs(z.w - Ek) > tol
    mask[kk] = False
    Uj = z.U[:, mask]
    return Uj @ ((Uj.T @ b1) / (z.w[mask] - Ek))


def correction_rhs(VPsi_prev: np.ndarray, E_hist: List[np.ndarray], Psi_hist: List[np.ndarray],
                   p: int) -> np.ndarray:
    """b = -V Psi^(p-1) + sum_{l=0}^{p-2} E^(p-l) Psi^(l), column by column (eq. exp_seq2)."""
    b = -VPsi_prev.copy()
    for l in range(0, p - 1):
        b += E_hist[p - l][None, :] * Psi_hist[l]
    return b


def correction_vectors(H: sp.csr_matrix, H0hat: np.ndarray, z: ZerothOrder, k: int,
                       E_hist: List[np.ndarray], Psi_hist: List[np.ndarray],
                       VPsi0: np.ndarray, shifts: Optional[np.ndarray] = None) -> tuple:
    """E^(p) and Psi^(p) for every wanted pair from the stored lower orders.

    Returns (E_p [k], Psi_p [n x k]).  Uses one direct product with H (oracle only).
    shifts (optional, [k]): sigma_k in place of E_k^(0) in eq. sm_first and eq. sm_lin_proj (the
    right-hand side of eq. exp_seq2 and E^(p) are unchanged); None is the paper's E^(0).
    """
    p = len(Psi_hist)
    n0 = H0hat.shape[0]
    Pprev = Psi_hist[p - 1]
    VPprev = H @ Pprev - apply_H0(H0hat, Pprev)            # eq. avoid_SpMV2, computed directly
    E_p = np.einsum("ij,ij->j", Pprev, VPsi0)              # eq. exp_seq: E^(p) = Psi^(p-1)^T V Psi^(0)
    E_all = E_hist + [E_p]
    b = correction_rhs(VPprev, E_all, Psi_hist, p)
    E0 = z.w[:k] if shifts is None else np.asarray(shifts, dtype=np.float64)
    Psi_p = np.empty_like(b)
    Psi_p[n0:] = -b[n0:] / E0[None, :]                     # eq. sm_first
    for kk in range(k):                                    # eq. sm_lin_proj
        Psi_p[:n0, kk] = small_solve(z, kk, b[:n0, kk], None if shifts is None else E0[kk])
    return E_p, Psi_p


def rs_corrections(H: sp.csr_matrix, n0: int, k: int, P: int):
    """Raw Rayleigh-Schroedinger corrections E^(0..P), Psi^(0..P) (eq. exp_seq), no projection.

    Used by the tests to check the recursion against H(c) = H0 + cV (eq. Hc, eq. exp).
    """
    H = sp.csr_matrix(H, dtype=np.float64)
    H0hat = small_space_matrix(H, n0)
    z = zeroth_order(H0hat)
    check_e0(z, k)
    n = H.shape[0]
    Psi0 = np.zeros((n, k))
    Psi0[:n0] = z.U[:, :k]
    VPsi0 = H @ Psi0 - apply_H0(H0hat, Psi0)
    E_hist = [z.w[:k].copy(), np.einsum("ij,ij->j", Psi0, VPsi0)]
    Psi_hist = [Psi0]
    for p in range(1, P + 1):
        E_p, Psi_p = correction_vectors(H, H0hat, z, k, E_hist[:p], Psi_hist, VPsi0)
        if p >= 2:
            E_hist.append(E_p)
        Psi_hist.append(Psi_p)
    # E^(P+1) completes the energy series through order P+1
    E_hist.append(np.einsum("ij,ij->j", Psi_hist[P], VPsi0))
    return E_hist, Psi_hist


# --------------------------------------------------------------------------- subspace


def orthonormalize_block(Q: np.ndarray, Psi: np.ndarray, tau_drop: float):
    """Block Gram-Schmidt against Q (eq. blkGS, applied twice) then QR (eq. QR).

    Returns (q, angles, kept) where angles_j = ||Phi_j|| / ||Psi_j|| is the sine of the
    angle between Psi_j and span(Q) (the stagnation diagnostic of Sec. VI), and kept
    lists the columns of Psi that contribute new directions.
    """
    nrm = np.linalg.norm(Psi, axis=0)
    nrm[nrm == 0] = 1.0
    Phi = Psi - Q @ (Q.T @ Psi)
    Phi = Phi - Q @ (Q.T @ Phi)
    angles = np.linalg.norm(Phi, axis=0) / nrm
    kept = np.nonzero(angles > tau_drop)[0]
    if kept.size == 0:
        return np.zeros((Q.shape[0], 0)), angles, kept
    q, R, piv = sla.qr(Phi[:, kept], mode="economic", pivoting=True)
    rdiag = np.abs(np.diag(R))
    ok = rdiag > tau_drop * nrm[kept[piv]]
    q = q[:, ok]
    kept = np.sort(kept[piv[ok]])
    # a second pass keeps q orthogonal to Q when the angles are tiny
    q = q - Q @ (Q.T @ q)
    q, _ = np.linalg.qr(q)
    return q, angles, kept


def rayleigh_ritz(Q: np.ndarray, HQ: np.ndarray, k: int):
    """theta, V (k lowest of T = Q^T H Q), Z = Q V and the residual norms (eqs. tilde_H, rrn)."""
    T = Q.T @ HQ
    T = 0.5 * (T + T.T)
    w, V = np.linalg.eigh(T)
    kk = min(k, T.shape[0])
    theta = w[:kk]
    V = V[:, :kk]
    Z = Q @ V
    HZ = HQ @ V
    R = HZ - Z * theta[None, :]
    rn = np.linalg.norm(R, axis=0)
    rrn = rn / np.where(np.abs(theta) > 1e-300, np.abs(theta), 1.0)
    return theta, V, Z, HZ, rrn, T


def jacobi_correction(diag: np.ndarray, theta: float, r: np.ndarray, z: np.ndarray) -> np.ndarray:
    """t = -(I - z z^T) M r with M = (diag(H) - theta)^-1, |denominator| clamped from below."""
    den = diag - theta
    floor = 1e-2 * max(1.0, abs(theta))
    small = np.abs(den) < floor
    den = np.where(small, np.where(den >= 0, floor, -floor), den)
    t = r / den
    t = t - z * (z @ t)
    return -t


def diag_precond(diag: np.ndarray, theta: float, r: np.ndarray) -> np.ndarray:
    """M r with M = (diag(H) - theta)^-1, |denominator| clamped from below as in the Jacobi step."""
    den = diag - theta
    floor = 1e-2 * max(1.0, abs(theta))
    den = np.where(np.abs(den) < floor, np.where(den >= 0, floor, -floor), den)
    return r / den


def diis_coefficients(A: np.ndarray) -> np.ndarray:
    """Pulay's DIIS: the a minimising a^T A a subject to sum(a) = 1 (A = the Gram matrix of the
    residuals of the iterates), from the bordered system [[A, 1], [1^T, 0]] [a; mu] = [0; 1]."""
    L = A.shape[0]
    M = np.zeros((L + 1, L + 1))
    # the minimiser does not depend on the scale of A; the residuals shrink to ~1e-10, so A is
    # scaled to a unit largest diagonal before it is bordered by ones
    M[:L, :L] = A / max(float(np.max(np.diag(A))), 1e-300)
    M[:L, L] = 1.0
    M[L, :L] = 1.0
    rhs = np.zeros(L + 1)
    rhs[L] = 1.0
    # the residuals of converging iterates become nearly parallel: least squares keeps the bordered
    # system solvable when A is (numerically) singular
    return np.linalg.lstsq(M, rhs, rcond=None)[0][:L]


def rmm_diis(H: sp.csr_matrix, diag: np.ndarray, x0: np.ndarray, Hx0: np.ndarray, tol: float,
             max_iter: int = 100, depth: int = 16):
    """Refines one approximate eigenpair by RMM-DIIS (the continuation of the hybrid of Sec. VI: one
    product with H per iteration, the diagonal preconditioner).  The iterates x_j (unit norm) with
    H x_j and residuals R_j = H x_j - theta_j x_j are kept (the last `depth`); each iteration
      1. combines them by DIIS: xb = sum a_j x_j, the a_j minimising |sum a_j R_j| with sum a_j = 1;
      2. normalises xb (and H xb), takes its Rayleigh quotient thb and residual Rb;
      3. stops when |Rb| / |thb| < tol;
      4. steps along t = M Rb (M the diagonal preconditioner) with the lam minimising
         |Rb + lam (H - thb) t|, i.e. lam = -Rb.u / u.u with u = H t - thb t (the product);
      5. keeps x_new = xb + lam t (normalised) as the next iterate.
    When the history is full it restarts from xb (DIIS over near-parallel residuals stalls
    otherwise).  Returns (theta, x, Hx, rrn, products, iterations)."""
    nrm = np.linalg.norm(x0)
    X = [x0 / nrm]
    HX = [Hx0 / nrm]
    R = [HX[0] - (X[0] @ HX[0]) * X[0]]
    products = 0
    for it in range(max_iter + 1):
        if len(X) == 1:
            a = np.ones(1)
        else:
            A = np.array([[ri @ rj for rj in R] for ri in R])
            a = diis_coefficients(A)
        xb = sum(ai * xi for ai, xi in zip(a, X))
        Hxb = sum(ai * hi for ai, hi in zip(a, HX))
        s = np.linalg.norm(xb)
        xb, Hxb = xb / s, Hxb / s
        thb = float(xb @ Hxb)
        Rb = Hxb - thb * xb
        rrn = np.linalg.norm(Rb) / abs(thb)
        if rrn < tol or it == max_iter:
            return thb, xb, Hxb, rrn, products, it
        t = diag_precond(diag, thb, Rb)
        Ht = H @ t
        products += 1
        u = Ht - thb * t
        lam = -(Rb @ u) / (u @ u)
        xn = xb + lam * t
        Hxn = Hxb + lam * Ht
        s = np.linalg.norm(xn)
        xn, Hxn = xn / s, Hxn / s
        if len(X) >= depth:
            X, HX, R = [xb], [Hxb], [Rb]
        X.append(xn)
        HX.append(Hxn)
        R.append(Hxn - (xn @ Hxn) * xn)


def small_space_correction(H: sp.csr_matrix, n0: int, theta: float, r: np.ndarray,
                           z: np.ndarray) -> np.ndarray:
    """t = -(I - z z^T) M r with M = (H0hat - theta)^-1 on the rows of the small space and the
    diagonal step (diag(H) - theta)^-1 (clamped as in jacobi_correction) on the other rows.

    Preconditioner of the continuation that uses the zeroth-order block H0hat of the split
    H = H0 + V (eq. split2); the small-space block is solved exactly (dense).
    """
    d = H.diagonal()
    den = d - theta
    floor = 1e-2 * max(1.0, abs(theta))
    den = np.where(np.abs(den) < floor, np.where(den >= 0, floor, -floor), den)
    t = r / den
    H0 = H[:n0, :n0].toarray()
    t[:n0] = np.linalg.solve(H0 - theta * np.eye(n0), r[:n0])
    t = t - z * (z @ t)
    return -t


# --------------------------------------------------------------------------- driver


@dataclass
class Options:
    tol: float = 1e-6
    maxiter: int = 30          # highest perturbation order for pure SPPC (Alg. 2 input)
    p_switch: int = 15         # switch point used in Sec. VI; None = pure SPPC up to maxiter
    continuation: bool = True  # preconditioned continuation after p_switch
    max_cont: int = 200
    m_max: int = 512           # thick restart of the continuation beyond this many columns
    tau_drop: float = 1e-10
    final_check: bool = True
    precond: Optional[Callable] = None  # (H, diag, theta_i, r_i, z_i, i) -> t_i; default Jacobi
    rmm_diis: bool = False     # the continuation refines each unconverged pair by RMM-DIIS instead
    diis_depth: int = 16       # iterates kept by DIIS
    diis_sweep: int = 4        # RMM-DIIS iterations per pair between two Rayleigh-Ritz rotations
    auto_switch: bool = False  # switch before p_switch once SPPC stagnates (see sppc_stagnated)
    shift: str = "E0"          # "E0": the paper's E^(0) in the small-space corrections; "ritz": the
                               # Ritz values of the step before (the theta-shifted variant)


@dataclass
class Result:
    theta: np.ndarray
    Z: np.ndarray
    rrn: np.ndarray
    converged: bool
    n_spmv: int
    history: List[dict] = field(default_factory=list)
    E_hist: List[np.ndarray] = field(default_factory=list)
    E0: Optional[np.ndarray] = None
    Q: Optional[np.ndarray] = None


def final_check(H: sp.csr_matrix, Z: np.ndarray):
    """Explicit H Z, Rayleigh-Ritz on span Z and the true relative residuals."""
    HZ = H @ Z
    S = Z.T @ HZ
    S = 0.5 * (S + S.T)
    w, W = np.linalg.eigh(S)
    Z2 = Z @ W
    HZ2 = HZ @ W
    R = HZ2 - Z2 * w[None, :]
    rrn = np.linalg.norm(R, axis=0) / np.abs(w)
    return w, Z2, rrn


def sppc_stagnated(hist: List[dict]) -> bool:
    """The automatic switch point (the paper leaves its detection open, Sec. VII).

    SPPC has stagnated after step p when a correction vector of that step lies almost in the
    subspace built so far (sine of the angle of Fig. 3 below 1e-4: the higher orders add nothing,
    Sec. VI), or when the largest residual norm has not halved since step p - 3.
    hist holds one record per SPPC step, p = 0 first.
    """
    if min(hist[-1]["angles"]) < 1e-4:
        return True
    return len(hist) >= 4 and not (max(hist[-1]["rrn"]) < 0.5 * max(hist[-4]["rrn"]))


def rmm_stagnated(top: List[float]) -> bool:
    """The hand-over of the RMM-DIIS refinement to the Davidson continuation.

    top[0] is the largest residual norm at the switch, top[s] the largest after sweep s (after the
    Rayleigh-Ritz rotation).  The refinement has stagnated when the largest residual has not halved
    since three sweeps before, the residual clause of sppc_stagnated applied to the sweeps.  A pair
    whose minimal-residual step along the diagonally preconditioned residual becomes orthogonal to
    the residual (an interior pair: H - theta and the preconditioner are both indefinite) makes no
    progress however many sweeps follow.
    """
    return len(top) >= 4 and not (top[-1] < 0.5 * top[-4])


def sppc_pair(H: sp.csr_matrix, n0: int, kk: int, opts: Options = Options(),
              callback: Optional[Callable] = None) -> Result:
    """Alg. 1: SPPC for the kk-th eigenpair alone (kk = 0 is the lowest).

    The zeroth order is the kk-th eigenpair of H0hat (reading of "the k-th nonzero eigenpair of
    H0"); the subspace is spanned by that pair's own corrections Psi_kk^(0..p) (eq. Man_P) and the
    approximation is the lowest Ritz pair of the subspace.  This is the SPPC iteration above with a
    single wanted pair whose zeroth order is (E_kk^(0), psi_kk): the eigendecomposition of H0hat is
    handed over reordered so that pair kk comes first (the spectral small solve sums over every
    other eigenvector whatever their order)."""
    H = sp.csr_matrix(H, dtype=np.float64)
    z = zeroth_order(small_space_matrix(H, n0))
    if not 0 <= kk < len(z.w):
        raise ValueError("pair index out of range")
    perm = np.concatenate([[kk], np.delete(np.arange(len(z.w)), kk)])
    return sppc(H, n0, 1, opts, z=ZerothOrder(z.w[perm], z.U[:, perm]), callback=callback)


def sppc(H: sp.csr_matrix, n0: int, k: int, opts: Options = Options(),
         z: Optional[ZerothOrder] = None, callback: Optional[Callable] = None) -> Result:
    """Alg. 2 (SPPC for the k lowest pairs) followed by the optional continuation."""
    H = sp.csr_matrix(H, dtype=np.float64)
    n = H.shape[0]
    H0hat = small_space_matrix(H, n0)
    if z is None:
        z = zeroth_order(H0hat)
    check_e0(z, k)
    diag = H.diagonal()

    # p = 0 (Alg. 2 steps 1-4)
    Psi0 = np.zeros((n, k))
    Psi0[:n0] = z.U[:, :k]
    Q = Psi0.copy()
    HQ = H @ Q
    n_spmv = k
    theta, V, Z, HZ, rrn, T = rayleigh_ritz(Q, HQ, k)
    hist = [dict(p=0, phase="sppc", theta=theta.copy(), rrn=rrn.copy(), m=Q.shape[1],
                 n_spmv=n_spmv, angles=np.ones(k), T0=T.copy())]
    if callback:
        callback(hist[-1])
    E_hist = [z.w[:k].copy(), np.zeros(k)]   # E^(0); E^(1) = 0 (eq. first_PC)
    Psi_hist = [Psi0]
    VPsi0 = H @ Psi0 - apply_H0(H0hat, Psi0)
    converged = bool(np.all(rrn < opts.tol))

    p = 0
    last_p = opts.maxiter if not opts.continuation or opts.p_switch is None \
        else min(opts.maxiter, opts.p_switch)
    while not converged and p < last_p:
        p += 1
        shifts = theta.copy() if opts.shift == "ritz" else None
        E_p, Psi_p = correction_vectors(H, H0hat, z, k, E_hist[:p], Psi_hist, VPsi0, shifts)
        if p >= 2:
            E_hist.append(E_p)
        Psi_hist.append(Psi_p)
        q, angles, kept = orthonormalize_block(Q, Psi_p, opts.tau_drop)
        if q.shape[1] > 0:
            Q = np.hstack([Q, q])
            HQ = np.hstack([HQ, H @ q])
            n_spmv += q.shape[1]
        theta, V, Z, HZ, rrn, T = rayleigh_ritz(Q, HQ, k)
        converged = bool(np.all(rrn < opts.tol))
        hist.append(dict(p=p, phase="sppc", theta=theta.copy(), rrn=rrn.copy(), m=Q.shape[1],
                         n_spmv=n_spmv, angles=angles.copy(), kept=kept.copy()))
        if callback:
            callback(hist[-1])
        if opts.auto_switch and opts.continuation and opts.p_switch is not None and not converged \
                and sppc_stagnated(hist):
            break

    # the hybrid of Sec. VI: each unconverged Ritz pair refined on its own by RMM-DIIS, in sweeps
    # of at most opts.diis_sweep iterations per pair; between sweeps, Rayleigh-Ritz on the span of
    # the k refined vectors (the subspace rotation of multi-pair RMM-DIIS: it separates pairs whose
    # eigenvalues are close, which a single-vector iteration resolves only slowly)
    done_its = 0
    stagnated = False
    top = [float(np.max(rrn))]
    while not converged and opts.continuation and opts.rmm_diis and done_its < opts.max_cont:
        sweep = 0
        for i in np.nonzero(rrn >= opts.tol)[0]:
            th, x, hx, r_i, prods, its = rmm_diis(H, diag, Z[:, i], HZ[:, i], opts.tol,
                                                  min(opts.diis_sweep, opts.max_cont - done_its),
                                                  opts.diis_depth)
            theta[i], Z[:, i], HZ[:, i], rrn[i] = th, x, hx, r_i
            n_spmv += prods
            sweep = max(sweep, its)
        done_its += max(sweep, 1)
        Qz, Rz = np.linalg.qr(Z)
        theta, V, Z, HZ, rrn, T = rayleigh_ritz(Qz, HZ @ np.linalg.inv(Rz), k)
        converged = bool(np.all(rrn < opts.tol))
        hist.append(dict(p=p, phase="rmmdiis", iterations=sweep, theta=theta.copy(), rrn=rrn.copy(),
                         m=Q.shape[1], n_spmv=n_spmv))
        if callback:
            callback(hist[-1])
        top.append(float(np.max(rrn)))
        if not converged and rmm_stagnated(top):
            # the Davidson continuation takes over from the refined Ritz vectors.  The basis
            # restarts on them (it does not hold them), with their products taken afresh: the
            # H x that RMM-DIIS carries through its combinations has drifted from H Z by
            # rounding, and Rayleigh-Ritz on the drifted columns cannot see below that drift
            stagnated = True
            Q = Z.copy()
            HQ = H @ Q
            n_spmv += k
            break

    # continuation with preconditioned residual blocks (after a stagnated RMM-DIIS refinement it
    # shares that refinement's budget of max_cont iterations)
    it = done_its if stagnated else 0
    while not converged and opts.continuation and (stagnated or not opts.rmm_diis) and it < opts.max_cont:
        it += 1
        R = HZ - Z * theta[None, :]
        act = np.nonzero(rrn >= opts.tol)[0]
        cols = []
        for i in act:
            if opts.precond is None:
                cols.append(jacobi_correction(diag, theta[i], R[:, i], Z[:, i]))
            else:
                cols.append(opts.precond(H, diag, theta[i], R[:, i], Z[:, i], i))
        Tb = np.stack(cols, axis=1)
        if Q.shape[1] + Tb.shape[1] > opts.m_max:
            # thick restart on the current Ritz vectors
            Q = Z.copy()
            HQ = HZ.copy()
        q, angles, kept = orthonormalize_block(Q, Tb, opts.tau_drop)
        if q.shape[1] > 0:
            Q = np.hstack([Q, q])
            HQ = np.hstack([HQ, H @ q])
            n_spmv += q.shape[1]
        theta, V, Z, HZ, rrn, T = rayleigh_ritz(Q, HQ, k)
        converged = bool(np.all(rrn < opts.tol))
        hist.append(dict(p=p + it, phase="cont", theta=theta.copy(), rrn=rrn.copy(),
                         m=Q.shape[1], n_spmv=n_spmv, angles=angles.copy(), active=act.copy()))
        if callback:
            callback(hist[-1])

    if opts.final_check:
        theta, Z, rrn = final_check(H, Z)
        converged = bool(np.all(rrn < opts.tol))
    return Result(theta, Z, rrn, converged, n_spmv, hist, E_hist, z.w[:k].copy(), Q)
