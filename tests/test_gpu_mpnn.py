"""Learned preconditioner on the GPU against the float64 CPU reference (through the C ABI)."""
import numpy as np
import pytest
import torch

import levelgen
import oracle
from oracle import mpnn as ompnn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2407_08901_amd as P
    P.lib()
    return P


def _problem(seed, S, sizes=(37, 250, 1800), d=30, nsmall=1):
    A = levelgen.generate(sizes, d, seed)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    Aoff, dg = ompnn.offdiag(H)
    lev = ompnn.level_feature(A.level_offsets, nsmall)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((A.n, S))
    X /= np.linalg.norm(X, axis=0)
    th = np.einsum("ij,ij->j", X, H @ X)
    R = H @ X - X * th[None, :]
    E = rng.standard_normal((A.n, S))
    E -= X * np.einsum("ij,ij->j", X, E)[None, :]
    w = (rng.standard_normal(ompnn.NPARAM) * 0.3).astype(np.float32)
    return A, H, Aoff, dg, lev, X, th, R, E, w


def _ctx(P, A, nsmall=1):
    rp, col, val = P.upload(A)
    return P.sppc_setup(rp, col, val, A.level_offsets, nsmall, 4, P.sppc_default_opts())


def _cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_forward_and_gradient_match_reference(P):
    S = 5
    A, H, Aoff, dg, lev, X, th, R, E, w = _problem(11, S)
    print("case mpnn fwd/grad n=%d S=%d" % (A.n, S), flush=True)
    ctx = _ctx(P, A)
    T, loss, grad = P.sppc_mpnn_eval(ctx, w, _cu(R), _cu(X), th, _cu(E), f64=True)
    T = T.cpu().numpy()
    w64 = w.astype(np.float64)
    g_ref = np.zeros(ompnn.NPARAM)
    for s in range(S):
        tp, _ = ompnn.forward(w64, Aoff, dg, lev, th[s], R[:, s], X[:, s])
        assert np.max(np.abs(T[:, s] - tp)) < 1e-11 * np.max(np.abs(tp))
        L, g = ompnn.loss_and_grad(w64, Aoff, dg, lev, th[s], R[:, s], X[:, s], E[:, s])
        assert abs(loss[s] - L) < 1e-11
        g_ref += g / S
    assert np.max(np.abs(np.array(grad) - g_ref)) < 1e-10 * np.max(np.abs(g_ref))
    # the solver's form: float32 arithmetic, bfloat16 weights
    wq = ompnn_bf16(w)
    _, loss32, grad32 = P.sppc_mpnn_eval(ctx, w, _cu(R), _cu(X), th, _cu(E), f64=False)
    g_q = sum(ompnn.loss_and_grad(wq, Aoff, dg, lev, th[s], R[:, s], X[:, s], E[:, s])[1] for s in range(S)) / S
    assert np.max(np.abs(np.array(grad32) - g_q)) < 2e-4 * np.max(np.abs(g_q))


def test_basis_projection_and_target_match_reference(P):
    S, m = 3, 9
    A, H, Aoff, dg, lev, X, th, R, E, w = _problem(13, S)
    print("case mpnn basis n=%d S=%d m=%d" % (A.n, S, m), flush=True)
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(np.column_stack([X, rng.standard_normal((A.n, m - S))]))
    Psi = rng.standard_normal((A.n, S))
    ctx = _ctx(P, A)
    Eg = P.sppc_mpnn_target(ctx, _cu(Q), _cu(Psi)).cpu().numpy()
    E_ref = Psi - Q @ (Q.T @ Psi)
    assert np.max(np.abs(Eg - E_ref)) < 1e-13 * np.max(np.abs(Psi))
    T, loss, grad = P.sppc_mpnn_eval(ctx, w, _cu(R), _cu(X), th, _cu(E_ref), f64=True, Q=_cu(Q))
    T = T.cpu().numpy()
    w64 = w.astype(np.float64)
    g_ref = np.zeros(ompnn.NPARAM)
    for s in range(S):
        tp, _ = ompnn.forward(w64, Aoff, dg, lev, th[s], R[:, s], X[:, s], Q)
        assert np.max(np.abs(T[:, s] - tp)) < 1e-11 * np.max(np.abs(tp))
        L, g = ompnn.loss_and_grad(w64, Aoff, dg, lev, th[s], R[:, s], X[:, s], E_ref[:, s], Q)
        assert abs(loss[s] - L) < 1e-11
        g_ref += g / S
    assert np.max(np.abs(np.array(grad) - g_ref)) < 1e-10 * np.max(np.abs(g_ref))


def ompnn_bf16(w):
    b = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def test_zero_network_solve_equals_jacobi(P):
    w = levelgen.WORKLOADS[0]
    A = w.generate()
    print("case mpnn zero net", flush=True)
    rp, col, val = P.upload(A)
    res = {}
    for kind in ("jacobi", "zero"):
        opts = P.sppc_default_opts(precond=P.SPPC_CORR_JACOBI if kind == "jacobi" else P.SPPC_CORR_MPNN)
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, w.k, opts)
        if kind == "zero":
            P.sppc_mpnn_set_weights(ctx, np.zeros(289, np.float32))
        res[kind] = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
    ev_j, _, _, st_j, _ = res["jacobi"]
    ev_z, _, _, st_z, _ = res["zero"]
    assert st_z["mpnn_steps"] > 0
    assert st_j["cont_steps"] == st_z["cont_steps"]
    assert np.max(np.abs(np.array(ev_j) - np.array(ev_z)) / np.abs(ev_j)) < 1e-12


def test_garbage_weights_fall_back_to_jacobi(P):
    w = levelgen.WORKLOADS[0]
    A = w.generate()
    print("case mpnn garbage", flush=True)
    rp, col, val = P.upload(A)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, 1, w.k, P.sppc_default_opts(precond=P.SPPC_CORR_MPNN))
    P.sppc_mpnn_set_weights(ctx, np.full(289, np.nan, np.float32))
    ev, Z, rrn, st, status = P.sppc_solve(ctx)
    assert status == P.SPPC_OK and st["mpnn_steps"] == 0
    lam = np.linalg.eigvalsh(oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n).toarray())[: w.k]
    assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-10


def test_training_step_lowers_the_loss(P):
    S = 8
    A, H, Aoff, dg, lev, X, th, R, E, w = _problem(5, S)
    print("case mpnn train", flush=True)
    ctx = _ctx(P, A)
    state = torch.zeros(4 * 289, dtype=torch.float32, device="cuda")
    state[:289] = torch.from_numpy(w * 0.1).cuda()
    Rg, Xg, Eg = _cu(R), _cu(X), _cu(E)
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(np.column_stack([X, rng.standard_normal((A.n, 4))]))
    Qg = _cu(Q)
    Eg = P.sppc_mpnn_target(ctx, Qg, Eg)
    losses = [P.sppc_mpnn_train_step(ctx, state, Rg, Xg, th, Eg, 1e-2, it + 1, Q=Qg) for it in range(40)]
    assert losses[-1] < losses[0] - 1e-3
    assert np.all(np.isfinite(losses))


def test_forward_matches_reference_with_two_small_levels(P):
    # five levels, the first two the small space: the level input is 0, 0, 1/2, 1, 1 (the kernel
    # computes it from the level offsets and the small-level count of the setup)
    S = 3
    A, H, Aoff, dg, lev, X, th, R, E, w = _problem(13, S, sizes=(30, 60, 200, 600, 1500), d=24, nsmall=2)
    print("case mpnn fwd five levels n=%d S=%d" % (A.n, S), flush=True)
    ctx = _ctx(P, A, nsmall=2)
    T, loss, grad = P.sppc_mpnn_eval(ctx, w, _cu(R), _cu(X), th, _cu(E), f64=True)
    T = T.cpu().numpy()
    for s in range(S):
        tp, _ = ompnn.forward(w.astype(np.float64), Aoff, dg, lev, th[s], R[:, s], X[:, s])
        assert np.max(np.abs(T[:, s] - tp)) < 1e-11 * np.max(np.abs(tp))
    P.sppc_destroy(ctx)
