"""Four solver forms on sixteen random level-structured matrices against dense eigenvalues.

The shapes are drawn from a fixed seed: two to five levels, each level 1.5 to 10 times the one
before (the first 5 to 60 rows), at most 3,000 rows in all, mean degree 10 to 80, one or two small
levels, k from 1 to 16 (below the size of the small space).  The forms: the float64 Davidson
continuation, float64 SPPC + RMM-DIIS, mixed SPPC + RMM-DIIS (all at rrn 1e-6), and the float64
Davidson continuation at 1e-9.  Each solve must succeed with orthonormal vectors whose true
residual (numpy's product with the symmetric matrix) meets the tolerance, and its eigenvalues must
be the lowest of numpy's eigvalsh: within 1e-9 relative, the error of eigvalsh itself included
(eps ||H|| / |lambda| is about 1e-12 for the eigenvalues near zero that some of these matrices
have).  Wider random sweeps of this kind found the breakdown of a basis that fills the whole space,
the float64 hybrid ending just above its tolerance, and the zeroth-order filter losing directions
when its block nearly fills a small space; each has a test of its own.
"""
import numpy as np
import pytest

import levelgen
import oracle

pytestmark = pytest.mark.gpu


def _shapes(seed=2026, count=16, nmax=3000):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        nlev = int(rng.integers(2, 6))
        s0 = int(rng.integers(5, 60))
        ratio = rng.uniform(3, 10)
        sizes = None
        for _ in range(60):  # shrink the ratio until the levels fit
            cand = [max(1, int(s0 * ratio ** j)) for j in range(nlev)]
            if sum(cand) <= nmax:
                sizes = cand
                break
            ratio = max(1.5, ratio * 0.9)
            s0 = max(3, int(s0 * 0.9))
        d = int(rng.integers(10, 80))
        sd = int(rng.integers(1, 10 ** 6))
        ns = 1 if nlev <= 2 else int(rng.integers(1, 3))
        if sizes is None:
            continue
        k = int(min(rng.integers(1, 17), sum(sizes[:ns]) - 1))
        if k >= 1:
            out.append((tuple(sizes), d, sd, ns, k))
    return out


SHAPES = _shapes()


@pytest.fixture(scope="module")
def P():
    import paper_2407_08901_amd as P
    P.lib()
    return P


@pytest.mark.parametrize("shape", SHAPES, ids=["n%d-L%d-k%d" % (sum(s[0]), len(s[0]), s[4]) for s in SHAPES])
def test_forms_on_random_shapes(P, shape):
    sizes, d, sd, ns, k = shape
    A = levelgen.generate(sizes, d, sd)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:k]
    rp, col, val = P.upload(A)
    forms = [("float64 Davidson", dict(), 1e-6), ("float64 RMM-DIIS", dict(precond=P.SPPC_CORR_RMMDIIS), 1e-6),
             ("mixed RMM-DIIS", dict(precision=P.SPPC_PREC_MIXED, precond=P.SPPC_CORR_RMMDIIS), 1e-6),
             ("float64 Davidson at 1e-9", dict(tol=1e-9), 1e-9)]
    for name, kw, tol in forms:
        print("case random shape %s d=%d seed=%d ns=%d k=%d: %s" % (sizes, d, sd, ns, k, name), flush=True)
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(**kw))
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK, name
        ev = np.array(ev)
        Zh = Z.cpu().numpy()
        assert np.max(np.abs(Zh.T @ Zh - np.eye(k))) < 1e-10, name
        assert np.max(np.linalg.norm(H @ Zh - Zh * ev[None, :], axis=0) / np.abs(ev)) < tol, name
        assert np.max(np.abs(ev - lam) / np.abs(lam)) < 1e-9, name
