"""Every solver form on a spread of small level-structured matrices, against dense eigenvalues.

Shapes with two to five levels, ragged sizes (none a multiple of the kernels' row blocks), small and
large densities, one or two small levels, and k from 1 to 12.  Each form must reach the k lowest
eigenvalues of the dense matrix (numpy eigh of the oracle's symmetric matrix): float64 forms to
1e-10, mixed forms to 1e-8 (both stop at rrn 1e-6 with the Kato-Temple bound far below), with the
true residual, recomputed from the oracle's matrix and the returned vectors, below the tolerance.
The forms: the Davidson continuation (diagonal step), the SPPC + RMM-DIIS hybrid, the small-space
continuation, the mixed form of each of the first two, and a forced column-panel copy.
"""
import numpy as np
import pytest
import torch

import levelgen
import oracle

pytestmark = pytest.mark.gpu

# (level sizes, d, seed, small levels, k)
SHAPES = [
    ((37, 411, 2203), 18, 501, 1, 3),
    ((101, 917, 5003), 45, 502, 1, 8),
    ((13, 129, 1187, 6011), 24, 503, 2, 5),
    ((251, 2503, 9001), 60, 504, 1, 12),
    ((7, 61, 509, 3001, 7919), 30, 505, 2, 4),
    ((400, 3999), 80, 506, 1, 1),
]

FORMS = [
    ("float64 Davidson", dict(), 1e-10),
    ("float64 RMM-DIIS", dict(precond=4), 1e-10),
    ("float64 small-space continuation", dict(precond=3), 1e-10),
    ("mixed Davidson", dict(precision=1), 1e-8),
    ("mixed RMM-DIIS", dict(precision=1, precond=4), 1e-8),
    ("float64, column panels", dict(panel_width=512), 1e-10),
]


@pytest.fixture(scope="module")
def P():
    import paper_2407_08901_amd as P
    P.lib()
    return P


@pytest.mark.parametrize("shape", SHAPES, ids=["L%d-n%d-k%d" % (len(s[0]), sum(s[0]), s[4]) for s in SHAPES])
def test_every_form_reaches_the_dense_eigenvalues(P, shape):
    sizes, d, seed, ns, k = shape
    A = levelgen.generate(sizes, d, seed)
    print("case sweep levels %s d=%d k=%d" % (sizes, d, k), flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:k]
    rp, col, val = P.upload(A)
    for name, kw, bound in FORMS:
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(**kw))
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK, name
        ev = np.array(ev)
        assert np.max(np.abs(ev - lam) / np.abs(lam)) < bound, name
        Zc = Z.cpu().numpy()
        R = H @ Zc - Zc * ev[None, :]
        assert np.max(np.linalg.norm(R, axis=0) / np.abs(ev)) < 1e-6, name
        assert np.max(np.abs(Zc.T @ Zc - np.eye(k))) < 1e-10, name
