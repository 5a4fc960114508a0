"""The seeded input generator: determinism and the structure the recipe promises."""
import numpy as np

import levelgen


def _levels(A):
    return np.searchsorted(A.level_offsets, np.arange(A.n), side="right") - 1


def test_deterministic_and_seed_dependent():
    a = levelgen.generate((50, 300, 900), 30, 7)
    b = levelgen.generate((50, 300, 900), 30, 7)
    c = levelgen.generate((50, 300, 900), 30, 8)
    assert a.sha256() == b.sha256()
    assert a.sha256() != c.sha256()


def test_upper_csr_structure_and_adjacency():
    A = levelgen.generate((40, 200, 700), 40, 11)
    rp, col = A.row_ptr, A.col
    assert rp[0] == 0 and rp[-1] == len(col)
    lev = _levels(A)
    for i in range(A.n):
        c = col[rp[i]:rp[i + 1]]
        assert c[0] == i                       # diagonal first
        assert np.all(np.diff(c) > 0)          # sorted, unique, upper
        assert np.all(np.abs(lev[c] - lev[i]) <= 1)  # same or adjacent level only


def test_values_diagonal_and_degree():
    A = levelgen.WORKLOADS[0].generate()
    lev = _levels(A)
    diag = A.val[A.row_ptr[:-1]]
    assert np.all(np.abs(diag - 10.0 * lev) < 1.0)
    off = np.ones(A.nnz, bool)
    off[A.row_ptr[:-1]] = False
    v = A.val[off].astype(np.float64)
    assert abs(v.std() - 0.5) < 0.01 and abs(v.mean()) < 0.01
    # mean full-row degree ~ d (each stored off-diagonal counts twice)
    full_deg = (2 * (A.nnz - A.n) + A.n) / A.n
    assert 58 < full_deg < 62
    assert A.val.dtype == np.float32


def test_workload_table():
    w = levelgen.WORKLOADS[1]
    assert w.n == 1172000 and w.n0 == 22000 and w.k == 8
    assert levelgen.WORKLOADS[4].n == 7722000
