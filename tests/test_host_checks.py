"""Argument checks of the C ABI that run on the host before any device work (no GPU needed).

sppc_workspace_size validates the problem and the options exactly as sppc_setup does, before it
touches device memory, so refused inputs can be exercised here with placeholder device pointers
(never dereferenced on these paths)."""
import ctypes

import pytest

import paper_2407_08901_amd as P

FAKE = 0x1000  # a non-null placeholder: every case below is refused before any device access


def _query(n, offsets, n_small, k, **opts):
    L = P.lib()
    H = P.sppc_csr(n, 3 * n, FAKE, FAKE, FAKE, P.SPPC_F64)
    lo = (ctypes.c_int64 * len(offsets))(*offsets)
    o = P.sppc_default_opts(**opts)
    out = ctypes.c_size_t(123)
    st = L.sppc_workspace_size(ctypes.byref(H), lo, len(offsets) - 1, n_small, k, ctypes.byref(o), ctypes.byref(out))
    return st, out.value, L.sppc_setup_error().decode()


def test_explicit_panels_are_refused_beyond_24_bit_columns():
    n = (1 << 24) + 4
    st, size, msg = _query(n, [0, 1000, n], 1, 4, panel_width=4096)
    assert st == 1 and size == 0 and "24 bits" in msg


@pytest.mark.parametrize("case", ["k17", "k_above_n0", "offsets_short", "offsets_unsorted", "pair_with_k4",
                                  "pair_index_range", "deflate_below_k", "m_max", "panel_width", "shift_kind",
                                  "rmm_precond"])
def test_refused_problems_and_options(case):
    n = 5000
    offs, ns, k, kw = [0, 100, 1000, n], 1, 4, {}
    if case == "k17":
        k = 17
    elif case == "k_above_n0":
        offs, k = [0, 3, 1000, n], 4
    elif case == "offsets_short":
        offs = [0, 100, 1000, n - 1]
    elif case == "offsets_unsorted":
        offs = [0, 1000, 100, n]
    elif case == "pair_with_k4":
        kw = dict(pair_index=1)
    elif case == "pair_index_range":
        k, kw = 1, dict(pair_index=27)
    elif case == "deflate_below_k":
        kw = dict(n_deflate=3)
    elif case == "m_max":
        kw = dict(m_max=7)
    elif case == "panel_width":
        kw = dict(panel_width=70000)
    elif case == "shift_kind":
        kw = dict(corr_shift=2)
    elif case == "rmm_precond":
        kw = dict(precond=P.SPPC_CORR_RMMDIIS, rmm_precond=P.SPPC_CORR_SMALL)
    st, size, msg = _query(n, offs, ns, k, **kw)
    assert st == 1 and size == 0 and msg, (case, st, msg)
