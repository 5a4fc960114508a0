"""The C-ABI library loads and exports every entry point declared in include/sppc.h (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sppc.h")
LIB = os.path.join(ROOT, "paper_2407_08901_amd", "libsppc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sppc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared()
    for n in ("sppc_setup", "sppc_spmm", "sppc_correct", "sppc_rayleigh_ritz", "sppc_solve", "sppc_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2407_08901_amd import build
        build.build()
    import torch  # noqa: F401  (same HIP runtime as the GPU path)
    L = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in declared():
        assert re.search(r"\bT %s\b" % n, out), n


def test_binding_names_match_abi():
    import paper_2407_08901_amd as P
    for n in declared():
        if n in ("sppc_last_error", "sppc_setup_error"):
            continue
        assert hasattr(P, n), n


def _header_struct(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*%s;" % name, text).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            typ, nm = decl.rsplit(None, 1)
            fields.append((nm.lstrip("*"), "ptr" if "*" in decl else typ.split()[-1]))
    return fields


CTYPE = {"int": "c_int", "int64_t": "c_int64", "double": "c_double", "sppc_dtype": "c_int", "ptr": "c_void_p"}


@pytest.mark.parametrize("name", ["sppc_csr", "sppc_opts", "sppc_stats"])
def test_binding_structs_match_header_layout(name):
    import paper_2407_08901_amd as P
    want = _header_struct(name)
    have = getattr(P, name)._fields_
    assert [f for f, _ in have] == [f for f, _ in want]
    for (f, t), (_, ht) in zip(have, want):
        assert t is getattr(ctypes, CTYPE[ht]), (name, f, t, ht)
