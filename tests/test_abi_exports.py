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
