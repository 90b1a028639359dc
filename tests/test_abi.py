"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nhq.h")
LIB = os.path.join(ROOT, "paper_2203_13601_amd", "libnhq.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nhq_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("nhq_build_index", "nhq_hybrid_search", "nhq_index_create", "nhq_index_free",
                 "nhq_bruteforce_hybrid_knn", "nhq_strerror"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnhq.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)      # loads without a GPU; nothing is called
    for n in declared():
        assert getattr(lib, n) is not None


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnhq.so not built")
def test_library_has_gfx950_code_only():
    blob = open(LIB, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2203_13601_amd._binding as b
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(ImportError):
        b.lib()
