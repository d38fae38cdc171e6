"""The C-ABI library loads without a GPU and exports every symbol the header
declares; host-only calls answer.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

import paper_2601_16522_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", txt)))


def test_header_symbols_exported():
    names = _declared()
    assert len(names) >= 20
    L = C.CDLL(pf.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(pf.EXPORTS) == names


def test_supported_nphi_and_errors_without_device():
    assert pf.supported_nphi() == [2, 3, 4, 8, 9, 13]
    L = pf.lib()
    assert L.pf_create(None, None) == -1          # PF_EINVAL before any device work
    assert L.pf_last_error(None) == b"null handle"


def test_binding_fails_loudly_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(pf, "LIB_PATH", str(tmp_path / "libpf.so"))
    monkeypatch.setattr(pf, "_lib", None)
    with pytest.raises(ImportError):
        pf.lib()
