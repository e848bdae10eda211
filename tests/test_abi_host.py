"""Host-side checks of the C ABI: the library loads and exports every function include/ssl.h
declares, the binding covers them, and the package refuses to run without the built library.
No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for n in ("ssl_corr_accum", "ssl_gsvd", "ssl_music_spectrum", "ssl_localize"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2504_03373_amd as S
    if not os.path.exists(S.LIB_PATH):
        pytest.fail("libssl_mi355x.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(S.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(S.EXPORTED)


def test_binding_has_every_entry_point():
    import paper_2504_03373_amd as S
    for n in declared_functions():
        assert callable(getattr(S, n)), n


def test_version_and_error_string_without_gpu():
    import paper_2504_03373_amd as S
    assert S.ssl_version() == 100
    assert isinstance(S.lib().ssl_last_error(), bytes)


def test_missing_library_fails_loudly(monkeypatch):
    import paper_2504_03373_amd as S
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", "/nonexistent/libssl_mi355x.so")
    with pytest.raises(ImportError):
        S.lib()


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    import paper_2504_03373_amd as S
    with pytest.raises(ValueError):
        S._ptr(torch.zeros(3))
