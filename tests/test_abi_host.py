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


def test_noalloc_scratch_limit_matches_header():
    import paper_2504_03373_amd as S
    text = open(HEADER).read()
    m = re.search(r"#define SSL_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "SSL_NOALLOC_SCRATCH_BYTES not found in the header"
    assert int(m.group(1)) << int(m.group(2)) == S.SSL_NOALLOC_SCRATCH_BYTES


def test_noalloc_scratch_bytes_host_only():
    import paper_2504_03373_amd as S
    # R and A (F M^2 complex64 each), E_n, P, Pbar, status, the signal vectors (F Ns M
    # complex64) and their inverse Cholesky factors (6 complex128 per bin), bin-sum partials;
    # 256-byte aligned
    a = lambda n: (n + 255) // 256 * 256
    F, M, Ns, D = 257, 60, 2, 1368
    want = (2 * a(F * M * M * 8) + a(F * (M - Ns) * M * 8) + a(F * D * 4) + a(D * 4) + a(F * 4)
            + a(F * Ns * M * 8) + a(F * 6 * 16) + a(((F + 15) // 16) * D * 4))
    assert S.ssl_localize_noalloc_bytes(F, M, Ns, D) == want
    assert want <= S.SSL_NOALLOC_SCRATCH_BYTES
    assert S.ssl_localize_noalloc_bytes(1100, 60, 2, 1368) > S.SSL_NOALLOC_SCRATCH_BYTES
    assert S.ssl_localize_noalloc_bytes(257, 65, 2, 1368) == 0
    assert S.ssl_localize_noalloc_bytes(257, 8, 8, 72) == 0
