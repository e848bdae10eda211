"""Pins of the oracle's GEVD-MUSIC subspace (orc_inv_sqrt, orc_gevd): the defining equations of
the Hermitian inverse square root and of generalized eigenvectors, the library generalized
eigensolver (scipy.linalg.eigh(R, K)), the K = I reduction to SEVD and planted noise-free
sources."""
import numpy as np
import pytest
import scipy.linalg

from conftest import crandn, random_pd


def test_inv_sqrt_definition(orc):
    rng = np.random.default_rng(51)
    for M, cond in ((4, 10.0), (12, 1e4), (30, 1e8)):
        K = random_pd(rng, M, cond)
        st, W = orc.inv_sqrt(K)
        assert st == 0
        assert np.allclose(W, W.conj().T, rtol=0, atol=1e-12 * np.linalg.norm(W))
        # W K W = I and W^2 = K^{-1}, to the conditioning of K
        e = np.linalg.norm(W @ K @ W - np.eye(M), 2)
        assert e <= 200 * M * cond ** 0.5 * 2.0 ** -53 * 10, (M, cond, e)
        Ki = np.linalg.solve(K, np.eye(M))
        assert np.linalg.norm(W @ W - Ki, 2) <= 1e-9 * np.linalg.norm(Ki, 2) * max(1.0, cond ** 0.5 / 1e2)
    D = np.diag([4.0, 9.0, 0.25, 1.0]).astype(complex)
    st, W = orc.inv_sqrt(D)
    assert st == 0 and np.allclose(W, np.diag([0.5, 1 / 3, 2.0, 1.0]), rtol=0, atol=1e-14)
    bad = np.diag([1.0, -1.0, 2.0]).astype(complex)
    assert orc.inv_sqrt(bad)[0] == orc.NOT_PD


@pytest.mark.parametrize("M,Ns,T", [(6, 2, 20), (16, 3, 40), (24, 2, 80)])
def test_gevd_generalized_eigenvectors(orc, M, Ns, T):
    rng = np.random.default_rng(52 + M)
    F = 3
    X = crandn(rng, F, T, M).astype(np.complex64)
    R = orc.corr(X)
    K = np.stack([random_pd(rng, M, 100.0) for _ in range(F)])
    En, sig, st = orc.gevd(K, R, Ns)
    assert np.all(st == 0)
    for f in range(F):
        E = En[f].T                                       # M x (M - Ns)
        lam_ref = scipy.linalg.eigh(R[f], K[f], eigvals_only=True)[::-1]
        assert np.allclose(sig[f], lam_ref, rtol=1e-10, atol=1e-12 * lam_ref[0])
        # R e = lambda K e for each noise vector, and K-orthonormality
        for c in range(M - Ns):
            lam = sig[f, Ns + c]
            res = R[f] @ E[:, c] - lam * K[f] @ E[:, c]
            assert np.linalg.norm(res) <= 1e-10 * (np.linalg.norm(R[f], 2) + lam * np.linalg.norm(K[f], 2)) * np.linalg.norm(E[:, c])
        assert np.allclose(E.conj().T @ K[f] @ E, np.eye(M - Ns), rtol=0, atol=1e-10)
        # same span as the library's generalized noise eigenvectors
        w, V = scipy.linalg.eigh(R[f], K[f])
        Vn = V[:, :M - Ns]
        Qa, _ = np.linalg.qr(E)
        Qb, _ = np.linalg.qr(Vn)
        gap = lam_ref[Ns - 1] - lam_ref[Ns]
        assert np.linalg.norm(Qa @ Qa.conj().T - Qb @ Qb.conj().T, 2) <= 1e-9 * lam_ref[0] / gap


def test_gevd_identity_noise_is_sevd(orc):
    rng = np.random.default_rng(53)
    M, Ns, F = 10, 2, 2
    R = orc.corr(crandn(rng, F, 30, M).astype(np.complex64))
    K = np.broadcast_to(np.eye(M, dtype=complex), (F, M, M)).copy()
    En, sig, st = orc.gevd(K, R, Ns)
    for f in range(F):
        w, V = np.linalg.eigh(R[f])
        Pn = V[:, :M - Ns] @ V[:, :M - Ns].conj().T
        E = En[f].T
        assert np.linalg.norm(E @ E.conj().T - Pn, 2) <= 1e-11
        assert np.allclose(sig[f], w[::-1], rtol=1e-11, atol=1e-12 * w[-1])


def test_gevd_planted_sources_are_nulled(orc):
    """Noise-free R = H_s S H_s^H with coloured K: the generalized noise vectors are orthogonal to
    the source steering vectors themselves (h_s^H e = 0), the property that places the MUSIC
    peaks."""
    rng = np.random.default_rng(54)
    M, Ns, F = 12, 2, 1
    Hs = crandn(rng, M, Ns)
    S = np.diag([3.0, 1.5])
    R = (Hs @ S @ Hs.conj().T)[None]
    K = random_pd(rng, M, 50.0)[None]
    En, sig, st = orc.gevd(K, R, Ns)
    assert st[0] == 0
    E = En[0].T
    assert np.max(np.abs(Hs.conj().T @ E)) <= 1e-10 * np.linalg.norm(Hs) * np.linalg.norm(E)
