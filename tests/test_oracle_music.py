"""Pins for the oracle's GSVD noise subspace, MUSIC spectrum (eq.5), bin sum (eq.6) and peak search.

Anchors: the K = I reduction to standard SEVD-MUSIC (LAPACK eigh), planted
noise-free sources (exact orthogonality), invariances the mathematics fixes
(scale, channel permutation, rotation inside E_n for p = 2, the rotational
symmetry of a uniform circular array), library evaluation of the spectrum,
hand-derived peak fixtures and a scipy maximum-filter cross-check.
"""
import json
import os

import numpy as np
import pytest

import synth
from conftest import crandn, projector, random_pd, random_unitary

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _planted(M, Ns, dirs_az, F=4, pos=None, el=0.0):
    pos = synth.circle_array(M, 0.1) if pos is None else pos
    freqs = synth.bin_freqs(F, 16000.0, 2 * (F - 1)) + 500.0           # avoid the DC bin
    u = synth.unit_vector(np.asarray(dirs_az, float), np.full(len(dirs_az), el))
    Hs = synth.steering(pos, u, freqs)                                  # [F][Ns][M]
    return Hs, freqs, pos


def test_sevd_reduction_when_K_is_identity(orc):
    """K = I: the GSVD noise subspace is the eigen-subspace of the M - Ns smallest eigenvalues of R."""
    rng = np.random.default_rng(20)
    F, T, M, Ns = 3, 40, 8, 2
    X = crandn(rng, F, T, M).astype(np.complex64)
    R = orc.corr(X)
    K = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    En, sig, st, _ = orc.gsvd(K, R, Ns)
    assert np.all(st == orc.OK)
    for f in range(F):
        w, V = np.linalg.eigh(R[f])                       # ascending eigenvalues
        assert np.max(np.abs(sig[f] - w[::-1])) <= 1e-12 * w[-1]
        relgap = (w[M - Ns] - w[M - Ns - 1]) / w[-1]
        err = np.linalg.norm(projector(En[f].T) - projector(V[:, :M - Ns]), 2)
        assert err <= 1e-12 / relgap


def test_planted_sources_identity_noise(orc):
    """Noise-free R = H_s S H_s^H with K = I: E_n is orthogonal to the source steering vectors and
    the spectrum at the source directions is (numerically) unbounded."""
    M, Ns = 8, 2
    grid = synth.DirectionGrid(72, 1)
    src = [10, 40]
    Hs, freqs, pos = _planted(M, Ns, [5.0 * d for d in src])
    F = freqs.shape[0]
    S = np.diag([2.0, 0.7])
    R = np.einsum("fsm,st,ftn->fmn", Hs.transpose(0, 1, 2), S, Hs.conj())   # sum_s p_s h_s h_s^H
    K = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    En, sig, st, _ = orc.gsvd(K, R, Ns)
    for f in range(F):
        hs = Hs[f].T                                        # [M][Ns]
        assert np.linalg.norm(hs.conj().T @ En[f].T) <= 1e-13 * np.linalg.norm(hs)
    H = synth.steering(pos, grid.unit_vectors(), freqs).astype(np.complex64)
    P, Pbar = orc.spectrum(H, En, Ns)
    pk, _ = orc.peaks(Pbar, 1, 72, Ns)
    assert sorted(pk.tolist()) == src
    others = np.delete(Pbar, src)
    assert Pbar[src].min() > 1e6 * others.max()


def test_planted_sources_general_noise(orc):
    """With K != I the GSVD noise subspace annihilates K^{-1} h_s (left singular vectors of K^{-1}R)."""
    rng = np.random.default_rng(21)
    M, Ns = 8, 2
    Hs, freqs, pos = _planted(M, Ns, [30.0, 120.0])
    F = freqs.shape[0]
    R = np.einsum("fsm,fsn->fmn", Hs, Hs.conj())
    K = np.stack([random_pd(rng, M, 50.0) for _ in range(F)])
    En, sig, st, _ = orc.gsvd(K, R, Ns)
    for f in range(F):
        kh = np.linalg.solve(K[f], Hs[f].T)
        assert np.linalg.norm(kh.conj().T @ En[f].T) <= 1e-13 * np.linalg.norm(kh)
        assert np.all(sig[f, Ns:] <= 1e-13 * sig[f, 0])


def test_spectrum_matches_library_evaluation(orc):
    rng = np.random.default_rng(22)
    F, D, M, Ns = 3, 11, 6, 2
    H = crandn(rng, F, D, M).astype(np.complex64)
    En = np.stack([random_unitary(rng, M)[:, Ns:].T for _ in range(F)])
    Hd = H.astype(np.complex128)
    for p in (1, 2):
        P, Pbar = orc.spectrum(H, En, Ns, p=p)
        G = np.einsum("fdm,fcm->fdc", Hd.conj(), En)        # H^H e_c
        den = np.sum(np.abs(G) ** p, axis=2)
        num = np.sum(np.abs(Hd) ** 2, axis=2)
        assert np.max(np.abs(P - num / den) / (num / den)) <= 1e-13
        assert np.max(np.abs(Pbar - P.sum(0)) / Pbar) <= 1e-14
    # p = 2 depends only on the projector: den = h^H (E E^H) h
    P2, _ = orc.spectrum(H, En, Ns, p=2)
    for f in range(F):
        Pi = projector(En[f].T)
        den = np.einsum("dm,mn,dn->d", Hd[f].conj(), Pi, Hd[f]).real
        num = np.sum(np.abs(Hd[f]) ** 2, axis=1)
        assert np.max(np.abs(P2[f] - num / den) / P2[f]) <= 1e-12


def test_p1_single_noise_vector_reduces_to_projector_form(orc):
    """p = 1 (eq.5 as printed) pinned where the noise subspace is one vector, unique up to phase:
    with M - Ns = 1, |H^H e| = sqrt(H^H Pi H), so P_1 = |H|^2 / sqrt(H^H Pi H) exactly, Pi being
    the projector onto the null vector that LAPACK's SVD gives for a rank-(M-1) matrix.  A dropped
    conjugate, a missing absolute value or a p = 2 square would fail it."""
    rng = np.random.default_rng(28)
    F, D, M = 3, 13, 6
    Ns = M - 1
    H = crandn(rng, F, D, M).astype(np.complex64)
    Hd = H.astype(np.complex128)
    En, want = [], []
    for f in range(F):
        B = crandn(rng, M - 1, M)                          # rank M - 1: null space of dim 1
        e = np.linalg.svd(B)[2][-1].conj()                 # B e = 0, |e| = 1
        assert np.linalg.norm(B @ e) <= 1e-13 * np.linalg.norm(B)
        e = e * np.exp(1j * rng.uniform(0, 2 * np.pi))      # arbitrary phase
        En.append(e[None, :])
        Pi = np.outer(e, e.conj())
        num = np.sum(np.abs(Hd[f]) ** 2, axis=1)
        quad = np.einsum("dm,mn,dn->d", Hd[f].conj(), Pi, Hd[f]).real
        want.append(num / np.sqrt(quad))
    En = np.stack(En)
    P1, Pbar1 = orc.spectrum(H, En, Ns, p=1)
    P2, _ = orc.spectrum(H, En, Ns, p=2)
    want = np.stack(want)
    assert np.max(np.abs(P1 - want) / want) <= 1e-13
    num = np.sum(np.abs(Hd) ** 2, axis=2)
    assert np.max(np.abs(P1 - np.sqrt(num * P2)) / P1) <= 1e-13     # P_1 = sqrt(|h|^2 P_2)
    assert np.max(np.abs(Pbar1 - want.sum(0)) / Pbar1) <= 1e-14


def test_p1_standard_basis_noise_vectors(orc):
    """p = 1 with coordinate vectors as the noise basis: sum_i |H^H e_i| = sum_{m in N} |H_m|
    (closed form); the result is unchanged by a phase on each noise vector and by their order,
    the two freedoms of an SVD with distinct singular values."""
    rng = np.random.default_rng(29)
    F, D, M, Ns = 2, 7, 5, 2
    H = crandn(rng, F, D, M).astype(np.complex64)
    Hd = H.astype(np.complex128)
    I = np.eye(M, dtype=np.complex128)
    En = np.stack([I[:, [4, 1, 3]].T for _ in range(F)])       # noise channels {1, 3, 4}
    P1, _ = orc.spectrum(H, En, Ns, p=1)
    num = np.sum(np.abs(Hd) ** 2, axis=2)
    den = np.abs(Hd[..., 1]) + np.abs(Hd[..., 3]) + np.abs(Hd[..., 4])
    assert np.max(np.abs(P1 - num / den) / P1) <= 1e-14
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, (F, M - Ns)))
    En2 = (En * ph[..., None])[:, ::-1]
    P1b, _ = orc.spectrum(H, np.ascontiguousarray(En2), Ns, p=1)
    assert np.max(np.abs(P1b - P1) / P1) <= 1e-14


def test_p1_planted_source_is_unbounded(orc):
    """Noise-free planted sources with K = I: H_s^H e_i = 0 for every noise vector, so the p = 1
    spectrum is unbounded at the sources as well (the floor DBL_MIN in the denominator)."""
    M, Ns = 8, 2
    grid = synth.DirectionGrid(72, 1)
    src = [12, 50]
    Hs, freqs, pos = _planted(M, Ns, [5.0 * d for d in src])
    F = freqs.shape[0]
    R = np.einsum("fsm,fsn->fmn", Hs, Hs.conj())
    K = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    En, _, st, _ = orc.gsvd(K, R, Ns)
    H = synth.steering(pos, grid.unit_vectors(), freqs).astype(np.complex64)
    P1, Pbar1 = orc.spectrum(H, En, Ns, p=1)
    pk, _ = orc.peaks(Pbar1, 1, 72, Ns)
    assert sorted(pk.tolist()) == src
    assert Pbar1[src].min() > 1e6 * np.delete(Pbar1, src).max()


def test_failed_bins_contribute_zero(orc):
    rng = np.random.default_rng(23)
    F, D, M, Ns = 4, 5, 4, 1
    H = crandn(rng, F, D, M).astype(np.complex64)
    En = np.stack([random_unitary(rng, M)[:, Ns:].T for _ in range(F)])
    st = np.array([0, 1, 0, 2], np.int32)
    P, Pbar = orc.spectrum(H, En, Ns, status=st)
    assert np.all(P[1] == 0) and np.all(P[3] == 0)
    P_all, _ = orc.spectrum(H, En, Ns)
    assert np.allclose(Pbar, P_all[0] + P_all[2], rtol=1e-15, atol=0)


def test_scale_invariance(orc):
    """R -> c R and K -> c' K leave E_n (as a projector) and P unchanged."""
    w = synth.workload_small(n_blocks=1)
    w.F = 9
    w.freqs = w.freqs[:9]
    X, _, _ = w.block(0)
    Kn = orc.noise_corr(w.noise_frames())
    R = orc.corr(X)
    H = w.steering_table()
    E1, s1, st1, _ = orc.gsvd(Kn, R, 1)
    E2, s2, st2, _ = orc.gsvd(0.25 * Kn, 3.7 * R, 1)
    assert np.all(st1 == 0) and np.all(st2 == 0)
    for f in range(1, 9):
        relgap = (s1[f, 0] - s1[f, 1]) / s1[f, 0]
        assert np.linalg.norm(projector(E1[f].T) - projector(E2[f].T), 2) <= 1e-12 / relgap
    P1, _ = orc.spectrum(H, E1, 1)
    P2, _ = orc.spectrum(H, E2, 1)
    assert np.max(np.abs(P1[1:] - P2[1:]) / P1[1:]) <= 1e-9


def test_channel_permutation_invariance(orc):
    w = synth.workload_small(n_blocks=1)
    X, _, _ = w.block(0)
    Xn = w.noise_frames()
    H = w.steering_table()
    perm = np.random.default_rng(24).permutation(8)
    o1 = orc.localize(X, orc.noise_corr(Xn), H, 72, 1, 1, want_P=True)
    o2 = orc.localize(np.ascontiguousarray(X[..., perm]), orc.noise_corr(np.ascontiguousarray(Xn[..., perm])),
                      np.ascontiguousarray(H[..., perm]), 72, 1, 1, want_P=True)
    assert np.max(np.abs(o1["Pbar"] - o2["Pbar"]) / o1["Pbar"]) <= 1e-10
    assert np.array_equal(o1["peaks"], o2["peaks"])


def test_p2_invariant_under_rotation_inside_noise_subspace(orc):
    rng = np.random.default_rng(25)
    F, D, M, Ns = 2, 9, 7, 3
    H = crandn(rng, F, D, M).astype(np.complex64)
    En = np.stack([random_unitary(rng, M)[:, Ns:].T for _ in range(F)])
    Q = random_unitary(rng, M - Ns)
    En2 = np.einsum("fcm,cd->fdm", En, Q)                 # E_n -> E_n Q
    P1, _ = orc.spectrum(H, En, Ns, p=2)
    P2, _ = orc.spectrum(H, En2, Ns, p=2)
    assert np.max(np.abs(P1 - P2) / P1) <= 1e-12
    P1, _ = orc.spectrum(H, En, Ns, p=1)                  # p = 1 is not invariant
    P2, _ = orc.spectrum(H, En2, Ns, p=1)
    assert np.max(np.abs(P1 - P2) / P1) > 1e-6


def test_uniform_circular_array_rotation(orc):
    """8-mic circle, 5 degree azimuth grid: shifting channels by one (a 45 degree array rotation)
    cyclically shifts P-bar by 9 azimuth steps."""
    w = synth.workload_small(n_blocks=1)
    X, _, _ = w.block(0)
    Xn = w.noise_frames()
    H = w.steering_table()
    sh = np.roll(np.arange(8), -1)                        # channel m <- m + 1
    o1 = orc.localize(X, orc.noise_corr(Xn), H, 72, 1, 1)
    o2 = orc.localize(np.ascontiguousarray(X[..., sh]), orc.noise_corr(np.ascontiguousarray(Xn[..., sh])),
                      H, 72, 1, 1)
    shifted = np.roll(o1["Pbar"], -9)
    assert np.max(np.abs(o2["Pbar"] - shifted) / shifted) <= 1e-6
    assert not np.allclose(o2["Pbar"], o1["Pbar"], rtol=1e-3)


def test_small_workload_localizes_planted_source(orc):
    """At 10 dB SNR the 8-mic workload's oracle finds the planted azimuth in every block."""
    w = synth.workload_small(n_blocks=3)
    K = orc.noise_corr(w.noise_frames())
    H = w.steering_table()
    for b in range(3):
        X, dirs, _ = w.block(b)
        o = orc.localize(X, K, H, 72, 1, 1, nthreads=4)
        assert np.all(o["status"] == 0)
        assert o["peaks"][0] == dirs[0]


# ----------------------------------------------------------------------------
# peaks
# ----------------------------------------------------------------------------
def test_peak_fixtures(orc):
    with open(os.path.join(GOLDEN, "peaks_cases.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        pk, vals = orc.peaks(np.asarray(c["Pbar"], float), c["n_el"], c["n_az"], c["Ns"])
        assert pk.tolist() == c["peaks"], c["name"]
        for k, d in enumerate(c["peaks"]):
            assert vals[k] == (c["Pbar"][d] if d >= 0 else 0.0)


def test_peaks_match_maximum_filter(orc):
    """Tie-free random grids: the local maxima are where a 3x3 maximum filter (azimuth wrapped,
    elevation padded with -inf) leaves the value unchanged; ranking by value."""
    ndi = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(26)
    for n_el, n_az in [(1, 72), (19, 72), (3, 7), (5, 2)]:
        for _ in range(5):
            v = rng.permutation(n_el * n_az).astype(float).reshape(n_el, n_az)
            padded = np.pad(v, ((1, 1), (0, 0)), constant_values=-np.inf)
            mf = ndi.maximum_filter(padded, size=(3, 3), mode="wrap")[1:-1]
            cand = np.flatnonzero((v == mf).ravel())
            order = cand[np.argsort(-v.ravel()[cand], kind="stable")]
            Ns = 4
            want = list(order[:Ns]) + [-1] * (Ns - min(Ns, len(order)))
            pk, _ = orc.peaks(v.ravel(), n_el, n_az, Ns)
            assert pk.tolist() == want


def test_peaks_invariant_under_monotone_map(orc):
    rng = np.random.default_rng(27)
    v = rng.random(19 * 72)
    a, _ = orc.peaks(v, 19, 72, 3)
    b, _ = orc.peaks(np.exp(3 * v) + 2.0, 19, 72, 3)
    assert np.array_equal(a, b)
