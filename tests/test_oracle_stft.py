"""Pins of the oracle's eq.1 front end (orc_stft, orc_hann), independent of its code: the
library real FFT of the windowed frames, closed forms of a sinusoid, Parseval, the frame and
channel indexing of an impulse, and the window itself."""
import numpy as np
import pytest


def test_hann_closed_form(orc):
    for N in (16, 512):
        n = np.arange(N)
        assert np.allclose(orc.hann(N), np.sin(np.pi * n / N) ** 2, rtol=0, atol=1e-15)
        w = orc.hann(N)
        assert w[0] == 0.0 and abs(w[N // 2] - 1.0) < 1e-15
        assert np.allclose(w[1:], w[1:][::-1], rtol=0, atol=1e-15)      # periodic symmetry


@pytest.mark.parametrize("N,hop,T,M", [(16, 5, 7, 1), (64, 16, 10, 3), (512, 160, 6, 4)])
def test_stft_matches_library_rfft(orc, N, hop, T, M):
    rng = np.random.default_rng(N + M)
    n = (T - 1) * hop + N + 3
    pcm = rng.standard_normal((n, M)).astype(np.float32)
    for win in (None, rng.uniform(0.2, 1.0, N)):
        X = orc.stft(pcm, N, hop, T, win)
        w = orc.hann(N) if win is None else win
        ref = np.stack([np.fft.rfft(w[:, None] * pcm[t * hop:t * hop + N].astype(np.float64), axis=0)
                        for t in range(T)], axis=1)
        assert X.shape == (N // 2 + 1, T, M)
        assert np.max(np.abs(X - ref)) <= 1e-12 * np.sqrt(N) * np.max(np.abs(pcm))


def test_stft_sinusoid_closed_form(orc):
    """x[n] = cos(2 pi k0 n / N): rectangular window gives N/2 at k0 and 0 elsewhere; the Hann
    window gives N/4 at k0 and -N/8 at k0 +- 1."""
    N, k0 = 64, 5
    n = np.arange(N)
    pcm = np.cos(2 * np.pi * k0 * n / N).astype(np.float32)[:, None]
    x32 = pcm[:, 0].astype(np.float64)
    Xr = orc.stft(pcm, N, N, 1, np.ones(N))[:, 0, 0]
    want = np.zeros(N // 2 + 1, complex)
    want[k0] = N / 2
    tol = N * np.max(np.abs(x32 - np.cos(2 * np.pi * k0 * n / N))) + 1e-12
    assert np.max(np.abs(Xr - want)) <= tol
    Xh = orc.stft(pcm, N, N, 1)[:, 0, 0]
    want = np.zeros(N // 2 + 1, complex)
    want[k0], want[k0 - 1], want[k0 + 1] = N / 4, -N / 8, -N / 8
    assert np.max(np.abs(Xh - want)) <= tol


def test_stft_parseval(orc):
    rng = np.random.default_rng(3)
    N = 128
    pcm = rng.standard_normal((N, 2)).astype(np.float32)
    X = orc.stft(pcm, N, N, 1, np.ones(N))[:, 0, :]
    c = np.full(N // 2 + 1, 2.0)
    c[0] = c[-1] = 1.0
    energy = np.sum(c[:, None] * np.abs(X) ** 2, axis=0) / N
    assert np.allclose(energy, np.sum(pcm.astype(np.float64) ** 2, axis=0), rtol=1e-12)


def test_stft_impulse_frames_and_channels(orc):
    """A unit impulse at sample s of channel m appears in exactly the frames that cover s, in
    channel m only, as win[s - t hop] e^{-2 pi i w (s - t hop) / N}."""
    N, hop, T, M = 32, 8, 9, 3
    s, m = 37, 2
    pcm = np.zeros(((T - 1) * hop + N, M), np.float32)
    pcm[s, m] = 1.0
    X = orc.stft(pcm, N, hop, T)
    w = orc.hann(N)
    k = np.arange(N // 2 + 1)
    for t in range(T):
        d = s - t * hop
        want = np.zeros(N // 2 + 1, complex)
        if 0 <= d < N:
            want = w[d] * np.exp(-2j * np.pi * k * d / N)
        assert np.max(np.abs(X[:, t, m] - want)) <= 1e-14
        assert np.all(X[:, t, :m] == 0) and np.all(X[:, t, m + 1:] == 0)


def test_stft_rejects_short_input(orc):
    with pytest.raises(ValueError):
        orc.stft(np.zeros((100, 2), np.float32), 64, 16, 4)
