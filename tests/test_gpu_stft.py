"""eq.1 front end: ssl_stft (FP32 radix-2 FFT in LDS) against the oracle's direct FP64 DFT, and the
whole path from time-domain PCM (STFT -> correlation -> GSVD -> spectrum -> peaks) against the
oracle's.  MI355X only."""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import U32, peak_ambiguity, to_dev, to_host

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    import paper_2504_03373_amd as S
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    S.lib()
    return S


@pytest.fixture(scope="module")
def ctx(S):
    c = S.ssl_ctx_create(0, 0)
    yield c
    S.ssl_ctx_destroy(c)


def gpu_stft(S, ctx, pcm, nfft, hop, T, window=None):
    import torch
    M = pcm.shape[1]
    X = torch.full((nfft // 2 + 1, T, M), complex(7.0, 7.0), dtype=torch.complex64,
                   device="cuda:0")
    S.ssl_stft(ctx, to_dev(pcm), nfft, hop, T, X,
               None if window is None else to_dev(window.astype(np.float32)))
    return to_host(X)


@pytest.mark.parametrize("nfft,hop,T,M,custom", [(16, 5, 7, 1, False), (64, 16, 10, 3, True),
                                                 (512, 160, 50, 60, False), (512, 160, 50, 8, True),
                                                 (1024, 256, 12, 17, False), (4096, 1000, 3, 5, True)])
def test_stft_parity(S, ctx, nfft, hop, T, M, custom):
    """Norm-wise per frame and channel: |dX| <= (8 log2 N + 4) u sqrt(N) |w x| (the FFT's
    forward error with FP32 twiddles, plus the window and product roundings)."""
    say(f"ssl_stft nfft={nfft} hop={hop} T={T} M={M} window={'custom' if custom else 'hann'}")
    rng = np.random.default_rng(nfft + M)
    n = (T - 1) * hop + nfft + 11
    pcm = rng.standard_normal((n, M)).astype(np.float32)
    win = rng.uniform(0.1, 1.0, nfft) if custom else None
    if custom:
        win = win.astype(np.float32).astype(np.float64)      # the bytes the GPU reads
    g = gpu_stft(S, ctx, pcm, nfft, hop, T, win)
    r = oracle.stft(pcm, nfft, hop, T, win)
    w = oracle.hann(nfft) if win is None else win
    frames = np.stack([pcm[t * hop:t * hop + nfft].astype(np.float64) for t in range(T)], axis=1)
    wx = np.linalg.norm(w[:, None, None] * frames, axis=0)                     # [T][M]
    err = np.linalg.norm(g.astype(np.complex128) - r, axis=0)                  # [T][M]
    bound = (8 * np.log2(nfft) + 4) * U32 * np.sqrt(nfft) * wx
    say(f"  max err / (u sqrt(N) |wx|) = {np.max(err / (U32 * np.sqrt(nfft) * wx)):.2f}")
    assert np.all(err <= bound)


def test_stft_argument_errors(S, ctx):
    import torch
    say("ssl_stft argument errors")
    pcm = torch.zeros((1000, 4), dtype=torch.float32, device="cuda:0")
    X = torch.zeros((257, 5, 4), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_stft(ctx, pcm, 512, 160, 5, X)                 # 4 * 160 + 512 > 1000 samples
    assert e.value.code == S.SSL_ERR_ARG
    X2 = torch.zeros((151, 3, 4), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_stft(ctx, pcm, 300, 100, 3, X2)               # not a power of two
    assert e.value.code == S.SSL_ERR_ARG


@pytest.mark.parametrize("M", [8, 60])
def test_pcm_to_peaks_matches_oracle(S, ctx, M):
    """Time-domain scene -> ssl_stft -> noise handle from the STFT of noise-only PCM -> ssl_localize,
    against the oracle's STFT and localization on the same PCM: Pbar within 1e-4, the same peaks,
    and the planted sources found."""
    import torch
    w, pcm_block, noise = synth.pcm_workload(M)
    nfft, hop, T = 512, 160, 50
    Tn = (noise.shape[0] - nfft) // hop + 1
    say(f"PCM -> peaks M={M}: noise {noise.shape} ({Tn} frames)")
    Xn = torch.zeros((nfft // 2 + 1, Tn, M), dtype=torch.complex64, device="cuda:0")
    S.ssl_stft(ctx, to_dev(noise), nfft, hop, Tn, Xn)
    Kd = torch.zeros((w.F, M, M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, Xn, 1.0 / Tn, 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    K_ref = oracle.noise_corr(oracle.stft(noise, nfft, hop, Tn).astype(np.complex64))
    H = w.steering_table()
    Hd = to_dev(H)
    for b in range(2):
        pcm, dirs = pcm_block(b)
        say(f"  block {b}: planted {dirs}")
        X = torch.zeros((nfft // 2 + 1, T, M), dtype=torch.complex64, device="cuda:0")
        S.ssl_stft(ctx, to_dev(pcm), nfft, hop, T, X)
        pk = torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0")
        pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
        Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
        st = torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0")
        S.ssl_localize(ctx, X, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, pk, pv, Pbar,
                       st)
        g_pk, g_Pbar, g_st = to_host(pk), to_host(Pbar), to_host(st)
        X_ref = oracle.stft(pcm, nfft, hop, T).astype(np.complex64)
        r = oracle.localize(X_ref, K_ref, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16)
        rel = float(np.max(np.abs(g_Pbar.astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
        say(f"    rel {rel:.2e} peaks gpu {g_pk} ref {r['peaks']} near-ties {amb}")
        assert np.all(g_st == 0) and np.all(r["status"] == 0)
        assert rel <= 1e-4
        assert not amb
        assert np.array_equal(g_pk, r["peaks"])
        assert sorted(g_pk.tolist()) == sorted(dirs)
    S.ssl_noise_destroy(n)
