"""Frame stream (eq.3's window of the T frames ending at each frame): the FP64 rank-2 updated
correlation against the direct window sum, and cold and warm-started localizations of successive
windows against the oracle run on each window.  MI355X only."""
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import crandn
from gpu_util import peak_ambiguity, to_dev, to_host

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


@pytest.mark.parametrize("F,M,T,chunks", [(9, 12, 10, [1, 3, 7, 1, 1, 12, 2, 25, 1]),
                                          (5, 60, 50, [50, 1, 1, 30, 49, 1, 70])])
def test_sliding_corr_is_the_window_sum(S, ctx, F, M, T, chunks):
    import torch
    say(f"ssl_sliding_push F={F} M={M} T={T} chunks {chunks}")
    rng = np.random.default_rng(F * M + T)
    N = sum(chunks)
    X = crandn(rng, F, N, M).astype(np.complex64)
    Xd = to_dev(X)
    s = S.ssl_sliding_create(ctx, F, M, T)
    R = torch.zeros((F, M, M), dtype=torch.complex128, device="cuda:0")
    f = 0
    Xa = np.abs(X.astype(np.complex128))
    for n in chunks:
        S.ssl_sliding_push(s, Xd[:, f:f + n, :])
        f += n
        assert S.ssl_sliding_frames(s) == f
        if f < T:
            continue
        S.ssl_sliding_corr(s, R)
        ref = oracle.sliding_corr(X, T, f - 1)
        W = Xa[:, f - T:f]
        bound = 1e-12 * np.einsum("fti,ftj->fij", W, W) / T + 1e-300
        assert np.all(np.abs(to_host(R) - ref) <= bound), f
    S.ssl_sliding_destroy(s)


def test_sliding_state_errors(S, ctx):
    import torch
    say("ssl_sliding errors")
    s = S.ssl_sliding_create(ctx, 4, 8, 10)
    X = torch.zeros((4, 5, 8), dtype=torch.complex64, device="cuda:0")
    S.ssl_sliding_push(s, X)
    H = torch.zeros((4, 72, 8), dtype=torch.complex64, device="cuda:0")
    pk = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    pv = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    with pytest.raises(S.SSLError) as e:                     # 5 frames, the window needs 10
        S.ssl_sliding_localize(s, None, H, S.SSL_FP32, 72, 1, 1, 2, 0, pk, pv)
    assert e.value.code == S.SSL_ERR_STATE
    S.ssl_sliding_destroy(s)
    with pytest.raises(S.SSLError) as e:
        S.ssl_sliding_create(ctx, 4, 65, 10)
    assert e.value.code == S.SSL_ERR_ARG


def frame_sequence(w, blocks):
    """Consecutive blocks of a workload as one frame sequence [F][50 * len(blocks)][M]."""
    return np.ascontiguousarray(np.concatenate([w.block(b)[0] for b in blocks], axis=1))


@pytest.mark.parametrize("name", ["small", "paper"])
def test_sliding_localize_matches_oracle_per_window(S, ctx, name):
    """Windows ending at frames 49, 59, .., 99 of two consecutive blocks (the sources change
    between them): cold and warm-started solves, each against the oracle on the same window."""
    import torch
    w = synth.workload_small(n_blocks=4) if name == "small" else synth.workload_paper(n_blocks=4)
    X = frame_sequence(w, [0, 1])
    T, hop = 50, 10
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    K = oracle.noise_corr(Xn)
    H = w.steering_table()
    Hd = to_dev(H)
    Xd = to_dev(X)
    states = {warm: S.ssl_sliding_create(ctx, w.F, w.M, T) for warm in (0, 1)}
    for st_ in states.values():
        S.ssl_sliding_push(st_, Xd[:, :T - hop, :])
    for f in range(T - 1, X.shape[1], hop):
        r = oracle.localize_frame(X, T, f, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16)
        for warm, st_ in states.items():
            S.ssl_sliding_push(st_, Xd[:, f - hop + 1:f + 1, :])
            pk = torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0")
            pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
            Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
            bst = torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0")
            conv = torch.zeros((w.F, 3), dtype=torch.int32, device="cuda:0")
            S.ssl_sliding_localize(st_, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, warm,
                                   pk, pv, Pbar, bst, conv)
            g_pk, g_P, g_st, g_cv = to_host(pk), to_host(Pbar), to_host(bst), to_host(conv)
            rel = float(np.max(np.abs(g_P.astype(np.float64) - r["Pbar"]) / r["Pbar"]))
            amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
            say(f"  {name} frame {f} {'warm' if warm else 'cold'}: sweeps {g_cv[:, 0].mean():.2f} "
                f"rel {rel:.2e} peaks {g_pk} ref {r['peaks']} near-ties {amb}")
            assert np.all(g_st == 0) and np.all(r["status"] == 0)
            assert rel <= 1e-4
            assert not amb
            assert np.array_equal(g_pk, r["peaks"])
    for st_ in states.values():
        S.ssl_sliding_destroy(st_)
    S.ssl_noise_destroy(n)
