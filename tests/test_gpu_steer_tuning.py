"""Projection (eq.5) tile shapes -- waves per workgroup -- and their autotuner.

A direction's value is computed by one wave in the same order whatever the tile shape, so every
variant must give bit-identical P and Pbar, on the single-block and the batched entry points; the
default variant's parity against the oracle is covered by the spectrum parity tests.  The
autotuner must time every candidate, return one of them and record it in the context.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import U32, to_dev, to_host

pytestmark = pytest.mark.gpu

WAVES = (4, 8, 16)


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


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def h_table(S, H, prec):
    import torch
    Hd = to_dev(H)
    if prec == S.SSL_FP32:
        return Hd
    F, D, M = H.shape
    dt = torch.bfloat16 if prec == S.SSL_BF16 else torch.float16
    return torch.view_as_real(Hd).reshape(F, D, 2 * M).to(dt).contiguous()


def spectrum(S, ctx, Hd, prec, En, Ns, F, D, p=2):
    import torch
    P = torch.zeros((F, D), dtype=torch.float32, device="cuda:0")
    Pbar = torch.zeros(D, dtype=torch.float32, device="cuda:0")
    S.ssl_music_spectrum(ctx, Hd, prec, to_dev(En), Ns, p, P, Pbar, None, F=F, D=D, M=En.shape[2])
    return to_host(P), to_host(Pbar)


# one case per noise-subspace class (M - Ns <= 16, <= 32, <= 64), ragged direction counts
CASES = [(8, 1, 72), (16, 3, 300), (33, 2, 129), (60, 2, 1368), (64, 1, 257)]


@pytest.mark.parametrize("M,Ns,D", CASES)
@pytest.mark.parametrize("pname", ["fp32", "bf16", "fp16"])
def test_steer_variants_bit_identical(S, M, Ns, D, pname):
    prec = {"fp32": S.SSL_FP32, "bf16": S.SSL_BF16, "fp16": S.SSL_FP16}[pname]
    rng = np.random.default_rng(900 + M + D)
    F = 9
    H = crandn(rng, F, D, M).astype(np.complex64)
    En = np.stack([np.linalg.qr(crandn(rng, M, M))[0][:, Ns:].T for _ in range(F)]).astype(np.complex64)
    Hd = h_table(S, H, prec)
    ctx = S.ssl_ctx_create(0, 0)
    assert S.ssl_ctx_get_steer_waves(ctx, M, Ns, prec) == 8
    out = {}
    for wv in WAVES:
        say(f"ssl_music_spectrum {pname} M={M} Ns={Ns} D={D} waves={wv}")
        S.ssl_ctx_set_steer_waves(ctx, M, Ns, prec, wv)
        assert S.ssl_ctx_get_steer_waves(ctx, M, Ns, prec) == wv
        out[wv] = spectrum(S, ctx, Hd, prec, En, Ns, F, D)
    for wv in WAVES:
        assert np.array_equal(out[wv][0], out[8][0]), wv
        assert np.array_equal(out[wv][1], out[8][1]), wv
    if prec == S.SSL_FP32:
        Pr, _ = oracle.spectrum(H, En.astype(np.complex128), Ns, p=2)
        rel = np.abs(out[4][0] - Pr) / Pr
        assert np.max(rel) <= 16 * M * U32 * np.max(Pr) / np.min(Pr) + 1e-5
    S.ssl_ctx_destroy(ctx)


def test_steer_waves_rejects_unavailable(S):
    ctx = S.ssl_ctx_create(0, 0)
    for bad in (0, 2, 12, 32):
        with pytest.raises(S.SSLError):
            S.ssl_ctx_set_steer_waves(ctx, 60, 2, S.SSL_BF16, bad)
    with pytest.raises(S.SSLError):
        S.ssl_ctx_set_steer_waves(ctx, 60, 2, S.SSL_FP64, 4)
    assert S.ssl_ctx_get_steer_waves(ctx, 60, 2, S.SSL_FP64) == -1
    # classes and precisions are independent
    S.ssl_ctx_set_steer_waves(ctx, 60, 2, S.SSL_BF16, 16)
    assert S.ssl_ctx_get_steer_waves(ctx, 60, 2, S.SSL_FP32) == 8
    assert S.ssl_ctx_get_steer_waves(ctx, 8, 1, S.SSL_BF16) == 8
    S.ssl_ctx_destroy(ctx)


def test_steer_autotune(S):
    rng = np.random.default_rng(950)
    M, Ns, F, D = 60, 2, 33, 1368
    H = crandn(rng, F, D, M).astype(np.complex64)
    En = np.stack([np.linalg.qr(crandn(rng, M, M))[0][:, Ns:].T for _ in range(F)]).astype(np.complex64)
    ctx = S.ssl_ctx_create(0, 0)
    Hd = h_table(S, H, S.SSL_BF16)
    for nb in (1, 8):
        say(f"ssl_autotune_steer bf16 M=60 F=33 D=1368 nblocks={nb}")
        best, ms = S.ssl_autotune_steer(ctx, Hd, S.SSL_BF16, to_dev(En), Ns, nblocks=nb, reps=2)
        say(f"  best {best} waves, ms {ms}")
        assert best in WAVES
        assert sorted(ms) == list(WAVES) and all(v > 0 for v in ms.values())
        assert ms[best] == min(ms.values())
        assert S.ssl_ctx_get_steer_waves(ctx, M, Ns, S.SSL_BF16) == best
    with pytest.raises(S.SSLError):
        S.ssl_autotune_steer(ctx, Hd, S.SSL_BF16, to_dev(En), Ns, nblocks=0)
    S.ssl_ctx_destroy(ctx)


def test_steer_variant_applies_to_batch(S):
    """Batched and single-block outputs stay bit-identical under a non-default tile shape (of the
    noise-vector projection, which the tile variants belong to)."""
    import torch
    import synth
    ctx = S.ssl_ctx_create(0, 0)
    S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_NOISE)
    w = synth.workload_paper(n_blocks=4)
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    Hd = h_table(S, w.steering_table(), S.SSL_BF16)
    Xs = [to_dev(w.block(b)[0]) for b in range(3)]
    mk = lambda: (torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
                  torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
                  torch.zeros(w.D, dtype=torch.float32, device="cuda:0"))
    res = {}
    for wv in (16, 4):
        S.ssl_ctx_set_steer_waves(ctx, w.M, w.Ns, S.SSL_BF16, wv)
        single = []
        for X in Xs:
            pk, pv, pb = mk()
            S.ssl_localize(ctx, X, n, Hd, S.SSL_BF16, 72, 19, w.Ns, 2, pk, pv, pb)
            single.append((to_host(pk), to_host(pb)))
        outs = [mk() for _ in Xs]
        say(f"ssl_localize_batch bf16 with {wv} waves per projection workgroup")
        S.ssl_localize_batch(ctx, [S.block_desc(X, n, Hd, 72, 19, w.Ns, o[0], o[1], o[2])
                                   for X, o in zip(Xs, outs)], S.SSL_BF16, 2)
        for (pk, pb), o in zip(single, outs):
            assert np.array_equal(pk, to_host(o[0])) and np.array_equal(pb, to_host(o[2]))
        res[wv] = single
    for a, b in zip(res[16], res[4]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    S.ssl_noise_destroy(n)
    S.ssl_ctx_destroy(ctx)
