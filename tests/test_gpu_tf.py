"""Transfer-function tables on the device: ssl_tf_load (FP32 table bit-exact; 16-bit layouts equal
to round-to-nearest-even conversion), ssl_steering_convert, a truncated file, and a localization
from a loaded table identical to one from the table in memory.  MI355X only."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import to_dev, to_host

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


def rne16(S, H, prec):
    import torch
    dt = torch.bfloat16 if prec == S.SSL_BF16 else torch.float16
    F, D, M = H.shape
    return torch.view_as_real(to_dev(H)).reshape(F, D, 2 * M).to(dt).contiguous()


@pytest.mark.parametrize("M", [8, 60])
def test_tf_load_all_precisions(S, ctx, tmp_path, M):
    import torch
    w = synth.workload_small(n_blocks=1) if M == 8 else synth.workload_paper(n_blocks=1)
    H = w.steering_table()
    F, D, _ = H.shape
    info = S.TfInfo(M=M, F=F, n_az=w.grid.n_az, n_el=w.grid.n_el, nfft=512, fs=16000.0,
                    az0_deg=0.0, az_step_deg=5.0, el0_deg=0.0, el_step_deg=5.0)
    p = str(tmp_path / f"h{M}.ssltf")
    S.ssl_tf_write(p, info, w.pos, H)
    say(f"ssl_tf_load M={M} F={F} D={D} ({H.nbytes / 1e6:.1f} MB)")
    H32 = torch.zeros((F, D, M), dtype=torch.complex64, device="cuda:0")
    S.ssl_tf_load(ctx, p, S.SSL_FP32, H32)
    assert np.array_equal(to_host(H32), H)
    for prec, dt in ((S.SSL_BF16, torch.bfloat16), (S.SSL_FP16, torch.float16)):
        H16 = torch.zeros((F, D, 2 * M), dtype=dt, device="cuda:0")
        S.ssl_tf_load(ctx, p, prec, H16)
        ref = rne16(S, H, prec)
        assert torch.equal(H16.view(torch.int16), ref.view(torch.int16))
        Hc = torch.zeros_like(H16)
        S.ssl_steering_convert(ctx, H32, prec, Hc)
        assert torch.equal(Hc.view(torch.int16), ref.view(torch.int16))


def test_tf_load_truncated(S, ctx, tmp_path):
    import torch
    w = synth.workload_small(n_blocks=1)
    H = w.steering_table()
    info = S.TfInfo(M=8, F=257, n_az=72, n_el=1, nfft=512, fs=16000.0, az0_deg=0.0,
                    az_step_deg=5.0, el0_deg=0.0, el_step_deg=5.0)
    p = tmp_path / "t.ssltf"
    S.ssl_tf_write(str(p), info, w.pos, H)
    raw = p.read_bytes()
    p.write_bytes(raw[:len(raw) - 1000])
    say("ssl_tf_load truncated file")
    Hd = torch.zeros(H.shape, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_tf_load(ctx, str(p), S.SSL_FP32, Hd)
    assert e.value.code == S.SSL_ERR_ARG


def test_localize_from_loaded_table(S, ctx, tmp_path):
    import torch
    w = synth.workload_paper(n_blocks=2)
    H = w.steering_table()
    info = S.TfInfo(M=60, F=257, n_az=72, n_el=19, nfft=512, fs=16000.0, az0_deg=0.0,
                    az_step_deg=5.0, el0_deg=0.0, el_step_deg=5.0)
    p = str(tmp_path / "ring60.ssltf")
    S.ssl_tf_write(p, info, w.pos, H)
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    X, dirs, _ = w.block(0)
    Xd = to_dev(X)
    for prec, dt in ((S.SSL_FP32, torch.complex64), (S.SSL_BF16, torch.bfloat16)):
        say(f"localize from a loaded table, prec {prec}")
        shape = (w.F, w.D, w.M) if prec == S.SSL_FP32 else (w.F, w.D, 2 * w.M)
        Hl = torch.zeros(shape, dtype=dt, device="cuda:0")
        S.ssl_tf_load(ctx, p, prec, Hl)
        Hm = to_dev(H) if prec == S.SSL_FP32 else rne16(S, H, prec)
        outs = []
        for Ht in (Hl, Hm):
            pk = torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0")
            pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
            Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
            S.ssl_localize(ctx, Xd, n, Ht, prec, w.grid.n_az, w.grid.n_el, w.Ns, 2, pk, pv, Pbar)
            outs.append((to_host(pk), to_host(Pbar)))
        assert np.array_equal(outs[0][0], outs[1][0])
        assert np.array_equal(outs[0][1].view(np.uint32), outs[1][1].view(np.uint32))
        say(f"  peaks {outs[0][0]} planted {dirs}")
    S.ssl_noise_destroy(n)
