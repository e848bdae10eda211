"""ssl_localize_noalloc (the entry point that allocates nothing) against ssl_localize, through the
C ABI, on two calls in a row -- the 60-mic paper-scale block, then a smaller 8-mic block that
reuses the same fixed scratch -- bit for bit, plus the size limit.  MI355X only."""
import sys

import numpy as np
import pytest

import oracle
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


def _noise(S, ctx, w):
    import torch
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    return n, Xn


def _outputs(w):
    import torch
    return dict(peaks=torch.full((w.Ns,), -7, dtype=torch.int32, device="cuda:0"),
                peak_val=torch.full((w.Ns,), -7.0, dtype=torch.float32, device="cuda:0"),
                Pbar=torch.full((w.D,), -7.0, dtype=torch.float32, device="cuda:0"),
                status=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))


def _run(S, fn, ctx, w, Xd, n, Hd):
    o = _outputs(w)
    fn(ctx, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, o["peaks"], o["peak_val"],
       o["Pbar"], o["status"])
    return o


def test_noalloc_matches_localize_two_calls(S):
    import torch
    ctx_na = S.ssl_ctx_create(0, 0)        # used only by the allocation-free calls
    ctx = S.ssl_ctx_create(0, 0)
    try:
        cases = [("60ch paper-scale block", synth.workload_paper(n_blocks=4)),
                 ("8ch small block", synth.workload_small(n_blocks=2))]
        for name, w in cases:
            say(f"ssl_localize_noalloc {name}: M={w.M} F={w.F} D={w.D} Ns={w.Ns}")
            n, Xn = _noise(S, ctx, w)
            X, dirs, _ = w.block(0)
            Xd, Hd = to_dev(X), to_dev(w.steering_table())
            need = S.ssl_localize_noalloc_bytes(w.F, w.M, w.Ns, w.D)
            assert 0 < need <= S.SSL_NOALLOC_SCRATCH_BYTES
            o_na = _outputs(w)
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            S.ssl_localize_noalloc(ctx_na, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns,
                                   2, o_na["peaks"], o_na["peak_val"], o_na["Pbar"],
                                   o_na["status"])
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == before
            assert S.ssl_ctx_workspace_bytes(ctx_na) == 0
            o_ws = _run(S, S.ssl_localize, ctx, w, Xd, n, Hd)
            torch.cuda.synchronize()
            a = {k: to_host(v) for k, v in o_na.items()}
            b = {k: to_host(v) for k, v in o_ws.items()}
            say(f"  peaks noalloc {a['peaks']} localize {b['peaks']} (planted {dirs})")
            assert np.all(a["status"] == 0)
            for k in ("peaks", "status"):
                assert np.array_equal(a[k], b[k]), k
            for k in ("peak_val", "Pbar"):
                assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k
            if w.M == 8:                     # and against the oracle (peaks, Pbar within 1e-4)
                r = oracle.localize(X, oracle.noise_corr(Xn), w.steering_table(), w.grid.n_az,
                                    w.grid.n_el, w.Ns, nthreads=8)
                assert np.array_equal(a["peaks"], r["peaks"])
                rel = np.max(np.abs(a["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"])
                assert rel <= 1e-4, rel
            S.ssl_noise_destroy(n)
    finally:
        S.ssl_ctx_destroy(ctx)
        S.ssl_ctx_destroy(ctx_na)


def test_noalloc_rejects_blocks_beyond_the_scratch(S):
    import torch
    say("ssl_localize_noalloc size limit: F=1100 M=60 Ns=2 D=1368")
    ctx = S.ssl_ctx_create(0, 0)
    try:
        F, M, T = 1100, 60, 50
        assert S.ssl_localize_noalloc_bytes(F, M, 2, 1368) > S.SSL_NOALLOC_SCRATCH_BYTES
        n = S.ssl_noise_create(ctx, F, M)
        eye = torch.eye(M, dtype=torch.complex128, device="cuda:0").expand(F, M, M).contiguous()
        S.ssl_noise_set(n, eye, S.SSL_FP64)
        X = torch.zeros((F, T, M), dtype=torch.complex64, device="cuda:0")
        pk = torch.full((2,), -7, dtype=torch.int32, device="cuda:0")
        pv = torch.zeros(2, dtype=torch.float32, device="cuda:0")
        with pytest.raises(S.SSLError) as e:
            # H is never read: the size check fails before anything is enqueued
            S.ssl_localize_noalloc(ctx, X, n, X, S.SSL_FP32, 72, 19, 2, 2, pk, pv)
        assert e.value.code == S.SSL_ERR_ARG
        torch.cuda.synchronize()
        assert np.all(to_host(pk) == -7)
        S.ssl_noise_destroy(n)
    finally:
        S.ssl_ctx_destroy(ctx)
