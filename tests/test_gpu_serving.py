"""Serving on the GPU: continuous batching over mixed array streams, each stream's K updated by
exponential averaging on the device.  Every served result equals the block computed alone
(ssl_localize) with the same K history -- bit for bit."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def steering_tables(streams, torch):
    out = {}
    for s in streams:
        if s.M not in out:
            out[s.M] = to_dev(synth.steering_table(s.pos, s.grid, s.freqs))
    return out


@pytest.mark.parametrize("k_lag", [0, 1])
def test_served_equals_alone(k_lag):
    """Each served block equals ssl_localize on the K version it was served with: version v is
    K0 blended with the noise frames of the stream's first v blocks, one plain in-place
    ssl_noise_update per block; with a lag of L, block n reads version max(0, n - L)."""
    import torch
    import paper_2504_03373_amd as S
    from paper_2504_03373_amd.serving import GpuExecutor, Server
    S.lib()
    streams = synth.serving_streams(n_streams=6, seed=77)
    say("streams M:", [s.M for s in streams], "k_lag", k_lag)
    H = steering_tables(streams, torch)
    ex = GpuExecutor(streams, H, alpha=0.95, k_update_every=1, hbm_budget_bytes=2 << 30, lanes=2,
                     pool=3, k_lag=k_lag)
    arrivals = synth.poisson_arrivals(len(streams), 0.25, 0.010, seed=78)
    say(f"serving {len(arrivals)} blocks")
    st = Server(ex, 2 << 30, max_batch=64).run(arrivals)
    say(f"  completed {st['completed']} p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms "
        f"mean batch {st['mean_batch']:.1f}")
    assert st["completed"] == len(arrivals)
    ex.close()

    by_stream = {}
    for r in st["requests"]:
        by_stream.setdefault(r.stream, []).append(r)
    ctx = S.ssl_ctx_create(0, 0)
    for sid, reqs in by_stream.items():
        s = streams[sid]
        reqs.sort(key=lambda r: r.seq)
        say(f"replay stream {sid} (M={s.M}) alone: {len(reqs)} blocks")
        Xn0 = to_dev(s.initial_noise_frames())
        K0 = torch.zeros((s.F, s.M, s.M), dtype=torch.complex128, device="cuda:0")
        S.ssl_corr_accum(ctx, Xn0, 1.0 / Xn0.shape[1], 0, S.SSL_FP64, K0)
        n = S.ssl_noise_create(ctx, s.F, s.M)
        S.ssl_noise_set(n, K0, S.SSL_FP64)
        versions = [n]                      # handle of K version v
        Kh = torch.zeros((s.F, s.M, s.M), dtype=torch.complex128, device="cuda:0")
        Kc = torch.zeros_like(Kh)
        pool = [s.block(q) for q in range(3)]
        for r in reqs:
            X, Xn = pool[r.seq % 3]
            assert r.k_version == max(0, r.seq - k_lag), (sid, r.seq, r.k_version)
            pk = torch.zeros(s.Ns, dtype=torch.int32, device="cuda:0")
            pv = torch.zeros(s.Ns, dtype=torch.float32, device="cuda:0")
            S.ssl_localize(ctx, to_dev(X), versions[r.k_version], H[s.M], S.SSL_FP32,
                           s.grid.n_az, s.grid.n_el, s.Ns, 2, pk, pv)
            assert np.array_equal(to_host(pk), r.peaks), (sid, r.seq)
            assert np.array_equal(to_host(pv), r.peak_val), (sid, r.seq)
            # next version: a fresh handle holding the latest K, updated in place
            S.ssl_noise_get(versions[-1], Kc)
            nv = S.ssl_noise_create(ctx, s.F, s.M)
            S.ssl_noise_set(nv, Kc, S.SSL_FP64)
            S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / s.T, 0, S.SSL_FP64, Kh)
            S.ssl_noise_update(nv, Kh, S.SSL_FP64, 0.95)
            versions.append(nv)
            if len(versions) > 3:               # keep the versions a later block can read
                S.ssl_noise_destroy(versions[-4])
                versions[-4] = None
        for h in versions:
            if h is not None:
                S.ssl_noise_destroy(h)
    S.ssl_ctx_destroy(ctx)
