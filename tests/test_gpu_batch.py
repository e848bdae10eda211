"""Batched path (ssl_localize_batch): uneven shapes in one set of launches, hipGraph replay.

* every block's Pbar / peaks / status are bit-identical to ssl_localize on that block alone,
  with graphs on (first capture and later replays, interleaved with unrelated GPU work), with
  graphs off and with per-kernel timing on, and at bf16 / fp16 (16-bit tables);
* uneven blocks match the FP64 oracle (Pbar within 1e-4; no near-tie within the measured error
  and the returned peaks identical).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import peak_ambiguity, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(60, 257, 2), (8, 257, 1), (16, 513, 3), (32, 257, 2), (60, 257, 3), (8, 513, 1),
          (16, 257, 1), (32, 513, 2)]


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
def env(S):
    """Per (M, F): workload, noise handle, host and device steering tables; blocks on device."""
    import torch
    ctx = S.ssl_ctx_create(0, 0)
    streams = {}
    blocks = []
    for i, (M, F, Ns) in enumerate(SHAPES):
        key = (M, F)
        if key not in streams:
            w = synth.workload_paper(n_blocks=8, seed=2000 + M * 10 + F, M=M, F=F, Ns=Ns)
            Xn = w.noise_frames()
            Kd = torch.zeros((F, M, M), dtype=torch.complex128, device="cuda:0")
            S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
            n = S.ssl_noise_create(ctx, F, M)
            S.ssl_noise_set(n, Kd, S.SSL_FP64)
            H = w.steering_table()
            streams[key] = dict(w=w, noise=n, K=oracle.noise_corr(Xn), H=H, Hd=to_dev(H))
        st = streams[key]
        w = synth.workload_paper(n_blocks=8, seed=2000 + M * 10 + F, M=M, F=F, Ns=Ns)
        X, dirs, _ = w.block(i % 8)
        blocks.append(dict(M=M, F=F, Ns=Ns, X=X, Xd=to_dev(X), s=st, D=w.D))
    yield S, ctx, blocks
    for st in streams.values():
        S.ssl_noise_destroy(st["noise"])
    S.ssl_ctx_destroy(ctx)


def outputs(blocks):
    import torch
    outs = []
    for b in blocks:
        outs.append(dict(pk=torch.zeros(b["Ns"], dtype=torch.int32, device="cuda:0"),
                         pv=torch.zeros(b["Ns"], dtype=torch.float32, device="cuda:0"),
                         Pbar=torch.zeros(b["D"], dtype=torch.float32, device="cuda:0"),
                         st=torch.full((b["F"],), -7, dtype=torch.int32, device="cuda:0")))
    return outs


def run_batch(S, ctx, blocks, outs):
    descs = [S.block_desc(b["Xd"], b["s"]["noise"], b["s"]["Hd"], 72, 19, b["Ns"], o["pk"], o["pv"],
                          o["Pbar"], o["st"]) for b, o in zip(blocks, outs)]
    S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
    return [{k: to_host(v) for k, v in o.items()} for o in outs]


def run_single(S, ctx, blocks):
    outs = outputs(blocks)
    for b, o in zip(blocks, outs):
        S.ssl_localize(ctx, b["Xd"], b["s"]["noise"], b["s"]["Hd"], S.SSL_FP32, 72, 19, b["Ns"], 2,
                       o["pk"], o["pv"], o["Pbar"], o["st"])
    return [{k: to_host(v) for k, v in o.items()} for o in outs]


def same(a, b):
    return all(np.array_equal(x[k], y[k]) for x, y in zip(a, b) for k in ("pk", "pv", "Pbar", "st"))


def test_batch_bit_identical_to_single(env):
    import torch
    S, ctx, blocks = env
    say(f"ssl_localize x{len(blocks)} (single-block reference), shapes {SHAPES}")
    ref = run_single(S, ctx, blocks)
    assert all(np.all(r["st"] == 0) for r in ref)
    S.ssl_ctx_use_graphs(ctx, True)
    for rep in range(4):
        say(f"ssl_localize_batch graphs on, call {rep}")
        got = run_batch(S, ctx, blocks, outputs(blocks))
        assert same(got, ref), rep
        # unrelated eager GPU work and a synchronisation between replays
        a = torch.randn(512, 512, device="cuda:0")
        (a @ a).sum().item()
    say("ssl_localize_batch graphs off")
    S.ssl_ctx_use_graphs(ctx, False)
    assert same(run_batch(S, ctx, blocks, outputs(blocks)), ref)
    S.ssl_ctx_use_graphs(ctx, True)
    say("ssl_localize_batch with per-kernel timing")
    S.ssl_ctx_timing(ctx, True)
    got = run_batch(S, ctx, blocks, outputs(blocks))
    S.ssl_ctx_timing(ctx, False)
    kt = S.ssl_ctx_timing_read(ctx, reset=True)
    assert same(got, ref)
    assert kt["jacobi"][0] == len({min(64, max(8, 1 << (b["M"] - 1).bit_length())) for b in blocks})


@pytest.mark.parametrize("pname", ["bf16", "fp16"])
def test_batch_bit_identical_to_single_16bit(env, pname):
    """The same uneven batch with 16-bit steering tables and correlation inputs (every block has
    Ns <= 3, so all take the signal-subspace projection on a 16-bit table): bit-identical to
    ssl_localize on each block alone at the same precision."""
    import torch
    S, ctx, blocks = env
    prec = S.SSL_BF16 if pname == "bf16" else S.SSL_FP16
    dt = torch.bfloat16 if pname == "bf16" else torch.float16
    tabs = {}
    for b in blocks:
        key = (b["M"], b["F"])
        if key not in tabs:
            Hd = b["s"]["Hd"]
            F, D, M = Hd.shape
            tabs[key] = torch.view_as_real(Hd).reshape(F, D, 2 * M).to(dt).contiguous()
    say(f"ssl_localize x{len(blocks)} at {pname} (single-block reference)")
    ref_o = outputs(blocks)
    for b, o in zip(blocks, ref_o):
        S.ssl_localize(ctx, b["Xd"], b["s"]["noise"], tabs[(b["M"], b["F"])], prec, 72, 19,
                       b["Ns"], 2, o["pk"], o["pv"], o["Pbar"], o["st"])
    ref = [{k: to_host(v) for k, v in o.items()} for o in ref_o]
    assert all(np.all(r["st"] == 0) for r in ref)
    for rep in range(2):
        say(f"ssl_localize_batch at {pname}, call {rep}")
        outs = outputs(blocks)
        descs = [S.block_desc(b["Xd"], b["s"]["noise"], tabs[(b["M"], b["F"])], 72, 19, b["Ns"],
                              o["pk"], o["pv"], o["Pbar"], o["st"]) for b, o in zip(blocks, outs)]
        S.ssl_localize_batch(ctx, descs, prec, 2)
        got = [{k: to_host(v) for k, v in o.items()} for o in outs]
        assert same(got, ref), rep


def test_batch_subset_and_reorder(env):
    """A different batch shape (subset, reversed) after a cached one: a new graph, same results."""
    S, ctx, blocks = env
    sub = blocks[::-1][:5]
    say("ssl_localize_batch reversed subset of 5")
    ref = run_single(S, ctx, sub)
    assert same(run_batch(S, ctx, sub, outputs(sub)), ref)
    assert same(run_batch(S, ctx, sub, outputs(sub)), ref)


def test_batch_shared_tables(env):
    """Blocks interleaved over two steering tables of one shape (one projection launch loops over
    each table's blocks), then the same shapes with one table: bit-identical to single calls,
    and the changed sharing pattern does not replay the first graph."""
    S, ctx, blocks = env
    b60 = [b for b in blocks if b["M"] == 60]
    Hb = b60[0]["s"]["Hd"].clone()
    mix = []
    for i, tab in enumerate("ABAABA"):
        b = dict(b60[i % len(b60)])
        b["s"] = dict(b["s"], Hd=Hb) if tab == "B" else b["s"]
        mix.append(b)
    say("ssl_localize_batch 6 blocks over two shared tables (ABAABA)")
    ref = run_single(S, ctx, mix)
    assert same(run_batch(S, ctx, mix, outputs(mix)), ref)
    assert same(run_batch(S, ctx, mix, outputs(mix)), ref)
    one = [dict(b, s=b60[0]["s"]) if b["s"]["Hd"] is Hb else b for b in mix]
    say("ssl_localize_batch same shapes, one table")
    assert same(run_batch(S, ctx, one, outputs(one)), run_single(S, ctx, one))


def test_batch_uneven_matches_oracle(env):
    S, ctx, blocks = env
    say("ssl_localize_batch uneven vs oracle")
    got = run_batch(S, ctx, blocks, outputs(blocks))
    worst = 0.0
    for b, g in zip(blocks, got):
        r = oracle.localize(b["X"], b["s"]["K"], b["s"]["H"], 72, 19, b["Ns"], nthreads=16)
        assert np.array_equal(g["st"], r["status"])
        rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        worst = max(worst, rel)
        # near-tie radius: this block's own measured error (see test_gpu_parity.check_block)
        amb = peak_ambiguity(r["Pbar"], 19, 72, b["Ns"], max(rel, 1e-7))
        say(f"  M={b['M']} F={b['F']} Ns={b['Ns']}: rel {rel:.2e} peaks {g['pk']} ref {r['peaks']} "
            f"near-ties {amb}")
        assert rel <= 1e-4
        assert not amb
        assert np.array_equal(g["pk"], r["peaks"])


def test_batch_argument_errors(env):
    S, ctx, blocks = env
    outs = outputs(blocks[:1])
    b = blocks[0]
    d = S.block_desc(b["Xd"], b["s"]["noise"], b["s"]["Hd"], 72, 19, b["Ns"], outs[0]["pk"],
                     outs[0]["pv"])
    d.M = 65
    with pytest.raises(S.SSLError) as e:
        S.ssl_localize_batch(ctx, [d], S.SSL_FP32, 2)
    assert e.value.code == S.SSL_ERR_ARG and "block 0" in str(e.value)
    with pytest.raises(S.SSLError):
        S.ssl_localize_batch(ctx, [], S.SSL_FP32, 2)


def test_batch_mixed_frame_counts(env):
    """Blocks of one size class with different T (one frame chunk, two chunks, a strided view) in
    one batch: each bin's first frame chunk is loaded under the previous bin's products, whatever
    the previous block's T; results bit-identical to single calls."""
    import torch
    S, ctx, blocks = env
    b60 = [b for b in blocks if b["M"] == 60][:2]
    X0, X1 = b60[0]["Xd"], b60[1]["Xd"]
    variants = [X0[:, :20].contiguous(),                 # T = 20
                torch.cat([X0, X1], dim=1).contiguous(),  # T = 100: two 64-frame chunks
                X1,                                       # T = 50
                torch.cat([X1, X0], dim=1)[:, ::2],       # T = 50, frame stride 2M
                X0[:, :1].contiguous()]                   # T = 1
    mixed = [dict(b60[i % 2], Xd=v) for i, v in enumerate(variants)]
    say("ssl_localize_batch, one class, T = 20 / 100 / 50 / 50 (strided) / 1")
    ref = run_single(S, ctx, mixed)
    assert same(run_batch(S, ctx, mixed, outputs(mixed)), ref)
    assert same(run_batch(S, ctx, mixed[::-1], outputs(mixed[::-1])), ref[::-1])
