"""SEVD-MUSIC mode -- no noise handle, E_n from the correlation matrix itself (the
standard-eigenvalue baseline of Sec. II) -- through the C ABI, against the FP64 oracle run with
K = I (the reduction pinned on the CPU against LAPACK eigh).  MI355X only."""
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import crandn
from gpu_util import U32, peak_ambiguity, projector, to_dev, to_host

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


def eye(F, M):
    return np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()


@pytest.mark.parametrize("M,Ns", [(8, 1), (16, 2), (60, 2)])
def test_sevd_gsvd_parity(S, ctx, M, Ns):
    import torch
    say(f"ssl_gsvd SEVD (K = NULL) M={M} Ns={Ns} F=19")
    F = 19
    rng = np.random.default_rng(900 + M)
    X = crandn(rng, F, 50, M).astype(np.complex64)
    R = oracle.corr(X).astype(np.complex64)
    Rd = to_dev(R)
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    sig = torch.zeros((F, M), dtype=torch.float32, device="cuda:0")
    st = torch.full((F,), -7, dtype=torch.int32, device="cuda:0")
    S.ssl_gsvd(ctx, Rd, None, Ns, En, sig, st)
    g_En, g_sig, g_st = to_host(En), to_host(sig), to_host(st)
    assert np.array_equal(to_host(Rd), R), "the caller's R must not be modified"
    En_ref, sig_ref, st_ref, _ = oracle.gsvd(eye(F, M), R.astype(np.complex128), Ns)
    assert np.all(g_st == 0) and np.all(st_ref == 0)
    worst = 0.0
    for f in range(F):
        nA = np.linalg.norm(R[f].astype(np.complex128))
        assert np.max(np.abs(g_sig[f] - sig_ref[f])) <= 8 * M * U32 * nA
        # R is Hermitian: its singular values are the moduli of its eigenvalues (rounded to
        # complex64, the rank-50 R of 60 channels is no longer exactly semi-definite)
        ev = np.sort(np.abs(np.linalg.eigvalsh(R[f].astype(np.complex128))))[::-1]
        assert np.max(np.abs(sig_ref[f] - ev)) <= 1e-12 * nA
        gap = sig_ref[f, Ns - 1] - sig_ref[f, Ns]
        err = np.linalg.norm(projector(g_En[f].T.astype(np.complex128)) - projector(En_ref[f].T), 2)
        assert err <= 16 * M * U32 * nA / gap, (f, err, gap)
        worst = max(worst, err * gap / nA)
    say(f"  projector error * gap / |R|: max {worst:.3g} ({worst / U32:.1f} u)")


def _localize(S, fn, ctx, w, Xd, Hd):
    import torch
    pk = torch.full((w.Ns,), -7, dtype=torch.int32, device="cuda:0")
    pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
    Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
    st = torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0")
    fn(ctx, Xd, None, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, pk, pv, Pbar, st)
    return dict(peaks=to_host(pk), peak_val=to_host(pv), Pbar=to_host(Pbar), status=to_host(st))


@pytest.mark.parametrize("name", ["small", "paper"])
def test_sevd_localize_matches_oracle(S, ctx, name):
    w = synth.workload_small(n_blocks=3) if name == "small" else synth.workload_paper(n_blocks=3)
    H = w.steering_table()
    Hd = to_dev(H)
    for b in range(3):
        X, dirs, _ = w.block(b)
        say(f"ssl_localize SEVD {name} M={w.M} block {b}")
        g = _localize(S, S.ssl_localize, ctx, w, to_dev(X), Hd)
        r = oracle.localize(X, eye(w.F, w.M), H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16)
        assert np.all(g["status"] == 0) and np.all(r["status"] == 0)
        rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
        say(f"  rel {rel:.2e} peaks gpu {g['peaks']} ref {r['peaks']} planted {dirs} near-ties {amb}")
        assert rel <= 1e-4
        assert not amb
        assert np.array_equal(g["peaks"], r["peaks"])


def test_sevd_batch_and_noalloc_bit_identical(S, ctx):
    """A batch mixing SEVD blocks (no handle) and GSVD blocks equals each block alone, bit for bit;
    so does the allocation-free entry point in SEVD mode."""
    import torch
    wp = synth.workload_paper(n_blocks=4)
    ws = synth.workload_small(n_blocks=4)
    handles = {}
    for w in (wp, ws):
        Xn = w.noise_frames()
        Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
        S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
        n = S.ssl_noise_create(ctx, w.F, w.M)
        S.ssl_noise_set(n, Kd, S.SSL_FP64)
        handles[w.M] = (n, to_dev(w.steering_table()))
    plan = [(wp, 0, True), (wp, 1, False), (ws, 0, True), (ws, 1, False), (wp, 2, True)]
    say(f"ssl_localize_batch mixing SEVD and GSVD blocks: {[(w.M, b, sevd) for w, b, sevd in plan]}")
    blocks, outs, descs = [], [], []
    for w, b, sevd in plan:
        X, _, _ = w.block(b)
        Xd = to_dev(X)
        n, Hd = handles[w.M]
        o = dict(pk=torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
                 pv=torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
                 Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
                 st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))
        blocks.append((w, Xd, None if sevd else n, Hd))
        outs.append(o)
        descs.append(S.block_desc(Xd, None if sevd else n, Hd, w.grid.n_az, w.grid.n_el, w.Ns,
                                  o["pk"], o["pv"], o["Pbar"], o["st"]))
    S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
    got = [{k: to_host(v) for k, v in o.items()} for o in outs]
    for i, (w, Xd, n, Hd) in enumerate(blocks):
        o = dict(pk=torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
                 pv=torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
                 Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
                 st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))
        S.ssl_localize(ctx, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, o["pk"],
                       o["pv"], o["Pbar"], o["st"])
        ref = {k: to_host(v) for k, v in o.items()}
        for k in ("pk", "pv", "Pbar", "st"):
            assert np.array_equal(got[i][k], ref[k]), (i, k)
        if n is None:
            o2 = dict(pk=torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
                      pv=torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
                      Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
                      st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))
            S.ssl_localize_noalloc(ctx, Xd, None, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2,
                                   o2["pk"], o2["pv"], o2["Pbar"], o2["st"])
            for k in ("pk", "pv", "Pbar", "st"):
                assert np.array_equal(to_host(o2[k]), ref[k]), (i, k, "noalloc")
    for n, _ in handles.values():
        S.ssl_noise_destroy(n)
