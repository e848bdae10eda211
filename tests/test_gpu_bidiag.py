"""The paper's own SVD (Householder bidiagonalisation, phase transform, implicit-shift QR, sort,
back-transformation) as the second backend (ssl_ctx_set_svd(SSL_SVD_BIDIAG_QR)), against the FP64
oracle and against the Jacobi backend on the GPU.  MI355X only."""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import U32, peak_ambiguity, projector, to_dev, to_host
from test_gpu_parity import gsvd_case, set_noise

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
    S.ssl_ctx_set_svd(c, S.SSL_SVD_BIDIAG_QR)
    assert S.ssl_ctx_get_svd(c) == S.SSL_SVD_BIDIAG_QR
    yield c
    S.ssl_ctx_destroy(c)


def run(S, ctx, R64, K, Ns):
    import torch
    F, M, _ = R64.shape
    n, _ = set_noise(S, ctx, K)
    Rd = to_dev(R64.astype(np.complex64))
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    sig = torch.zeros((F, M), dtype=torch.float32, device="cuda:0")
    st = torch.full((F,), -7, dtype=torch.int32, device="cuda:0")
    conv = torch.zeros((F, 3), dtype=torch.int32, device="cuda:0")
    S.ssl_gsvd(ctx, Rd, n, Ns, En, sig, st, conv)
    out = dict(En=to_host(En), sigma=to_host(sig), status=to_host(st), conv=to_host(conv))
    assert np.array_equal(to_host(Rd), R64.astype(np.complex64), equal_nan=True)   # R intact
    S.ssl_noise_destroy(n)
    return out


@pytest.mark.parametrize("M,Ns", [(2, 1), (3, 1), (8, 1), (13, 3), (16, 2), (31, 2), (60, 2), (64, 5)])
def test_bidiag_qr_parity(S, ctx, M, Ns):
    say(f"ssl_gsvd bidiagonal QR M={M} Ns={Ns} F=19")
    F = 19
    R, K = gsvd_case(M, F, Ns, seed=300 + M)
    g = run(S, ctx, R, K, Ns)
    En_ref, sig_ref, st_ref, _ = oracle.gsvd(K, R, Ns)
    assert np.all(st_ref == 0) and np.all(g["status"] == 0), g["status"]
    worst = 0.0
    for f in range(F):
        A = np.linalg.solve(K[f], R[f])
        nA = np.linalg.norm(A)
        assert np.max(np.abs(g["sigma"][f] - sig_ref[f])) <= 8 * M * U32 * nA
        gap = sig_ref[f, Ns - 1] - sig_ref[f, Ns]
        err = np.linalg.norm(projector(g["En"][f].T.astype(np.complex128)) - projector(En_ref[f].T), 2)
        assert err <= 16 * M * U32 * nA / gap, (f, err, gap)
        E = g["En"][f].T.astype(np.complex128)
        assert np.linalg.norm(E.conj().T @ E - np.eye(M - Ns), 2) <= 8 * M * U32
        worst = max(worst, err * gap / nA)
    say(f"  QR steps per bin: mean {g['conv'][:, 0].mean():.1f} max {g['conv'][:, 0].max()}, "
        f"zero-diagonal chases mean {g['conv'][:, 1].mean():.1f}; projector error * gap / |A| "
        f"max {worst / U32:.1f} u")


def test_bidiag_qr_status_paths(S, ctx):
    say("bidiagonal QR status paths M=8 F=6")
    F, M, Ns = 6, 8, 2
    R, K = gsvd_case(M, F, Ns, seed=31)
    w, V = np.linalg.eigh(K[1])
    w[0] = -1.0
    K[1] = (V * w) @ V.conj().T                 # NOT_PD
    R[3, 2, 5] = np.nan                          # NONFINITE
    g = run(S, ctx, R, K, Ns)
    assert g["status"].tolist() == [0, 1, 0, 3, 0, 0]
    assert np.all(g["En"][1] == 0) and np.all(g["En"][3] == 0)


def test_bidiag_and_jacobi_agree(S, ctx):
    """The two GPU backends on the same whitened products: projectors within twice the bound."""
    import torch
    say("bidiagonal QR vs Jacobi, 60-mic workload, 257 bins")
    w = synth.workload_paper(n_blocks=2)
    X, _, _ = w.block(0)
    K = oracle.noise_corr(w.noise_frames())
    R = oracle.corr(X).astype(np.complex64).astype(np.complex128)
    g_gk = run(S, ctx, R, K, w.Ns)
    cj = S.ssl_ctx_create(0, 0)
    g_j = run(S, cj, R, K, w.Ns)
    S.ssl_ctx_destroy(cj)
    En_ref, sig_ref, _, _ = oracle.gsvd(K, R, w.Ns, nthreads=16)
    worst = 0.0
    for f in range(w.F):
        nA = np.linalg.norm(np.linalg.solve(K[f], R[f]))
        gap = sig_ref[f, w.Ns - 1] - sig_ref[f, w.Ns]
        d = np.linalg.norm(projector(g_gk["En"][f].T.astype(np.complex128))
                           - projector(g_j["En"][f].T.astype(np.complex128)), 2)
        assert d <= 32 * w.M * U32 * nA / gap, (f, d, gap)
        worst = max(worst, d * gap / nA)
    say(f"  max |P_gk - P_jacobi| * gap / |A| = {worst / U32:.1f} u; QR steps mean "
        f"{g_gk['conv'][:, 0].mean():.1f}")


def test_bidiag_localize_and_batch(S, ctx):
    """Whole path with the bidiagonal backend on the 60-mic workload against the oracle, and the
    batched call bit-identical to one call per block."""
    import torch
    w = synth.workload_paper(n_blocks=3)
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    K = oracle.noise_corr(Xn)
    H = w.steering_table()
    Hd = to_dev(H)
    outs, descs, Xds = [], [], []
    for b in range(3):
        X, dirs, _ = w.block(b)
        Xd = to_dev(X)
        Xds.append(Xd)
        o = dict(pk=torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
                 pv=torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
                 Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
                 st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))
        say(f"ssl_localize bidiagonal QR 60ch block {b}")
        S.ssl_localize(ctx, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, o["pk"],
                       o["pv"], o["Pbar"], o["st"])
        g = {k: to_host(v) for k, v in o.items()}
        r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16)
        rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
        say(f"  rel {rel:.2e} peaks {g['pk']} ref {r['peaks']} planted {dirs} near-ties {amb}")
        assert np.all(g["st"] == 0)
        assert rel <= 1e-4 and not amb and np.array_equal(g["pk"], r["peaks"])
        outs.append(g)
        descs.append(None)
    bo = [dict(pk=torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
               pv=torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
               Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
               st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0")) for _ in range(3)]
    ds = [S.block_desc(Xds[b], n, Hd, w.grid.n_az, w.grid.n_el, w.Ns, bo[b]["pk"], bo[b]["pv"],
                       bo[b]["Pbar"], bo[b]["st"]) for b in range(3)]
    S.ssl_localize_batch(ctx, ds, S.SSL_FP32, 2)
    for b in range(3):
        for k in ("pk", "pv", "Pbar", "st"):
            assert np.array_equal(to_host(bo[b][k]), outs[b][k]), (b, k)
    S.ssl_noise_destroy(n)
