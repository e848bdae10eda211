"""The Jacobi solve stopped at the noise subspace (ssl_ctx_set_stop): E_n is an orthonormal basis
of the span of the M - Ns smallest left singular vectors, compared as a projector with the
oracle's and with the full solve's, within the same bound; localizations with p = 2 equal the full
solve's within the P-bar bar; the fallback to the full solve when the dominance check fails.
MI355X only."""
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import crandn, random_pd
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


def gsvd_mode(S, ctx, R, K, Ns, mode):
    """ssl_gsvd without sigma (so the subspace stop may apply) under the given stop mode."""
    import torch
    F, M, _ = R.shape
    n = S.ssl_noise_create(ctx, F, M)
    S.ssl_noise_set(n, to_dev(K.astype(np.complex128)), S.SSL_FP64)
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    st = torch.full((F,), -7, dtype=torch.int32, device="cuda:0")
    conv = torch.zeros((F, 3), dtype=torch.int32, device="cuda:0")
    S.ssl_ctx_set_stop(ctx, mode)
    try:
        S.ssl_gsvd(ctx, to_dev(R.astype(np.complex64)), n, Ns, En, None, st, conv)
        out = to_host(En), to_host(st), to_host(conv)
    finally:
        S.ssl_ctx_set_stop(ctx, S.SSL_STOP_LOCALIZE)
        S.ssl_noise_destroy(n)
    return out


@pytest.mark.parametrize("M,Ns", [(8, 1), (16, 2), (33, 3), (60, 2), (64, 8)])
def test_subspace_stop_projector(S, ctx, M, Ns):
    """Random R (rank min(M, 50)) and coloured K: the subspace-stopped E_n is orthonormal and its
    projector meets the full solve's bound against the oracle."""
    say(f"ssl_gsvd stop at the subspace M={M} Ns={Ns} F=19")
    F = 19
    rng = np.random.default_rng(1600 + M)
    X = crandn(rng, F, 50, M).astype(np.complex64)
    # a dominant subspace of dimension Ns, as with Ns sources
    Hs = crandn(rng, F, M, Ns)
    X = (X + 6.0 * np.einsum("fmk,ftk->ftm", Hs, crandn(rng, F, 50, Ns))).astype(np.complex64)
    R = oracle.corr(X).astype(np.complex64).astype(np.complex128)
    K = np.stack([random_pd(rng, M, 100.0) for _ in range(F)])
    E_sub, st_sub, cv_sub = gsvd_mode(S, ctx, R, K, Ns, S.SSL_STOP_ALSO_GSVD)
    E_full, st_full, cv_full = gsvd_mode(S, ctx, R, K, Ns, S.SSL_STOP_NEVER)
    En_ref, sig_ref, st_ref, _ = oracle.gsvd(K, R, Ns)
    assert np.all(st_sub == 0) and np.all(st_full == 0) and np.all(st_ref == 0)
    worst = 0.0
    for f in range(F):
        A = np.linalg.solve(K[f], R[f])
        nA = np.linalg.norm(A)
        gap = sig_ref[f, Ns - 1] - sig_ref[f, Ns]
        E = E_sub[f].T.astype(np.complex128)
        assert np.linalg.norm(E.conj().T @ E - np.eye(M - Ns), 2) <= 8 * M * U32
        err = np.linalg.norm(projector(E) - projector(En_ref[f].T), 2)
        assert err <= 16 * M * U32 * nA / gap, (f, err, gap)
        d = np.linalg.norm(projector(E) - projector(E_full[f].T.astype(np.complex128)), 2)
        assert d <= 32 * M * U32 * nA / gap, (f, d)
        worst = max(worst, err * gap / nA)
    say(f"  projector error * gap / |A| max {worst / U32:.1f} u; sweeps subspace "
        f"{cv_sub[:, 0].mean():.2f} vs full {cv_full[:, 0].mean():.2f}")
    assert cv_sub[:, 0].mean() <= cv_full[:, 0].mean()


def test_subspace_stop_fallback(S, ctx):
    """A spectrum whose noise block is too heavy for the dominance check (sigma = 10, 9 then
    fourteen 5s: 81 < 14 * 25): the solve falls back to full sweeps and still meets the bound."""
    import torch
    M, Ns, F = 16, 2, 6
    rng = np.random.default_rng(1610)
    R = np.zeros((F, M, M), np.complex128)
    lam = np.r_[10.0, 9.0, np.full(M - 2, 5.0) * (1 + 0.05 * rng.random(M - 2))]
    for f in range(F):
        Q, _ = np.linalg.qr(crandn(rng, M, M))
        R[f] = (Q * lam) @ Q.conj().T
    R = R.astype(np.complex64).astype(np.complex128)
    K = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    E_sub, st_sub, cv_sub = gsvd_mode(S, ctx, R, K, Ns, S.SSL_STOP_ALSO_GSVD)
    En_ref, sig_ref, st_ref, _ = oracle.gsvd(K, R, Ns)
    assert np.all(st_sub == 0)
    for f in range(F):
        nA = np.linalg.norm(R[f])
        gap = sig_ref[f, Ns - 1] - sig_ref[f, Ns]
        E = E_sub[f].T.astype(np.complex128)
        err = np.linalg.norm(projector(E) - projector(En_ref[f].T), 2)
        assert err <= 16 * M * U32 * nA / gap, (f, err)
        # the fallback ends in the full solve: its noise vectors are singular vectors
        Rf = R[f]
        resid = np.linalg.norm(Rf @ E - E @ np.diag(np.diag(E.conj().T @ Rf @ E)), 2)
        assert resid <= 64 * M * U32 * nA, (f, resid)


@pytest.mark.parametrize("name", ["small", "paper"])
def test_localize_stop_modes_agree(S, ctx, name):
    """ssl_localize (p = 2) with the subspace stop (default) and with the full solve: P-bar within
    1e-4 of each other and of the oracle, the same peaks."""
    import torch
    w = synth.workload_small(n_blocks=4) if name == "small" else synth.workload_paper(n_blocks=4)
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    K = oracle.noise_corr(Xn)
    H = w.steering_table()
    Hd = to_dev(H)
    assert S.ssl_ctx_get_stop(ctx) == S.SSL_STOP_LOCALIZE
    for b in range(4):
        X, dirs, _ = w.block(b)
        Xd = to_dev(X)
        out = {}
        for mode in (S.SSL_STOP_LOCALIZE, S.SSL_STOP_NEVER):
            S.ssl_ctx_set_stop(ctx, mode)
            pk = torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0")
            pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
            Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
            st = torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0")
            S.ssl_localize(ctx, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, pk, pv,
                           Pbar, st)
            out[mode] = (to_host(pk), to_host(Pbar), to_host(st))
        S.ssl_ctx_set_stop(ctx, S.SSL_STOP_LOCALIZE)
        r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16)
        (pk_s, P_s, st_s), (pk_f, P_f, st_f) = out[S.SSL_STOP_LOCALIZE], out[S.SSL_STOP_NEVER]
        assert np.all(st_s == 0) and np.all(st_f == 0)
        rel_sf = float(np.max(np.abs(P_s.astype(np.float64) - P_f) / P_f))
        rel = float(np.max(np.abs(P_s.astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
        say(f"  {name} block {b}: subspace vs full {rel_sf:.2e}, vs oracle {rel:.2e}, peaks "
            f"{pk_s} {pk_f} ref {r['peaks']}")
        assert rel_sf <= 1e-4 and rel <= 1e-4
        assert not amb
        assert np.array_equal(pk_s, r["peaks"]) and np.array_equal(pk_f, r["peaks"])
    S.ssl_noise_destroy(n)


def test_stop_mode_errors(S, ctx):
    with pytest.raises(S.SSLError) as e:
        S.ssl_ctx_set_stop(ctx, 4)
    assert e.value.code == S.SSL_ERR_ARG
    assert S.ssl_ctx_get_stop(ctx) == S.SSL_STOP_LOCALIZE


def test_batch_mode_only(S, ctx):
    """SSL_STOP_BATCH: the batch stops at the subspace, single blocks run the full solve; the
    batch equals single blocks run under SSL_STOP_LOCALIZE bit for bit and the full solve's
    single blocks within the P-bar bar."""
    import torch
    w = synth.workload_paper(n_blocks=3)
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    Hd = to_dev(w.steering_table())
    Xs = [to_dev(w.block(b)[0]) for b in range(3)]

    def outs():
        return dict(pk=torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
                    pv=torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
                    Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
                    st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))

    def single(Xd):
        o = outs()
        S.ssl_localize(ctx, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, o["pk"],
                       o["pv"], o["Pbar"], o["st"])
        return {k: to_host(v) for k, v in o.items()}

    try:
        S.ssl_ctx_set_stop(ctx, S.SSL_STOP_BATCH)
        bo = [outs() for _ in Xs]
        descs = [S.block_desc(Xd, n, Hd, w.grid.n_az, w.grid.n_el, w.Ns, o["pk"], o["pv"],
                              o["Pbar"], o["st"]) for Xd, o in zip(Xs, bo)]
        S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
        got = [{k: to_host(v) for k, v in o.items()} for o in bo]
        full = [single(Xd) for Xd in Xs]                   # one block per call: full solve
        S.ssl_ctx_set_stop(ctx, S.SSL_STOP_LOCALIZE)
        sub = [single(Xd) for Xd in Xs]
    finally:
        S.ssl_ctx_set_stop(ctx, S.SSL_STOP_LOCALIZE)
    for g, f_, s_ in zip(got, full, sub):
        for k in ("pk", "pv", "Pbar", "st"):
            assert np.array_equal(g[k], s_[k]), k
        rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - f_["Pbar"]) / f_["Pbar"]))
        assert rel <= 1e-4 and np.array_equal(g["pk"], f_["pk"])
    S.ssl_noise_destroy(n)
