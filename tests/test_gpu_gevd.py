"""GEVD-MUSIC mode (the generalized-eigenvalue alternative of Sec. II: noise vectors e with
R e = lambda K e for the M - Ns smallest lambda) through the C ABI, against the FP64 oracle's GEVD
(pinned on the CPU against scipy's generalized eigensolver).  MI355X only."""
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
    S.ssl_ctx_set_subspace(c, S.SSL_SUBSPACE_GEVD)
    yield c
    S.ssl_ctx_destroy(c)


def gevd_noise(S, ctx, K, enable=True):
    import torch
    F, M, _ = K.shape
    n = S.ssl_noise_create(ctx, F, M)
    st = torch.full((F,), -7, dtype=torch.int32, device="cuda:0")
    S.ssl_noise_set(n, to_dev(K.astype(np.complex128)), S.SSL_FP64, st)
    if enable:
        S.ssl_noise_enable_gevd(n)
    return n


def sqrt_pd(K):
    w, V = np.linalg.eigh(K)
    return (V * np.sqrt(w)) @ V.conj().T


@pytest.mark.parametrize("M,Ns,cond", [(3, 1, 10.0), (8, 1, 100.0), (16, 2, 100.0), (31, 3, 1e3),
                                       (60, 2, 100.0), (64, 5, 1e4)])
def test_gevd_gsvd_parity(S, ctx, M, Ns, cond):
    """ssl_gsvd in GEVD mode: sigma are the generalized eigenvalues; E_n spans the generalized
    noise eigenvectors (compared in the whitened coordinates K^{1/2} E, where the decomposition's
    own error bound lives), and E_n is K-orthonormal."""
    import torch
    say(f"ssl_gsvd GEVD M={M} Ns={Ns} cond(K)={cond:g} F=19")
    F = 19
    rng = np.random.default_rng(1300 + M)
    X = crandn(rng, F, 50, M).astype(np.complex64)
    R = oracle.corr(X).astype(np.complex64).astype(np.complex128)
    K = np.stack([random_pd(rng, M, cond) for _ in range(F)])
    n = gevd_noise(S, ctx, K)
    Rd = to_dev(R.astype(np.complex64))
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    sig = torch.zeros((F, M), dtype=torch.float32, device="cuda:0")
    st = torch.full((F,), -7, dtype=torch.int32, device="cuda:0")
    S.ssl_gsvd(ctx, Rd, n, Ns, En, sig, st)
    g_En, g_sig, g_st = to_host(En), to_host(sig), to_host(st)
    En_ref, sig_ref, st_ref = oracle.gevd(K, R, Ns)
    assert np.all(g_st == 0) and np.all(st_ref == 0), g_st
    worst = 0.0
    for f in range(F):
        Kh = sqrt_pd(K[f])
        Ki = np.linalg.inv(Kh)
        C = Ki @ R[f] @ Ki
        nC = np.linalg.norm(C)
        # generalized eigenvalues = singular values of C, backward stable to ~ M u |C|
        assert np.max(np.abs(g_sig[f] - sig_ref[f])) <= 8 * M * U32 * nC, f
        gap = sig_ref[f, Ns - 1] - sig_ref[f, Ns]
        Yg = Kh @ g_En[f].T.astype(np.complex128)
        Yr = Kh @ En_ref[f].T
        err = np.linalg.norm(projector(Yg) - projector(Yr), 2)
        bound = 16 * M * U32 * nC / gap + 4 * np.sqrt(M * cond) * U32
        assert err <= bound, (f, err, bound)
        worst = max(worst, err / bound)
        # K-orthonormal: E^H K E = Y^H Y = I
        assert np.linalg.norm(Yg.conj().T @ Yg - np.eye(M - Ns), 2) <= 8 * M * U32 + \
            4 * np.sqrt(M * cond) * U32
    say(f"  worst projector error / bound {worst:.3g}")
    S.ssl_noise_destroy(n)


def test_gevd_identity_noise_equals_gsvd(S, ctx):
    """K = I: K^{-1/2} = I, so GEVD and GSVD decompose the same matrix; the two modes give the
    same singular values and noise subspace to rounding."""
    import torch
    M, Ns, F = 16, 2, 7
    rng = np.random.default_rng(1401)
    R = oracle.corr(crandn(rng, F, 50, M).astype(np.complex64)).astype(np.complex64)
    K = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    n = gevd_noise(S, ctx, K)
    out = {}
    for mode in (S.SSL_SUBSPACE_GEVD, S.SSL_SUBSPACE_GSVD):
        S.ssl_ctx_set_subspace(ctx, mode)
        En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
        sig = torch.zeros((F, M), dtype=torch.float32, device="cuda:0")
        S.ssl_gsvd(ctx, to_dev(R), n, Ns, En, sig)
        out[mode] = (to_host(En), to_host(sig))
    S.ssl_ctx_set_subspace(ctx, S.SSL_SUBSPACE_GEVD)
    assert S.ssl_ctx_get_subspace(ctx) == S.SSL_SUBSPACE_GEVD
    (Eg, sg), (Es, ss) = out[S.SSL_SUBSPACE_GEVD], out[S.SSL_SUBSPACE_GSVD]
    for f in range(F):
        nR = np.linalg.norm(R[f].astype(np.complex128))
        assert np.max(np.abs(sg[f] - ss[f])) <= 8 * M * U32 * nR
        gap = ss[f, Ns - 1] - ss[f, Ns]
        err = np.linalg.norm(projector(Eg[f].T.astype(np.complex128)) -
                             projector(Es[f].T.astype(np.complex128)), 2)
        assert err <= 32 * M * U32 * nR / gap
    S.ssl_noise_destroy(n)


def test_gevd_planted_sources_nulled(S, ctx):
    """Noise-free R = H_s S H_s^H with coloured K: the generalized noise vectors the GPU returns are
    orthogonal to the source steering vectors themselves."""
    import torch
    M, Ns, F = 12, 2, 5
    rng = np.random.default_rng(1402)
    R = np.zeros((F, M, M), np.complex128)
    Hs = []
    for f in range(F):
        h = crandn(rng, M, Ns)
        R[f] = h @ np.diag([3.0, 1.5]) @ h.conj().T
        Hs.append(h)
    K = np.stack([random_pd(rng, M, 50.0) for _ in range(F)])
    n = gevd_noise(S, ctx, K)
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    S.ssl_gsvd(ctx, to_dev(R.astype(np.complex64)), n, Ns, En)
    g = to_host(En)
    for f in range(F):
        E = g[f].T.astype(np.complex128)
        # the complex64 rounding of R and of C limits the null to ~ M u cond(K)^(1/2) |h| |E|
        lim = 64 * M * U32 * np.sqrt(50.0) * np.linalg.norm(Hs[f]) * np.linalg.norm(E)
        assert np.max(np.abs(Hs[f].conj().T @ E)) <= lim, f
    S.ssl_noise_destroy(n)


def test_gevd_state_and_argument_errors(S, ctx):
    import torch
    say("GEVD state errors")
    M, Ns, F = 8, 1, 3
    rng = np.random.default_rng(1403)
    K = np.stack([random_pd(rng, M, 10.0) for _ in range(F)])
    n = gevd_noise(S, ctx, K, enable=False)
    R = torch.zeros((F, M, M), dtype=torch.complex64, device="cuda:0")
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_gsvd(ctx, R, n, Ns, En)
    assert e.value.code == S.SSL_ERR_STATE
    X = torch.zeros((F, 4, M), dtype=torch.complex64, device="cuda:0")
    H = torch.zeros((F, 72, M), dtype=torch.complex64, device="cuda:0")
    pk = torch.zeros(Ns, dtype=torch.int32, device="cuda:0")
    pv = torch.zeros(Ns, dtype=torch.float32, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_localize(ctx, X, n, H, S.SSL_FP32, 72, 1, Ns, 2, pk, pv)
    assert e.value.code == S.SSL_ERR_STATE
    with pytest.raises(S.SSLError) as e:
        S.ssl_localize_noalloc(ctx, X, n, H, S.SSL_FP32, 72, 1, Ns, 2, pk, pv)
    assert e.value.code == S.SSL_ERR_STATE
    d = S.block_desc(X, n, H, 72, 1, Ns, pk, pv)
    with pytest.raises(S.SSLError) as e:
        S.ssl_localize_batch(ctx, [d], S.SSL_FP32, 2)
    assert e.value.code == S.SSL_ERR_STATE and "block 0" in str(e.value)
    with pytest.raises(S.SSLError) as e:
        S.ssl_ctx_set_subspace(ctx, 2)
    assert e.value.code == S.SSL_ERR_ARG
    assert S.ssl_ctx_get_subspace(ctx) == S.SSL_SUBSPACE_GEVD
    # a NULL handle is SEVD-MUSIC in either mode: no state needed
    S.ssl_gsvd(ctx, R, None, Ns, En)
    # enabling on a handle not yet set computes K^{-1/2} at the first set
    n2 = S.ssl_noise_create(ctx, F, M)
    S.ssl_noise_enable_gevd(n2)
    S.ssl_noise_set(n2, to_dev(K), S.SSL_FP64)
    S.ssl_gsvd(ctx, R, n2, Ns, En)
    S.ssl_noise_destroy(n2)
    S.ssl_noise_destroy(n)


def localize(S, fn, ctx, w, Xd, n, Hd):
    import torch
    pk = torch.full((w.Ns,), -7, dtype=torch.int32, device="cuda:0")
    pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
    Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
    st = torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0")
    fn(ctx, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, pk, pv, Pbar, st)
    return dict(peaks=to_host(pk), peak_val=to_host(pv), Pbar=to_host(Pbar), status=to_host(st))


def noise_handle(S, ctx, w):
    import torch
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_enable_gevd(n)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    return n, oracle.noise_corr(Xn), Kd


@pytest.mark.parametrize("name,blocks", [("small", 6), ("paper", 4)])
def test_gevd_localize_matches_oracle(S, ctx, name, blocks):
    """Whole blocks in GEVD mode against the oracle's GEVD-MUSIC: Pbar within 1e-4, peaks identical
    outside near-ties; the allocation-free entry point gives the same bytes."""
    w = synth.workload_small(n_blocks=blocks) if name == "small" else \
        synth.workload_paper(n_blocks=blocks)
    n, K, _ = noise_handle(S, ctx, w)
    H = w.steering_table()
    Hd = to_dev(H)
    worst = 0.0
    for b in range(blocks):
        X, dirs, _ = w.block(b)
        say(f"ssl_localize GEVD {name} M={w.M} block {b}")
        Xd = to_dev(X)
        g = localize(S, S.ssl_localize, ctx, w, Xd, n, Hd)
        r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16, gevd=True)
        assert np.all(g["status"] == 0) and np.all(r["status"] == 0)
        rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
        say(f"  rel {rel:.2e} peaks gpu {g['peaks']} ref {r['peaks']} planted {dirs} near-ties {amb}")
        worst = max(worst, rel)
        assert rel <= 1e-4
        assert not amb
        assert np.array_equal(g["peaks"], r["peaks"])
        na = localize(S, S.ssl_localize_noalloc, ctx, w, Xd, n, Hd)
        for k in g:
            assert np.array_equal(na[k], g[k]), k
    say(f"  max Pbar relative error {worst:.3g}")
    S.ssl_noise_destroy(n)


def test_gevd_batch_bit_identical(S, ctx):
    """A batch mixing GEVD blocks of two array sizes and SEVD blocks equals each block alone."""
    import torch
    wp = synth.workload_paper(n_blocks=3)
    ws = synth.workload_small(n_blocks=3)
    handles = {w.M: (noise_handle(S, ctx, w)[0], to_dev(w.steering_table())) for w in (wp, ws)}
    plan = [(wp, 0, False), (ws, 0, False), (wp, 1, True), (ws, 1, False), (wp, 2, False)]
    say(f"ssl_localize_batch GEVD: {[(w.M, b, sevd) for w, b, sevd in plan]}")
    blocks, outs, descs = [], [], []
    for w, b, sevd in plan:
        Xd = to_dev(w.block(b)[0])
        n, Hd = handles[w.M]
        o = dict(pk=torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0"),
                 pv=torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0"),
                 Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
                 st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))
        blocks.append((w, Xd, None if sevd else n, Hd))
        outs.append(o)
        descs.append(S.block_desc(Xd, None if sevd else n, Hd, w.grid.n_az, w.grid.n_el, w.Ns,
                                  o["pk"], o["pv"], o["Pbar"], o["st"]))
    for rep in range(2):                             # the second call replays the captured batch
        for o in outs:
            o["Pbar"].zero_()
        S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
        got = [{k: to_host(v) for k, v in o.items()} for o in outs]
        for i, (w, Xd, n, Hd) in enumerate(blocks):
            ref = localize(S, S.ssl_localize, ctx, w, Xd, n, Hd)
            assert np.array_equal(got[i]["pk"], ref["peaks"]), (rep, i)
            assert np.array_equal(got[i]["pv"], ref["peak_val"]), (rep, i)
            assert np.array_equal(got[i]["Pbar"], ref["Pbar"]), (rep, i)
            assert np.array_equal(got[i]["st"], ref["status"]), (rep, i)
    for n, _ in handles.values():
        S.ssl_noise_destroy(n)


def test_gevd_noise_update_recomputes(S, ctx):
    """After ssl_noise_update and ssl_noise_update_frames the handle's K^{-1/2} follows the new K:
    the localization equals that of a fresh handle set to the blended K (read back with
    ssl_noise_get), bit for bit."""
    import torch
    w = synth.workload_small(n_blocks=2)
    n, _, Kd = noise_handle(S, ctx, w)
    Hd = to_dev(w.steering_table())
    Xd = to_dev(w.block(0)[0])
    rng = np.random.default_rng(1404)
    Khat = np.stack([random_pd(rng, w.M, 30.0) for _ in range(w.F)])
    S.ssl_noise_update(n, to_dev(Khat), S.SSL_FP64, 0.3)
    Xn2 = to_dev(crandn(rng, w.F, 40, w.M).astype(np.complex64))
    S.ssl_noise_update_frames(ctx, [n], [Xn2], 0.5)
    Kb = torch.zeros_like(Kd)
    S.ssl_noise_get(n, Kb)
    fresh = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(fresh, Kb, S.SSL_FP64)
    S.ssl_noise_enable_gevd(fresh)
    a = localize(S, S.ssl_localize, ctx, w, Xd, n, Hd)
    b = localize(S, S.ssl_localize, ctx, w, Xd, fresh, Hd)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # and against the oracle on the blended K
    r = oracle.localize(w.block(0)[0], to_host(Kb), w.steering_table(), w.grid.n_az, w.grid.n_el,
                        w.Ns, nthreads=8, gevd=True)
    rel = float(np.max(np.abs(a["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
    assert rel <= 1e-4
    S.ssl_noise_destroy(fresh)
    S.ssl_noise_destroy(n)


def test_gevd_sliding_window(S, ctx):
    """The frame stream in GEVD mode: windows ending at frames 49, 69, 89 against the oracle's
    GEVD-MUSIC on the same window (cold solves)."""
    import torch
    w = synth.workload_small(n_blocks=2)
    X = np.ascontiguousarray(np.concatenate([w.block(b)[0] for b in (0, 1)], axis=1))
    T = 50
    n, K, _ = noise_handle(S, ctx, w)
    H = w.steering_table()
    Hd = to_dev(H)
    Xd = to_dev(X)
    s = S.ssl_sliding_create(ctx, w.F, w.M, T)
    S.ssl_sliding_push(s, Xd[:, :30, :])
    for f in (49, 69, 89):
        S.ssl_sliding_push(s, Xd[:, f - 19:f + 1, :])
        pk = torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0")
        pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
        Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
        bst = torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0")
        S.ssl_sliding_localize(s, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, w.Ns, 2, 0, pk, pv,
                               Pbar, bst)
        r = oracle.localize(np.ascontiguousarray(X[:, f - T + 1:f + 1, :]), K, H, w.grid.n_az,
                            w.grid.n_el, w.Ns, nthreads=8, gevd=True)
        g_P = to_host(Pbar)
        rel = float(np.max(np.abs(g_P.astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
        say(f"  sliding GEVD frame {f}: rel {rel:.2e} peaks {to_host(pk)} ref {r['peaks']}")
        assert np.all(to_host(bst) == 0)
        assert rel <= 1e-4
        assert not amb
        assert np.array_equal(to_host(pk), r["peaks"])
    S.ssl_sliding_destroy(s)
    S.ssl_noise_destroy(n)


def test_gevd_not_pd_noise(S, ctx):
    """A bin whose K is not positive definite is flagged SSL_BIN_NOT_PD and excluded, as in GSVD
    mode."""
    import torch
    M, Ns, F = 8, 1, 4
    rng = np.random.default_rng(1405)
    K = np.stack([random_pd(rng, M, 10.0) for _ in range(F)])
    K[2] = np.diag(np.r_[1.0, -1.0, np.ones(M - 2)]).astype(complex)
    n = gevd_noise(S, ctx, K)
    R = oracle.corr(crandn(rng, F, 30, M).astype(np.complex64)).astype(np.complex64)
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    st = torch.full((F,), -7, dtype=torch.int32, device="cuda:0")
    S.ssl_gsvd(ctx, to_dev(R), n, Ns, En, None, st)
    g = to_host(st)
    assert g[2] == S.SSL_BIN_NOT_PD and np.all(g[[0, 1, 3]] == 0), g
    S.ssl_noise_destroy(n)
