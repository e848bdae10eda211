"""HIP path vs the FP64 oracle, element by element, through the C ABI (MI355X only).

Each test prints the case (entry point, shape, seed) before its GPU step.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import crandn, random_pd
from gpu_util import U32, corr_bound, peak_ambiguity, projector, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def gpu_corr(S, ctx, X, prec, scale=None, accumulate=False, R0=None):
    import torch
    Xd = to_dev(X) if isinstance(X, np.ndarray) else X
    F, T, M = Xd.shape
    dt = torch.complex128 if prec == S.SSL_FP64 else torch.complex64
    R = torch.zeros((F, M, M), dtype=dt, device="cuda:0") if R0 is None else to_dev(R0)
    S.ssl_corr_accum(ctx, Xd, (1.0 / T) if scale is None else scale, accumulate, prec, R)
    return to_host(R)


def set_noise(S, ctx, K):
    import torch
    F, M, _ = K.shape
    n = S.ssl_noise_create(ctx, F, M)
    st = torch.zeros(F, dtype=torch.int32, device="cuda:0")
    S.ssl_noise_set(n, to_dev(K.astype(np.complex128)), S.SSL_FP64, st)
    return n, to_host(st)


# ------------------------------------------------------------------------------------------------
# A1: correlation
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("M,T", [(1, 5), (3, 7), (8, 50), (17, 50), (33, 65), (60, 50), (64, 130)])
def test_corr_fp32(S, ctx, M, T):
    say(f"ssl_corr_accum fp32 M={M} T={T} seed={M * 1000 + T}")
    rng = np.random.default_rng(M * 1000 + T)
    F = 5
    X = crandn(rng, F, T, M).astype(np.complex64)
    R = gpu_corr(S, ctx, X, S.SSL_FP32)
    ref = oracle.corr(X)
    assert np.all(np.abs(R.astype(np.complex128) - ref) <= corr_bound(X) + 1e-30)
    # Hermitian to the bit, real diagonal
    assert np.array_equal(R, np.conj(np.swapaxes(R, 1, 2)))
    assert np.all(np.diagonal(R, axis1=1, axis2=2).imag == 0)


def test_corr_fp32_strided_and_accumulate(S, ctx):
    import torch
    say("ssl_corr_accum fp32 strided + accumulate M=60 T=50")
    rng = np.random.default_rng(7)
    F, T, M = 9, 50, 60
    big = crandn(rng, F, T + 3, M + 5).astype(np.complex64)
    Xd = to_dev(big)[:, 2:T + 2, :M]
    assert Xd.stride() == ((T + 3) * (M + 5), M + 5, 1)
    X = big[:, 2:T + 2, :M]
    R0 = oracle.corr(crandn(rng, F, 4, M).astype(np.complex64)).astype(np.complex64)
    R = gpu_corr(S, ctx, Xd, S.SSL_FP32, accumulate=True, R0=R0)
    ref = oracle.corr(X) + R0.astype(np.complex128)
    assert np.all(np.abs(R - ref) <= corr_bound(X) + 4 * U32 * np.abs(R0) + 1e-30)


@pytest.mark.parametrize("M,T", [(8, 50), (60, 240), (64, 3)])
def test_corr_fp64(S, ctx, M, T):
    say(f"ssl_corr_accum fp64 M={M} T={T}")
    rng = np.random.default_rng(11 + M)
    F = 4
    X = crandn(rng, F, T, M).astype(np.complex64)
    R = gpu_corr(S, ctx, X, S.SSL_FP64)
    ref = oracle.corr(X)
    Xa = np.abs(X.astype(np.complex128))
    bound = (2 * T + 4) * 2.0 ** -53 * np.einsum("fti,ftj->fij", Xa, Xa) / T
    assert np.all(np.abs(R - ref) <= bound + 1e-300)
    assert np.array_equal(R, np.conj(np.swapaxes(R, 1, 2)))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_corr_low_precision(S, ctx, prec):
    """bf16/fp16 MFMA inputs, FP32 accumulation: the inputs' rounding (2^-9 / 2^-12 relative)
    dominates; the bound uses the rounded inputs' error, not FP32 roundoff."""
    say(f"ssl_corr_accum {prec} M=60 T=50")
    rng = np.random.default_rng(12)
    F, T, M = 3, 50, 60
    X = crandn(rng, F, T, M).astype(np.complex64)
    p = S.SSL_BF16 if prec == "bf16" else S.SSL_FP16
    R = gpu_corr(S, ctx, X, p)
    ref = oracle.corr(X)
    u = 2.0 ** -9 if prec == "bf16" else 2.0 ** -12
    Xa = np.abs(X.astype(np.complex128))
    bound = (2 * u + (2 * T + 4) * U32) * np.einsum("fti,ftj->fij", Xa, Xa) / T * 2
    assert np.all(np.abs(R - ref) <= bound)
    assert np.array_equal(R, np.conj(np.swapaxes(R, 1, 2)))


# ------------------------------------------------------------------------------------------------
# A2: noise handle (FP64 Gauss-Jordan inverse; its pivots are the Cholesky pivots of the PD test)
# ------------------------------------------------------------------------------------------------
def test_noise_set_get_and_not_pd(S, ctx):
    import torch
    say("ssl_noise_set / get / NOT_PD F=6 M=12")
    rng = np.random.default_rng(13)
    F, M = 6, 12
    K = np.stack([random_pd(rng, M, 1e4) for _ in range(F)])
    # bin 2: negative eigenvalue; bin 4: rank deficient (fewer frames than channels)
    w, V = np.linalg.eigh(K[2])
    w[0] = -1.0
    K[2] = (V * w) @ V.conj().T
    K[4] = oracle.corr(crandn(rng, 1, M - 4, M).astype(np.complex64))[0]
    n, st = set_noise(S, ctx, K)
    want = np.array([oracle.cholesky(K[f])[0] for f in range(F)])
    assert np.array_equal(st, want) and st[2] == S.SSL_BIN_NOT_PD and st[4] == S.SSL_BIN_NOT_PD
    Kout = torch.zeros((F, M, M), dtype=torch.complex128, device="cuda:0")
    S.ssl_noise_get(n, Kout)
    assert np.array_equal(to_host(Kout), K)
    S.ssl_noise_destroy(n)


def test_noise_update_blend(S, ctx):
    import torch
    say("ssl_noise_update alpha=0.95 F=3 M=8")
    rng = np.random.default_rng(14)
    F, M = 3, 8
    K0 = np.stack([random_pd(rng, M, 10.0) for _ in range(F)])
    K1 = np.stack([random_pd(rng, M, 10.0) for _ in range(F)])
    n, _ = set_noise(S, ctx, K0)
    st = torch.zeros(F, dtype=torch.int32, device="cuda:0")
    S.ssl_noise_update(n, to_dev(K1), S.SSL_FP64, 0.95, st)
    Kout = torch.zeros((F, M, M), dtype=torch.complex128, device="cuda:0")
    S.ssl_noise_get(n, Kout)
    assert np.allclose(to_host(Kout), 0.95 * K0 + 0.05 * K1, rtol=1e-15, atol=1e-15)
    assert np.all(to_host(st) == 0)
    S.ssl_noise_destroy(n)


# ------------------------------------------------------------------------------------------------
# A3-A5: GSVD (whitening, Jacobi SVD, sort, noise subspace)
# ------------------------------------------------------------------------------------------------
def run_gsvd(S, ctx, R64, K, Ns, max_sweeps=0):
    import torch
    F, M, _ = R64.shape
    n, kst = set_noise(S, ctx, K)
    Rd = to_dev(R64.astype(np.complex64))
    En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device="cuda:0")
    sig = torch.zeros((F, M), dtype=torch.float32, device="cuda:0")
    st = torch.zeros(F, dtype=torch.int32, device="cuda:0")
    conv = torch.zeros((F, 3), dtype=torch.int32, device="cuda:0")
    S.ssl_gsvd(ctx, Rd, n, Ns, En, sig, st, conv, max_sweeps)
    out = dict(En=to_host(En), sigma=to_host(sig), status=to_host(st), conv=to_host(conv))
    S.ssl_noise_destroy(n)
    return out


def gsvd_case(M, F, Ns, seed, cond=100.0, T=50):
    rng = np.random.default_rng(seed)
    X = crandn(rng, F, T, M).astype(np.complex64)
    R = oracle.corr(X).astype(np.complex64).astype(np.complex128)   # the bytes the GPU reads
    K = np.stack([random_pd(rng, M, cond) for _ in range(F)])
    return R, K


@pytest.mark.parametrize("M,Ns", [(2, 1), (3, 1), (8, 1), (13, 3), (16, 2), (31, 2), (60, 2), (64, 5)])
def test_gsvd_parity(S, ctx, M, Ns):
    say(f"ssl_gsvd M={M} Ns={Ns} F=19")
    F = 19
    R, K = gsvd_case(M, F, Ns, seed=300 + M)
    g = run_gsvd(S, ctx, R, K, Ns)
    En_ref, sig_ref, st_ref, _ = oracle.gsvd(K, R, Ns)
    assert np.all(st_ref == 0) and np.all(g["status"] == 0), g["status"]
    assert np.all(g["conv"][:, 0] <= 20)
    # R comes from T = 50 frames: rank min(M, 50), found by the pivoted QR
    assert np.all(g["conv"][:, 2] == min(M, 50))
    errs = []
    for f in range(F):
        A = np.linalg.solve(K[f], R[f])
        nA = np.linalg.norm(A)
        # singular values: backward-stable to ~ M u |A|
        assert np.max(np.abs(g["sigma"][f] - sig_ref[f])) <= 8 * M * U32 * nA
        gap = sig_ref[f, Ns - 1] - sig_ref[f, Ns]
        err = np.linalg.norm(projector(g["En"][f].T.astype(np.complex128)) - projector(En_ref[f].T), 2)
        errs.append(err * gap / nA)
        assert err <= 16 * M * U32 * nA / gap, (f, err, gap)
        # unitary columns
        E = g["En"][f].T.astype(np.complex128)
        assert np.linalg.norm(E.conj().T @ E - np.eye(M - Ns), 2) <= 8 * M * U32
    say(f"  projector error * gap / |A|: max {max(errs):.3g} (units of u: {max(errs) / U32:.1f})")


@pytest.mark.parametrize("M,Ns,T", [(8, 7, 50), (60, 59, 130)])
def test_gsvd_single_noise_vector(S, ctx, M, Ns, T):
    """Ns = M - 1: E_n is one vector (full-rank R so that it is unique up to phase)."""
    say(f"ssl_gsvd M={M} Ns={Ns} T={T} F=7")
    F = 7
    R, K = gsvd_case(M, F, Ns, seed=700 + M, T=T)
    g = run_gsvd(S, ctx, R, K, Ns)
    En_ref, sig_ref, st_ref, _ = oracle.gsvd(K, R, Ns)
    assert np.all(g["status"] == 0) and np.all(g["conv"][:, 2] == M)
    for f in range(F):
        nA = np.linalg.norm(np.linalg.solve(K[f], R[f]))
        gap = sig_ref[f, Ns - 1] - sig_ref[f, Ns]
        err = np.linalg.norm(projector(g["En"][f].T.astype(np.complex128)) - projector(En_ref[f].T), 2)
        assert err <= 16 * M * U32 * nA / gap, (f, err, gap)


def test_gsvd_max_bins(S, ctx):
    """F at its limit (65535 bins, M = 2): every bin converged; sampled bins against the oracle."""
    say("ssl_gsvd F=65535 M=2 Ns=1")
    F, M, Ns = 65535, 2, 1
    R, K = gsvd_case(M, F, Ns, seed=65535, T=5)
    g = run_gsvd(S, ctx, R, K, Ns)
    assert np.all(g["status"] == 0)
    pick = np.random.default_rng(1).choice(F, 200, replace=False)
    En_ref, sig_ref, _, _ = oracle.gsvd(K[pick], R[pick], Ns)
    for i, f in enumerate(pick):
        nA = np.linalg.norm(np.linalg.solve(K[f], R[f]))
        gap = sig_ref[i, 0] - sig_ref[i, 1]
        err = np.linalg.norm(projector(g["En"][f].T.astype(np.complex128)) - projector(En_ref[i].T), 2)
        assert err <= 16 * M * U32 * nA / gap, (f, err, gap)


def test_empty_and_out_of_range_shapes(S, ctx):
    """Empty inputs (F = 0, T = 0, an empty batch) and sizes past the limits are argument errors:
    nothing is enqueued."""
    import torch
    say("empty / out-of-range shapes")
    R = torch.zeros((1, 8, 8), dtype=torch.complex64, device="cuda:0")
    X0 = torch.zeros((0, 5, 8), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_corr_accum(ctx, X0, 1.0, 0, S.SSL_FP32, R[:0])            # F = 0
    assert e.value.code == S.SSL_ERR_ARG
    XT = torch.zeros((1, 0, 8), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_corr_accum(ctx, XT, 1.0, 0, S.SSL_FP32, R)                # T = 0
    assert e.value.code == S.SSL_ERR_ARG
    with pytest.raises(S.SSLError) as e:
        S.ssl_localize_batch(ctx, [], S.SSL_FP32, 2)                     # no blocks
    assert e.value.code == S.SSL_ERR_ARG
    with pytest.raises(S.SSLError) as e:
        S.ssl_noise_create(ctx, 65536, 2)                                # F past 65535
    assert e.value.code == S.SSL_ERR_ARG
    with pytest.raises(S.SSLError) as e:
        S.ssl_noise_create(ctx, 4, 65)                                   # M past 64
    assert e.value.code == S.SSL_ERR_ARG


def test_gsvd_status_paths(S, ctx):
    say("ssl_gsvd status paths M=8 F=6")
    F, M, Ns = 6, 8, 2
    R, K = gsvd_case(M, F, Ns, seed=31)
    w, V = np.linalg.eigh(K[1])
    w[0] = -1.0
    K[1] = (V * w) @ V.conj().T                 # NOT_PD
    R[3, 2, 5] = np.nan                          # NONFINITE
    g = run_gsvd(S, ctx, R, K, Ns)
    assert g["status"].tolist() == [0, 1, 0, 3, 0, 0]
    assert np.all(g["En"][1] == 0) and np.all(g["En"][3] == 0) and np.all(g["sigma"][3] == 0)
    # max_sweeps = 1 cannot converge a random problem: NO_CONV reported, E_n zeroed
    R2, K2 = gsvd_case(16, 3, 2, seed=32)
    g = run_gsvd(S, ctx, R2, K2, 2, max_sweeps=1)
    assert np.all(g["status"] == 2) and np.all(g["conv"][:, 0] == 1)


def test_gsvd_identity_noise_is_sevd(S, ctx):
    """K = I: E_n spans the eigenvectors of the M - Ns smallest eigenvalues of R (LAPACK eigh)."""
    say("ssl_gsvd K=I M=60 F=7")
    F, M, Ns = 7, 60, 2
    R, _ = gsvd_case(M, F, Ns, seed=33)
    K = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    g = run_gsvd(S, ctx, R, K, Ns)
    for f in range(F):
        w, V = np.linalg.eigh(R[f])
        gap = w[M - Ns] - w[M - Ns - 1]
        err = np.linalg.norm(projector(g["En"][f].T.astype(np.complex128)) - projector(V[:, :M - Ns]), 2)
        assert err <= 16 * M * U32 * np.linalg.norm(R[f]) / gap


def test_gsvd_zero_matrix(S, ctx):
    say("ssl_gsvd R=0 M=8")
    F, M, Ns = 2, 8, 1
    R = np.zeros((F, M, M), np.complex128)
    K = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    g = run_gsvd(S, ctx, R, K, Ns)
    assert np.all(g["status"] == 0) and np.all(g["sigma"] == 0)
    assert np.array_equal(np.abs(g["En"][0].T), np.eye(M)[:, Ns:])


# ------------------------------------------------------------------------------------------------
# A6-A7: spectrum, bin sum, peaks
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("M,Ns,D,p", [(8, 1, 72, 2), (8, 1, 72, 1), (60, 2, 1368, 2), (33, 4, 100, 2),
                                       (64, 1, 37, 2), (5, 3, 1, 2)])
def test_spectrum_parity(S, ctx, M, Ns, D, p):
    import torch
    say(f"ssl_music_spectrum M={M} Ns={Ns} D={D} p={p}")
    rng = np.random.default_rng(400 + M + D)
    F = 21
    H = crandn(rng, F, D, M).astype(np.complex64)
    En = np.stack([np.linalg.qr(crandn(rng, M, M))[0][:, Ns:].T for _ in range(F)]).astype(np.complex64)
    st = np.zeros(F, np.int32)
    st[5] = 1
    P = torch.zeros((F, D), dtype=torch.float32, device="cuda:0")
    Pbar = torch.zeros(D, dtype=torch.float32, device="cuda:0")
    S.ssl_music_spectrum(ctx, to_dev(H), S.SSL_FP32, to_dev(En), Ns, p, P, Pbar, to_dev(st))
    Pg, Pbg = to_host(P), to_host(Pbar)
    Pr, Pbr = oracle.spectrum(H, En.astype(np.complex128), Ns, p=p, status=st)
    assert np.all(Pg[5] == 0)
    ok = np.arange(F) != 5
    # den is a sum of 2(M-Ns) squares of length-2M dot products: relative error ~ 4 M u P / M
    rel = np.abs(Pg[ok] - Pr[ok]) / Pr[ok]
    assert np.max(rel) <= 16 * M * U32 * np.max(Pr[ok]) / np.min(Pr[ok]) + 1e-5
    assert np.max(np.abs(Pbg - Pbr) / Pbr) <= 1e-5


def test_peaks_fixtures_on_gpu(S, ctx):
    import torch
    with open(os.path.join(GOLDEN, "peaks_cases.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        say(f"ssl_peaks fixture '{c['name']}'")
        pk = torch.zeros(c["Ns"], dtype=torch.int32, device="cuda:0")
        pv = torch.zeros(c["Ns"], dtype=torch.float32, device="cuda:0")
        S.ssl_peaks(ctx, to_dev(np.asarray(c["Pbar"], np.float32)), c["n_az"], c["n_el"], c["Ns"], pk, pv)
        assert to_host(pk).tolist() == c["peaks"], c["name"]


@pytest.mark.parametrize("n_el,n_az,Ns", [(19, 72, 3), (1, 72, 1), (19, 72, 2), (7, 3, 5), (100, 100, 4)])
def test_peaks_bit_exact(S, ctx, n_el, n_az, Ns):
    """Same float32 values on both sides (the oracle compares their exact FP64 widening)."""
    import torch
    say(f"ssl_peaks random grid {n_el}x{n_az} Ns={Ns}")
    rng = np.random.default_rng(n_el * n_az + Ns)
    for trial in range(4):
        v = rng.random(n_el * n_az).astype(np.float32)
        if trial >= 2:                                   # plateaus and exact ties
            v = np.round(v * 6).astype(np.float32)
        pk = torch.zeros(Ns, dtype=torch.int32, device="cuda:0")
        pv = torch.zeros(Ns, dtype=torch.float32, device="cuda:0")
        S.ssl_peaks(ctx, to_dev(v), n_az, n_el, Ns, pk, pv)
        want, wv = oracle.peaks(v.astype(np.float64), n_el, n_az, Ns)
        assert np.array_equal(to_host(pk), want)
        assert np.array_equal(to_host(pv).astype(np.float64), wv)


# ------------------------------------------------------------------------------------------------
# whole path
# ------------------------------------------------------------------------------------------------
def localize_gpu(S, ctx, w, X, noise, Hd, prec=None, p=2):
    import torch
    prec = S.SSL_FP32 if prec is None else prec
    pk = torch.zeros(w.Ns, dtype=torch.int32, device="cuda:0")
    pv = torch.zeros(w.Ns, dtype=torch.float32, device="cuda:0")
    Pbar = torch.zeros(w.D, dtype=torch.float32, device="cuda:0")
    st = torch.zeros(w.F, dtype=torch.int32, device="cuda:0")
    S.ssl_localize(ctx, to_dev(X), noise, Hd, prec, w.grid.n_az, w.grid.n_el, w.Ns, p, pk, pv, Pbar, st)
    return dict(peaks=to_host(pk), peak_val=to_host(pv), Pbar=to_host(Pbar), status=to_host(st))


def noise_from_frames(S, ctx, w):
    import torch
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    return n, oracle.noise_corr(Xn)


def check_block(o_gpu, o_ref, w, Ns=None):
    """Pbar relative error against the oracle, and the peak comparison.  A peak decision can
    differ between two correct evaluations only where the reference values are within twice the
    evaluation's own error of each other: the near-tie radius is this block's measured maximum
    relative Pbar error, so outside the reasons listed the returned peaks must be identical."""
    Ns = w.Ns if Ns is None else Ns
    rel = np.abs(o_gpu["Pbar"].astype(np.float64) - o_ref["Pbar"]) / o_ref["Pbar"]
    rel = float(rel.max())
    amb = peak_ambiguity(o_ref["Pbar"], w.grid.n_el, w.grid.n_az, Ns, max(rel, 1e-7))
    same = np.array_equal(o_gpu["peaks"], o_ref["peaks"])
    return rel, same, amb


@pytest.mark.parametrize("blocks", [range(10)])
def test_localize_small_workload(S, ctx, blocks):
    """All 10 blocks of the 8-mic workload: peaks bit-exact, Pbar within 1e-4 (FP32 path)."""
    w = synth.workload_small(n_blocks=10)
    n, K = noise_from_frames(S, ctx, w)
    Hd = to_dev(w.steering_table())
    H = w.steering_table()
    worst = 0.0
    for b in blocks:
        say(f"ssl_localize 8ch block {b}")
        X, dirs, _ = w.block(b)
        g = localize_gpu(S, ctx, w, X, n, Hd)
        r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=8)
        assert np.all(g["status"] == 0) and np.all(r["status"] == 0)
        rel, same, amb = check_block(g, r, w)
        worst = max(worst, rel)
        assert rel <= 1e-4, (b, rel)
        assert not amb, (b, amb)
        assert same, (b, g["peaks"], r["peaks"])
        assert g["peaks"][0] == dirs[0]
    say(f"  max Pbar relative error {worst:.3g}")
    S.ssl_noise_destroy(n)


def test_localize_paper_workload(S, ctx):
    """60-mic, 257-bin, 1368-direction blocks at full size (the paper-scale workload, eight seeded
    blocks): Pbar within 1e-4 of the FP64 oracle, no near-tie within the measured error, and the
    returned peaks identical."""
    w = synth.workload_paper(n_blocks=1000)
    n, K = noise_from_frames(S, ctx, w)
    H = w.steering_table()
    Hd = to_dev(H)
    worst = 0.0
    for b in range(8):
        say(f"ssl_localize 60ch block {b}")
        X, dirs, snr = w.block(b)
        g = localize_gpu(S, ctx, w, X, n, Hd)
        r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16)
        assert np.array_equal(g["status"], r["status"])
        rel, same, amb = check_block(g, r, w)
        worst = max(worst, rel)
        say(f"  block {b}: snr {snr:.1f} dB, rel {rel:.3g}, peaks gpu {g['peaks']} ref {r['peaks']} "
            f"src {dirs} near-ties {amb}")
        assert rel <= 1e-4
        assert not amb
        assert same
        # the peak values are Pbar at the peaks: within the same bound
        assert np.all(np.abs(g["peak_val"] - r["peak_val"]) <= 1e-4 * r["peak_val"])
    say(f"  max Pbar relative error over 8 blocks {worst:.3g}")
    S.ssl_noise_destroy(n)


def test_api_errors(S, ctx):
    import torch
    say("argument validation")
    X = torch.zeros((4, 5, 8), dtype=torch.complex64, device="cuda:0")
    R = torch.zeros((4, 8, 8), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_corr_accum(ctx, X, 1.0, 0, 7, R)
    assert e.value.code == S.SSL_ERR_ARG
    n = S.ssl_noise_create(ctx, 4, 8)
    En = torch.zeros((4, 7, 8), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(S.SSLError) as e:
        S.ssl_gsvd(ctx, R, n, 1, En)                   # never set
    assert e.value.code == S.SSL_ERR_STATE
    with pytest.raises(S.SSLError) as e:
        S.ssl_gsvd(ctx, R, n, 8, En)                   # Ns == M
    assert e.value.code == S.SSL_ERR_ARG
    S.ssl_noise_destroy(n)
    small = S.ssl_ctx_create(0, 1024)
    with pytest.raises(S.SSLError) as e:
        S.ssl_noise_create(small, 4, 8)
    assert e.value.code == S.SSL_ERR_BUDGET
    S.ssl_ctx_destroy(small)
