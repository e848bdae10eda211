"""eq.5 with p = 2 through the signal subspace (ssl_ctx_set_projection, the default at every table
precision):
den = |h|^2 - |L^{-1} E_s^H h|^2 in FP64.  Against the noise-vector projection and the FP64
oracle's eq.5 (a sum over the noise vectors): P-bar within the FP32 bar, the same peaks; batches
mixing blocks that use it and blocks that cannot (Ns > 3, GEVD, SEVD) equal each block alone;
failed bins contribute nothing.  MI355X only."""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import peak_ambiguity, to_dev, to_host

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


def outs(w, Ns):
    import torch
    return dict(pk=torch.full((Ns,), -7, dtype=torch.int32, device="cuda:0"),
                pv=torch.zeros(Ns, dtype=torch.float32, device="cuda:0"),
                Pbar=torch.zeros(w.D, dtype=torch.float32, device="cuda:0"),
                st=torch.full((w.F,), -7, dtype=torch.int32, device="cuda:0"))


def single(S, ctx, w, Xd, n, Hd, Ns):
    o = outs(w, Ns)
    S.ssl_localize(ctx, Xd, n, Hd, S.SSL_FP32, w.grid.n_az, w.grid.n_el, Ns, 2, o["pk"], o["pv"],
                   o["Pbar"], o["st"])
    return {k: to_host(v) for k, v in o.items()}


def noise_handle(S, ctx, w):
    import torch
    Xn = w.noise_frames()
    Kd = torch.zeros((w.F, w.M, w.M), dtype=torch.complex128, device="cuda:0")
    S.ssl_corr_accum(ctx, to_dev(Xn), 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, Kd, S.SSL_FP64)
    return n, oracle.noise_corr(Xn)


@pytest.mark.parametrize("name,blocks", [("small", 6), ("paper", 6)])
def test_signal_form_matches_noise_form_and_oracle(S, ctx, name, blocks):
    w = synth.workload_small(n_blocks=blocks) if name == "small" else \
        synth.workload_paper(n_blocks=blocks)
    n, K = noise_handle(S, ctx, w)
    H = w.steering_table()
    Hd = to_dev(H)
    assert S.ssl_ctx_get_projection(ctx) == S.SSL_PROJ_SIGNAL
    worst = 0.0
    for b in range(blocks):
        X, dirs, _ = w.block(b)
        Xd = to_dev(X)
        g = single(S, ctx, w, Xd, n, Hd, w.Ns)
        S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_NOISE)
        try:
            gn = single(S, ctx, w, Xd, n, Hd, w.Ns)
        finally:
            S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_SIGNAL)
        r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16)
        assert np.all(g["st"] == 0) and np.all(gn["st"] == 0)
        rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
        rel_n = float(np.max(np.abs(g["Pbar"].astype(np.float64) - gn["Pbar"]) / gn["Pbar"]))
        amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, w.Ns, max(rel, 1e-7))
        say(f"  {name} block {b}: signal form vs oracle {rel:.2e}, vs noise form {rel_n:.2e}, "
            f"peaks {g['pk']} {gn['pk']} ref {r['peaks']}")
        worst = max(worst, rel)
        assert rel <= 1e-4 and rel_n <= 1e-4
        assert not amb
        assert np.array_equal(g["pk"], r["peaks"]) and np.array_equal(gn["pk"], r["peaks"])
        assert np.all(np.abs(g["pv"] - r["peak_val"]) <= 1e-4 * r["peak_val"])
    say(f"  max Pbar relative error {worst:.3g}")
    S.ssl_noise_destroy(n)


@pytest.mark.parametrize("Ns", [1, 3])
def test_signal_form_other_ns(S, ctx, Ns):
    """Ns = 1 and 3 on the 60-channel workload (the workload's sources are 2: the form holds
    whatever the split, the oracle decides with the same Ns)."""
    w = synth.workload_paper(n_blocks=2)
    n, K = noise_handle(S, ctx, w)
    H = w.steering_table()
    Hd = to_dev(H)
    X, _, _ = w.block(0)
    g = single(S, ctx, w, to_dev(X), n, Hd, Ns)
    r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, Ns, nthreads=16)
    rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
    amb = peak_ambiguity(r["Pbar"], w.grid.n_el, w.grid.n_az, Ns, max(rel, 1e-7))
    say(f"  Ns={Ns}: rel {rel:.2e} peaks {g['pk']} ref {r['peaks']} near-ties {amb}")
    assert np.all(g["st"] == 0)
    assert rel <= 1e-4
    if not amb:
        assert np.array_equal(g["pk"], r["peaks"])
    S.ssl_noise_destroy(n)


def test_batch_mixing_forms_equals_single(S, ctx):
    """One steering table, blocks with Ns = 1, 2, 3 (signal form), Ns = 4 (noise form) and an SEVD
    block (signal form): every block's outputs equal its single-block call bit for bit, twice (the
    second call replays the captured batch).  GEVD blocks (noise form) mixed with SEVD blocks are
    covered by the GEVD tests."""
    import torch
    w = synth.workload_paper(n_blocks=4)
    n, _ = noise_handle(S, ctx, w)
    Hd = to_dev(w.steering_table())
    Xs = [to_dev(w.block(b)[0]) for b in range(4)]
    plan = [(Xs[0], n, 1), (Xs[1], n, 2), (Xs[2], n, 3), (Xs[3], n, 4), (Xs[0], None, 2),
            (Xs[1], n, 2)]
    for rep in range(2):
        bo = [outs(w, ns) for _, _, ns in plan]
        descs = [S.block_desc(Xd, nh, Hd, w.grid.n_az, w.grid.n_el, ns, o["pk"], o["pv"],
                              o["Pbar"], o["st"]) for (Xd, nh, ns), o in zip(plan, bo)]
        S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
        got = [{k: to_host(v) for k, v in o.items()} for o in bo]
        for i, (Xd, nh, ns) in enumerate(plan):
            ref = single(S, ctx, w, Xd, nh, Hd, ns)
            for k in ("pk", "pv", "Pbar", "st"):
                assert np.array_equal(got[i][k], ref[k]), (rep, i, k)
    S.ssl_noise_destroy(n)


def test_failed_bins_contribute_nothing(S, ctx):
    """A bin whose K is not positive definite: status NOT_PD, P = 0 there in both forms, so the
    two P-bars agree within the bar."""
    import torch
    w = synth.workload_small(n_blocks=2)
    Xn = w.noise_frames()
    K = oracle.noise_corr(Xn)
    K[5] = np.diag(np.r_[1.0, -1.0, np.ones(w.M - 2)]).astype(complex)
    n = S.ssl_noise_create(ctx, w.F, w.M)
    S.ssl_noise_set(n, to_dev(K), S.SSL_FP64)
    Hd = to_dev(w.steering_table())
    Xd = to_dev(w.block(0)[0])
    g = single(S, ctx, w, Xd, n, Hd, w.Ns)
    S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_NOISE)
    try:
        gn = single(S, ctx, w, Xd, n, Hd, w.Ns)
    finally:
        S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_SIGNAL)
    assert g["st"][5] == S.SSL_BIN_NOT_PD and np.sum(g["st"] != 0) == 1
    rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - gn["Pbar"]) / gn["Pbar"]))
    assert rel <= 1e-4
    S.ssl_noise_destroy(n)


def test_projection_mode_errors(S, ctx):
    with pytest.raises(S.SSLError) as e:
        S.ssl_ctx_set_projection(ctx, 2)
    assert e.value.code == S.SSL_ERR_ARG
    assert S.ssl_ctx_get_projection(ctx) == S.SSL_PROJ_SIGNAL


@pytest.mark.parametrize("mode", ["gsvd", "sevd"])
def test_signal_form_per_bin(S, ctx, mode):
    """P of single bins (the table zero in every other bin, so that P-bar is that bin's P) against
    the oracle's per-bin P, for both forms: a per-bin check sees what the sum over 257 bins can
    average out (a wrong conjugation of E_s^H h left P-bar within 3e-7 but single bins at 2e-4).
    Low bins, where the strongest source dominates (sigma_1 / sigma_2 up to about 370 in SEVD mode),
    and a few others."""
    import torch
    w = synth.workload_paper(n_blocks=1)
    X, _, _ = w.block(0)
    H = w.steering_table()
    if mode == "gsvd":
        n, K = noise_handle(S, ctx, w)
    else:
        n, K = None, np.broadcast_to(np.eye(w.M, dtype=np.complex128), (w.F, w.M, w.M)).copy()
    r = oracle.localize(X, K, H, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16, want_P=True)
    Xd = to_dev(X)
    worst = {}
    for f in (1, 2, 7, 35, 183, 233):
        Hm = np.zeros_like(H)
        Hm[f] = H[f]
        Hd = to_dev(Hm)
        for form in ("signal", "noise"):
            S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_SIGNAL if form == "signal" else S.SSL_PROJ_NOISE)
            try:
                g = single(S, ctx, w, Xd, n, Hd, w.Ns)
            finally:
                S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_SIGNAL)
            assert np.all(g["st"] == 0)
            rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["P"][f]) / r["P"][f]))
            worst[form] = max(worst.get(form, 0.0), rel)
            say(f"  {mode} bin {f} {form} form: P rel {rel:.2e}")
            assert rel <= 1e-4, (f, form, rel)
    say(f"  {mode}: worst per-bin P error {worst}")
    if n is not None:
        S.ssl_noise_destroy(n)


@pytest.mark.parametrize("pname", ["bf16", "fp16"])
def test_signal_form_16bit_table_per_bin(S, ctx, pname):
    """The 16-bit paths on inputs that are exact in their type (X and H rounded to bf16 / fp16 on
    the host, and the oracle given the same rounded values): the correlation's products are then
    exact and the table's pairs widen exactly to FP64, so single bins must meet the FP32 bar (1e-4
    per bin P), i.e. the 16-bit path adds no error beyond the rounding of its inputs."""
    import torch
    prec = S.SSL_BF16 if pname == "bf16" else S.SSL_FP16
    dt = torch.bfloat16 if pname == "bf16" else torch.float16
    w = synth.workload_paper(n_blocks=1)
    X, _, _ = w.block(0)
    H = w.steering_table()

    def rounded(a):
        r = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(a))).to(dt).to(torch.float64)
        return torch.view_as_complex(r.contiguous()).numpy()

    Xr = rounded(X).astype(np.complex64)          # exact: 16-bit values are FP32 values
    Hr = rounded(H).astype(np.complex64)
    assert np.all(np.isfinite(Xr.view(np.float32))) and np.all(np.isfinite(Hr.view(np.float32)))
    n, K = noise_handle(S, ctx, w)
    r = oracle.localize(Xr, K, Hr, w.grid.n_az, w.grid.n_el, w.Ns, nthreads=16, want_P=True)
    Xd = to_dev(Xr)
    worst = 0.0
    for f in (1, 7, 35, 183):
        Hm = np.zeros_like(H)
        Hm[f] = H[f]
        Hd = torch.view_as_real(to_dev(Hm)).reshape(w.F, w.D, 2 * w.M).to(dt).contiguous()
        o = outs(w, w.Ns)
        S.ssl_localize(ctx, Xd, n, Hd, prec, w.grid.n_az, w.grid.n_el, w.Ns, 2, o["pk"], o["pv"],
                       o["Pbar"], o["st"])
        g = {k: to_host(v) for k, v in o.items()}
        assert np.all(g["st"] == 0)
        rel = float(np.max(np.abs(g["Pbar"].astype(np.float64) - r["P"][f]) / r["P"][f]))
        worst = max(worst, rel)
        say(f"  {pname} table, bin {f}: P rel {rel:.2e}")
        assert rel <= 1e-4, (f, rel)
    say(f"  {pname}: worst per-bin P error {worst:.2e} (exact 16-bit inputs)")
    S.ssl_noise_destroy(n)


def test_batch_conv_statistics(S, ctx):
    """ssl_block_desc.conv: the batch's per-bin Jacobi statistics.  With the noise-vector form the
    batch runs the same solve as ssl_gsvd under SSL_STOP_ALSO_GSVD, so the counts agree bin for bin;
    with the signal form (sweeps on R~^H, no second QR) every bin reports the numerical rank of the
    pivoted QR and a sweep count within the limit."""
    import torch
    w = synth.workload_paper(n_blocks=1)
    n, _ = noise_handle(S, ctx, w)
    Hd = to_dev(w.steering_table())
    Xd = to_dev(w.block(0)[0])
    out = {}
    for form in ("noise", "signal"):
        o = outs(w, w.Ns)
        cv = torch.full((w.F, 3), -7, dtype=torch.int32, device="cuda:0")
        S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_NOISE if form == "noise" else S.SSL_PROJ_SIGNAL)
        try:
            d = S.block_desc(Xd, n, Hd, w.grid.n_az, w.grid.n_el, w.Ns, o["pk"], o["pv"], o["Pbar"],
                             o["st"], cv)
            S.ssl_localize_batch(ctx, [d], S.SSL_FP32, 2)
        finally:
            S.ssl_ctx_set_projection(ctx, S.SSL_PROJ_SIGNAL)
        out[form] = to_host(cv)
    R = torch.zeros((w.F, w.M, w.M), dtype=torch.complex64, device="cuda:0")
    S.ssl_corr_accum(ctx, Xd, 1.0 / w.T, 0, S.SSL_FP32, R)
    En = torch.zeros((w.F, w.M - w.Ns, w.M), dtype=torch.complex64, device="cuda:0")
    cg = torch.full((w.F, 3), -7, dtype=torch.int32, device="cuda:0")
    S.ssl_ctx_set_stop(ctx, S.SSL_STOP_ALSO_GSVD)
    try:
        S.ssl_gsvd(ctx, R, n, w.Ns, En, None, None, cg, 0)
    finally:
        S.ssl_ctx_set_stop(ctx, S.SSL_STOP_LOCALIZE)
    assert np.array_equal(out["noise"], to_host(cg))
    sg = out["signal"]
    say(f"  signal form: mean sweeps {sg[:, 0].mean():.2f} (noise form {out['noise'][:, 0].mean():.2f}), "
        f"ranks {np.unique(sg[:, 2])}")
    assert np.all(sg[:, 2] == out["noise"][:, 2])
    assert np.all((sg[:, 0] >= 0) & (sg[:, 0] <= 20)) and np.all(sg[:, 1] >= 0)
    S.ssl_noise_destroy(n)


def test_batch_more_blocks_than_one_descriptor_chunk(S, ctx):
    """300 blocks sharing one steering table: the projection reads the blocks' descriptors in
    chunks of 256, so the second chunk's blocks must equal their single-block calls bit for bit,
    like the first chunk's."""
    import torch
    nb = 300
    w = synth.workload_small(n_blocks=4)
    n, _ = noise_handle(S, ctx, w)
    Hd = to_dev(w.steering_table())
    Xs = [to_dev(w.block(b)[0]) for b in range(4)]
    bo = [outs(w, w.Ns) for _ in range(nb)]
    descs = [S.block_desc(Xs[b % 4], n, Hd, w.grid.n_az, w.grid.n_el, w.Ns, o["pk"], o["pv"],
                          o["Pbar"], o["st"]) for b, o in enumerate(bo)]
    S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
    refs = [single(S, ctx, w, Xs[q], n, Hd, w.Ns) for q in range(4)]
    for b in (0, 3, 255, 256, 257, 299):
        got = {k: to_host(v) for k, v in bo[b].items()}
        for k in ("pk", "pv", "Pbar", "st"):
            assert np.array_equal(got[k], refs[b % 4][k]), (b, k)
    say(f"  {nb} blocks in one steering group: chunk boundaries equal single-block calls")
    S.ssl_noise_destroy(n)
