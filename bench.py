#!/usr/bin/env python3
"""GSVD-MUSIC localization throughput on one MI355X.

Workload: blocks of the 60-channel scene (M = 60 microphones in 4 rings, F = 257 bins, T = 50
frames, D = 72 x 19 = 1368 directions, Ns = 2).  A step is one pass of the whole localization
path -- correlation (eq.2-3), A = K^{-1} R in FP64 and the Jacobi-SVD noise subspace (eq.4), MUSIC
spectrum (eq.5), bin sum (eq.6) and peak search -- over one batch of `--batch` distinct blocks via
ssl_localize_batch (all HIP kernels of the library).  Inputs (distinct seeded blocks, steering
table, resident noise factor) are in HBM before any timed region starts.

The headline path (`--prec`, default fp32) is the paper's arithmetic: correlation on FP32 MFMA,
K^{-1}R in FP64, the Jacobi SVD in FP32 and eq.5 through the signal subspace in FP64 (|h|^2 minus
the squared projection on the Ns signal vectors, FP64 MFMA).  The mixed-precision paths (bf16 and
fp16 MFMA inputs with FP32 accumulation for the correlation, a bf16 / fp16 steering table read by
the same FP64 signal-subspace projection, the rest unchanged) are measured in the same run as
secondary keys, batched and one block per call.

Timed regions per precision (each bracketed by torch.cuda.synchronize()):
  * main: `--steps` batch steps with per-kernel HIP events on the launch stream -> `value`, the
    per-kernel rooflines (algorithmic bytes or flops per launch / average launch duration);
  * graph: the same steps replayed from the captured HIP graph (no events) -> `graph_value`;
  * per-block: ssl_localize one block at a time -> `per_block`;
  * host-to-device (headline precision): the same steps with every block's X copied from pinned
    host memory, serial and double-buffered on a side stream -> `h2d`.
Serving: 64 array streams through paper_2504_03373_amd.serving, batched at the headline precision
(its p50/p99 are `latency_ms`) and at bf16, and the FP32 path one block per call for comparison.
The FP64 CPU oracle is timed on a bounded sample of the same workload on this host's cores, and
the headline step's results for those blocks are compared with it (`cpu_baseline.parity`).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # the same without packed FP32, which this build leaves off
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}


def jacobi_flops(M: int, sweeps, rotations, rank, Ns: int = 0, sub: bool = False,
                 sig: bool = False) -> float:
    """Algorithmic real flops of the SVD kernel summed over bins (rank r per bin).
    Pivoted QR: step k = 0..r-1 has trailing size n = M - k; each of the n - 1 remaining columns
    costs w = v^H x (8n), x -= v (tau w) (8n) and its trailing norm (4n): 20 n (n - 1).
    Second QR of R^H (M x r, no pivoting): step k updates r - k - 1 columns of length M - k,
    16 (M - k)(r - k - 1).  Jacobi on X (r x r): each pair visit forms |x_i|^2, |x_j|^2, x_i^H x_j
    (16 r); each applied rotation rewrites two columns (20 r); pair visits = sweeps r(r-1)/2.
    Normalisation of W: 6 r per column.  U = Q U_R: reflector k applied to the M columns,
    16 (M - k) M.
    sub: the solve stopped at the noise subspace (p = 2 localization), which switches to the
    subspace sweeps before any full one: every sweep visits the Ns (r - Ns) + Ns (Ns - 1) / 2
    pairs with a member in the signal set (a bin that fell back to full sweeps is counted the same
    way, which undercounts it); the r - Ns complement vectors each pass Ns reflectors (16 r), and
    W is not normalised.
    sig: only the Ns signal vectors are formed (eq.5 through the signal subspace): the sweeps run
    on Z = R~^H (M x r, no second QR, columns of length M: 16M per pair visit, 20M per rotation),
    the signal vectors are A w_s (8 M^2 Ns), and neither the complement nor the back-transformation
    runs."""
    import numpy as np
    total = 0.0
    for s, rot, r in zip(np.asarray(sweeps), np.asarray(rotations), np.asarray(rank)):
        r = int(r)
        k = np.arange(r, dtype=np.float64)
        n = M - k
        if sig:
            visits = float(s) * (Ns * (r - Ns) + Ns * (Ns - 1) / 2.0) if sub and r > Ns \
                else float(s) * r * (r - 1) / 2.0
            total += float(np.sum(20.0 * n * (n - 1))) + visits * 16.0 * M + \
                float(rot) * 20.0 * M + 8.0 * M * M * Ns
            continue
        total += float(np.sum(20.0 * n * (n - 1)) + np.sum(16.0 * n * (r - k - 1))
                       + np.sum(16.0 * n * M))
        if sub and r > Ns:
            visits = float(s) * (Ns * (r - Ns) + Ns * (Ns - 1) / 2.0)
            total += visits * 16.0 * r + float(rot) * 20.0 * r + (r - Ns) * Ns * 16.0 * r
        else:
            total += float(s) * r * (r - 1) / 2.0 * 16.0 * r + float(rot) * 20.0 * r + 6.0 * r * r
    return total


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jacobi_persistent_60ch_257bin_hbm_traffic.json")
JACOBI_SRC = os.path.join(ROOT, "paper_2504_03373_amd", "csrc", "jacobi.hip")


def _sha256(path: str) -> str:
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_bytes(batch: int):
    """HBM bytes per Jacobi launch from the committed counter summary, or None when it is absent,
    was taken at another batch size, or the kernel source has changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != _sha256(JACOBI_SRC) or t.get("blocks_per_launch") != batch:
        return None
    return t.get("bytes_per_launch")


def _pmc_rows(d: str, counter: str):
    """(kernel name, value) per dispatch from a rocprofv3 --pmc csv output directory."""
    import csv
    import glob
    rows = []
    for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {d}")
    return rows


def pmc_summarize(fetch_dir: str, write_dir: str, calib_mb: int, batch: int) -> int:
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of jacobi_persistent, each scaled by what the
    same counter reads for the calibration kernel (calib_mb MiB read and written once)."""
    import numpy as np
    if calib_mb <= 0:
        raise SystemExit("--calib-copy-mb is needed to scale the counters")
    calib = calib_mb * (1 << 20)
    out = {"kernel": "jacobi_persistent", "blocks_per_launch": batch,
           "source_sha256": _sha256(JACOBI_SRC), "calibration_bytes": calib}
    total = 0.0
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _pmc_rows(d, name)
        cal = [v for k, v in rows if "neg" in k.lower()]
        # the variant the timed steps ran: the most frequent one (the autotuner also launches the
        # others a few times)
        names = [k for k, _ in rows if "jacobi_persistent" in k]
        top = max(set(names), key=names.count) if names else None
        jac = [v for k, v in rows if k == top]
        if not cal or not jac:
            raise SystemExit(f"{name}: calibration or Jacobi dispatches missing in {d}")
        scale = calib / (max(cal) * 1024.0)
        per_launch = float(np.median(jac)) * 1024.0 * scale
        out[name.lower()] = {"kib_per_dispatch_median": float(np.median(jac)),
                             "dispatches": len(jac), "calibration_kib": max(cal),
                             "scale": scale, "bytes_per_launch": per_launch}
        total += per_launch
    out["bytes_per_launch"] = total
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
    return 0


def serving_phase(args, variants: dict) -> dict:
    """Serving: `--serve-streams` array streams through paper_2504_03373_amd.serving, batched at
    the headline precision (the configured load and the light one) and at bf16 (the configured
    load), then the FP32 path one block per call; the kernel variants tuned for the 60-channel
    class (`variants`) are applied to the serving contexts."""
    import torch

    import paper_2504_03373_amd as S
    import synth
    from paper_2504_03373_amd.serving import GpuExecutor, Server
    dev = "cuda:0"
    S.lib()
    PREC = {"fp32": S.SSL_FP32, "bf16": S.SSL_BF16, "fp16": S.SSL_FP16}
    streams = synth.serving_streams(n_streams=args.serve_streams)
    H32 = {}
    for s_ in streams:
        if s_.M not in H32:
            H32[s_.M] = torch.from_numpy(synth.steering_table(s_.pos, s_.grid, s_.freqs)).to(dev)

    def tables(prec):
        if prec == S.SSL_FP32:
            return H32
        dt = torch.bfloat16 if prec == S.SSL_BF16 else torch.float16
        return {M: torch.view_as_real(h).reshape(h.shape[0], h.shape[1], 2 * M).to(dt).contiguous()
                for M, h in H32.items()}

    budget = int(args.serve_budget_gb * (1 << 30))
    M, Ns = variants["M"], variants["Ns"]
    mix = {m: sum(1 for s_ in streams if s_.M == m) for m in sorted({s_.M for s_ in streams})}

    def executor(pname, lanes=None):
        prec = PREC[pname]

        def configure(c):
            if variants.get("jacobi_lanes"):
                S.ssl_ctx_set_jacobi_lanes(c, M, variants["jacobi_lanes"])
            w_ = (variants.get("steer_waves") or {}).get(pname)
            if w_:
                S.ssl_ctx_set_steer_waves(c, M, Ns, prec, w_)

        return GpuExecutor(streams, tables(prec), prec=prec, alpha=0.95,
                           k_update_every=args.k_update_every, hbm_budget_bytes=budget,
                           lanes=args.serve_lanes if lanes is None else lanes, pool=4,
                           configure=configure, k_lag=args.k_lag)

    def serve(srv, ex, pname, period_ms: float, seconds: float) -> dict:
        arrivals = synth.poisson_arrivals(len(streams), seconds, period_ms * 1e-3)
        sv = srv.run(arrivals)
        return {"streams": len(streams), "streams_by_M": mix, "period_ms": period_ms,
                "prec": pname, "offered_blocks_per_s": round(len(arrivals) / seconds, 1),
                "completed": sv["completed"], "blocks_per_s": round(sv["blocks_per_s"], 1),
                "p50_ms": round(sv["p50_ms"], 3), "p99_ms": round(sv["p99_ms"], 3),
                "max_ms": round(sv["max_ms"], 3), "mean_batch": round(sv["mean_batch"], 2),
                "max_queue": sv["max_queue"], "k_update_every": args.k_update_every,
                "k_lag": args.k_lag, "stream_depth": ex.stream_depth,
                "hbm_budget_gb": args.serve_budget_gb, "emitted_seconds": seconds,
                "lanes": ex.lanes, "process": "in-process" if args.serve_inproc else
                "child process",
                "host_s": {k: round(sv[k], 3) for k in ("loop_s", "submit_s", "collect_s",
                                                        "sleep_s")}}

    out = {}
    legs = [(args.prec, "serving", True)]
    if args.serve_mixed and args.serve_mixed != args.prec:
        legs.append((args.serve_mixed, f"serving_{args.serve_mixed}", False))
    for pname, key, headline in legs:
        ex = executor(pname)
        srv = Server(ex, budget, max_batch=128)
        srv.run(synth.poisson_arrivals(len(streams), 0.1, args.serve_period_ms * 1e-3, seed=7))
        out[key] = serve(srv, ex, pname, args.serve_period_ms, args.serve_seconds)
        if headline and args.serve_light_period_ms > 0:
            out["serving_light"] = serve(srv, ex, pname, args.serve_light_period_ms,
                                         args.serve_seconds)
        ex.close()
        del ex, srv
        torch.cuda.synchronize()
    if args.serve_fp32_seconds > 0:
        # the plain FP32 path served one block per call (one lane, batches of one block), same
        # streams and load, a shorter emission window: its capacity is far below the load
        ex1 = executor("fp32", lanes=1)
        srv1 = Server(ex1, budget, max_batch=1)
        srv1.run(synth.poisson_arrivals(len(streams), 0.05, args.serve_period_ms * 1e-3, seed=7))
        arrivals = synth.poisson_arrivals(len(streams), args.serve_fp32_seconds,
                                          args.serve_period_ms * 1e-3)
        sv = srv1.run(arrivals)
        ex1.close()
        out["serving_fp32_per_block"] = {
            "period_ms": args.serve_period_ms, "prec": "fp32", "lanes": 1, "max_batch": 1,
            "offered_blocks_per_s": round(len(arrivals) / args.serve_fp32_seconds, 1),
            "completed": sv["completed"], "blocks_per_s": round(sv["blocks_per_s"], 1),
            "p50_ms": round(sv["p50_ms"], 3), "p99_ms": round(sv["p99_ms"], 3),
            "emitted_seconds": args.serve_fp32_seconds,
            "kind": "same streams and load; FP32 MFMA inputs, one block per batch on one lane"}
    out["latency_ms"] = {"p50": out["serving"]["p50_ms"], "p99": out["serving"]["p99_ms"],
                         "prec": args.prec, "kind": "served, batched: emission to peaks on the host"}
    return out


def uneven_phase(args) -> dict:
    """The uneven batch: `--uneven-blocks` blocks with M in {8, 16, 32, 60}, F in {257, 513} and
    Ns in {1, 2, 3} (uniform, seeded), all in one ssl_localize_batch call per step (persistent
    Jacobi launch, graph replay after the first call), every block its own device copy of X.
    Kernel variants are autotuned per channel class on this mix (F = 257, Ns = 2 blocks)."""
    import torch

    import paper_2504_03373_amd as S
    import synth
    dev = "cuda:0"
    PREC = {"fp32": S.SSL_FP32, "bf16": S.SSL_BF16, "fp16": S.SSL_FP16}
    prec = PREC[args.prec]
    shapes = synth.uneven_shapes(args.uneven_blocks)
    ctx = S.ssl_ctx_create(0, 0)
    geo, pool = {}, {}
    t0 = time.time()
    for M, F, Ns in sorted(set(shapes)):
        if (M, F) not in geo:
            w = synth.workload_paper(n_blocks=2, seed=3000 + 10 * M + F, M=M, F=F)
            Xn = torch.from_numpy(w.noise_frames()).to(dev)
            K = torch.zeros((F, M, M), dtype=torch.complex128, device=dev)
            S.ssl_corr_accum(ctx, Xn, 1.0 / Xn.shape[1], 0, S.SSL_FP64, K)
            n = S.ssl_noise_create(ctx, F, M)
            S.ssl_noise_set(n, K, S.SSL_FP64)
            H = torch.from_numpy(w.steering_table()).to(dev)
            if prec != S.SSL_FP32:
                H = torch.view_as_real(H).reshape(F, w.D, 2 * M).to(
                    torch.bfloat16 if prec == S.SSL_BF16 else torch.float16).contiguous()
            geo[(M, F)] = dict(noise=n, H=H, D=w.D, grid=w.grid)
        wk = synth.workload_paper(n_blocks=2, seed=3100 + 10 * M + F + Ns, M=M, F=F, Ns=Ns)
        pool[(M, F, Ns)] = [wk.block(q)[0] for q in range(2)]
    gen_s = time.time() - t0
    tuned = {}
    if not args.no_autotune:
        for M in (8, 16, 32, 60):
            g = geo.get((M, 257))
            if g is None or (M, 257, 2) not in pool:
                continue
            X = torch.from_numpy(pool[(M, 257, 2)][0]).to(dev)
            R = torch.zeros((257, M, M), dtype=torch.complex64, device=dev)
            En = torch.zeros((257, M - 2, M), dtype=torch.complex64, device=dev)
            S.ssl_corr_accum(ctx, X, 1.0 / X.shape[1], 0, prec, R)
            S.ssl_gsvd(ctx, R, g["noise"], 2, En, None, None, None, 0)
            lanes, _ = S.ssl_autotune_jacobi(ctx, R, g["noise"], 2, nblocks=32, reps=2)
            waves, _ = S.ssl_autotune_steer(ctx, g["H"], prec, En, 2, p=2, nblocks=32, reps=2)
            tuned[str(M)] = {"jacobi_lanes": lanes, "steer_waves": waves}
    descs, outs = [], []
    for i, (M, F, Ns) in enumerate(shapes):
        g = geo[(M, F)]
        X = torch.from_numpy(pool[(M, F, Ns)][i % 2]).to(dev)
        o = (torch.zeros(Ns, dtype=torch.int32, device=dev),
             torch.zeros(Ns, dtype=torch.float32, device=dev),
             torch.zeros(g["D"], dtype=torch.float32, device=dev),
             torch.zeros(F, dtype=torch.int32, device=dev), X)
        outs.append(o)
        descs.append(S.block_desc(X, g["noise"], g["H"], g["grid"].n_az, g["grid"].n_el, Ns,
                                  o[0], o[1], o[2], o[3]))
    for _ in range(2):                       # the first call captures the graph
        S.ssl_localize_batch(ctx, descs, prec, 2)
    torch.cuda.synchronize()
    tt = time.perf_counter()
    for _ in range(args.uneven_steps):
        S.ssl_localize_batch(ctx, descs, prec, 2)
    torch.cuda.synchronize()
    el = time.perf_counter() - tt
    bins = sum(F for _, F, _ in shapes)
    ok = all(bool((o[3] == S.SSL_BIN_OK).all()) for o in outs)
    for g in geo.values():
        S.ssl_noise_destroy(g["noise"])
    S.ssl_ctx_destroy(ctx)
    mix = {f"M{m}": sum(1 for s_ in shapes if s_[0] == m) for m in (8, 16, 32, 60)}
    return {"blocks": len(shapes), "bins": bins, "value": round(len(shapes) * args.uneven_steps / el, 1),
            "unit": "blocks/s", "bins_per_s": round(bins * args.uneven_steps / el, 1),
            "ms_per_step": round(1e3 * el / args.uneven_steps, 3), "steps": args.uneven_steps,
            "prec": args.prec, "blocks_by_M": mix,
            "blocks_F513": sum(1 for s_ in shapes if s_[1] == 513),
            "tuned": tuned or "defaults", "status_ok": ok, "input_gen_s": round(gen_s, 2),
            "kind": "one ssl_localize_batch per step over all blocks (persistent Jacobi, graph "
                    "replay), M in {8,16,32,60}, F in {257,513}, Ns in {1,2,3}"}


def _timed_batch_steps(S, ctx, w, noise, H32, Xs, steps: int):
    """FP32 batch steps over the bench's blocks: one untimed call (captures the launch sequence),
    then `steps` timed ones; returns (seconds, per-kernel (launches, ms), statuses all OK)."""
    import torch
    dev = "cuda:0"
    B, F, Ns, D = Xs.shape[0], w.F, w.Ns, w.D
    pk = torch.zeros((B, Ns), dtype=torch.int32, device=dev)
    pv = torch.zeros((B, Ns), dtype=torch.float32, device=dev)
    pb = torch.zeros((B, D), dtype=torch.float32, device=dev)
    st = torch.full((B, F), -7, dtype=torch.int32, device=dev)
    descs = [S.block_desc(Xs[b], noise, H32, w.grid.n_az, w.grid.n_el, Ns, pk[b], pv[b], pb[b],
                          st[b]) for b in range(B)]
    S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
    torch.cuda.synchronize()
    S.ssl_ctx_timing_read(ctx, reset=True)
    S.ssl_ctx_timing(ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        S.ssl_localize_batch(ctx, descs, S.SSL_FP32, 2)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.ssl_ctx_timing(ctx, False)
    kt = S.ssl_ctx_timing_read(ctx, reset=True)
    return el, kt, bool((st.cpu() == 0).all())


def bidiag_phase(args, S, ctx, w, noise, H32, Xs) -> dict:
    """The same FP32 batch step with the paper's own SVD (Householder bidiagonalisation + implicit
    QR) in place of the Jacobi backend: blocks/s and the SVD kernel's average time."""
    B = Xs.shape[0]
    S.ssl_ctx_set_svd(ctx, S.SSL_SVD_BIDIAG_QR)
    try:
        el, kt, ok = _timed_batch_steps(S, ctx, w, noise, H32, Xs, args.bidiag_steps)
    finally:
        S.ssl_ctx_set_svd(ctx, S.SSL_SVD_JACOBI)
    n, ms = kt["jacobi"]
    return {"value": round(args.bidiag_steps * B / el, 2), "unit": "blocks/s", "prec": "fp32",
            "svd_avg_ms": round(ms / max(n, 1), 4), "blocks_per_step": B, "status_ok": ok,
            "kind": "FP32 batch step with the Householder-bidiagonalisation + implicit-QR SVD "
                    "(one workgroup per bin, per-event timing)"}


def gevd_phase(args, S, ctx, w, Kd, H32, Xs) -> dict:
    """The same FP32 batch step in GEVD-MUSIC mode (C = K^{-1/2} R K^{-1/2} in FP64, the Jacobi SVD
    of C, E_n = K^{-1/2} Y_n): blocks/s, the two FP64 products' and the SVD's average times, and
    the one-off K^{-1/2} time of the noise handle."""
    import torch
    B, F, M = Xs.shape[0], w.F, w.M
    noise = S.ssl_noise_create(ctx, F, M)
    S.ssl_noise_set(noise, Kd, S.SSL_FP64)
    torch.cuda.synchronize()
    S.ssl_ctx_timing_read(ctx, reset=True)
    S.ssl_ctx_timing(ctx, True)
    S.ssl_noise_enable_gevd(noise)
    torch.cuda.synchronize()
    S.ssl_ctx_timing(ctx, False)
    isq_n, isq_ms = S.ssl_ctx_timing_read(ctx, reset=True)["noise"]
    S.ssl_ctx_set_subspace(ctx, S.SSL_SUBSPACE_GEVD)
    try:
        el, kt, ok = _timed_batch_steps(S, ctx, w, noise, H32, Xs, args.gevd_steps)
    finally:
        S.ssl_ctx_set_subspace(ctx, S.SSL_SUBSPACE_GSVD)
        S.ssl_noise_destroy(noise)
    avg = lambda k: round(kt[k][1] / max(kt[k][0], 1), 4)
    return {"value": round(args.gevd_steps * B / el, 2), "unit": "blocks/s", "prec": "fp32",
            "gevd_products_ms_per_step": round(kt["whiten"][1] / args.gevd_steps, 4),
            "svd_avg_ms": avg("jacobi"),
            "noise_isqrt_ms": round(isq_ms, 4), "blocks_per_step": B, "status_ok": ok,
            "kind": "FP32 batch step in GEVD-MUSIC mode (FP64 K^{-1/2} R K^{-1/2} and K^{-1/2} Y_n "
                    "products, one workgroup per bin; per-event timing)"}


def streaming_phase(args, S, ctx, w, noise, H32, Xs) -> dict:
    """One 60-channel stream localized at frame rate (eq.3: the window of the T frames ending at
    each new frame): per frame, push the frame (rank-2 FP64 update of the window sum) and run the
    whole method on the window, FP32 path; warm-started Jacobi (from the previous frame's singular
    vectors) and cold solves, device time per frame with events on the launch stream."""
    import numpy as np
    import torch
    dev = "cuda:0"
    F, T, M, Ns, D = w.F, w.T, w.M, w.Ns, w.D
    frames = torch.cat([Xs[0], Xs[1]], dim=1).contiguous()          # [F][2T][M]
    n = min(args.stream_frames, frames.shape[1] - T)
    pk = torch.zeros(Ns, dtype=torch.int32, device=dev)
    pv = torch.zeros(Ns, dtype=torch.float32, device=dev)
    bst = torch.zeros(F, dtype=torch.int32, device=dev)
    conv = torch.zeros((F, 3), dtype=torch.int32, device=dev)
    res = {"M": M, "F": F, "T": T, "D": D, "frames": n, "prec": "fp32",
           "kind": "one stream, one frame per step: push (rank-2 FP64 window update) + "
                   "localization of the window; device time per frame"}
    for warm in (1, 0):
        s = S.ssl_sliding_create(ctx, F, M, T)
        S.ssl_sliding_push(s, frames[:, :T, :])
        S.ssl_sliding_localize(s, noise, H32, S.SSL_FP32, w.grid.n_az, w.grid.n_el, Ns, 2, 0, pk,
                               pv, None, bst, conv)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n)]
        sweeps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n):
            ev[k][0].record()
            S.ssl_sliding_push(s, frames[:, T + k:T + k + 1, :])
            S.ssl_sliding_localize(s, noise, H32, S.SSL_FP32, w.grid.n_az, w.grid.n_el, Ns, 2,
                                   warm, pk, pv, None, bst, conv)
            ev[k][1].record()
            sweeps.append(conv[:, 0].clone())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        ok = bool((bst.cpu().numpy() == 0).all())
        sw = float(torch.stack(sweeps).float().mean().item())
        res["warm" if warm else "cold"] = {
            "frames_per_s": round(n / wall, 1), "p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4), "mean_sweeps": round(sw, 3),
            "status_ok": ok}
        S.ssl_sliding_destroy(s)
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed batch steps")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=128, help="blocks per step")
    ap.add_argument("--prec", choices=["fp32", "bf16", "fp16"], default="fp32",
                    help="MFMA input type of the headline path")
    ap.add_argument("--compare", default="bf16,fp16",
                    help="comma-separated secondary MFMA input types measured in the same run "
                         "('' = none)")
    ap.add_argument("--no-h2d", action="store_true",
                    help="skip the host-to-device region (its copies share the CUs)")
    ap.add_argument("--per-block-steps", type=int, default=100)
    ap.add_argument("--cpu-blocks", type=int, default=48, help="oracle sample size (blocks)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel variants (no Jacobi / projection autotuning)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one plain streaming kernel of this size first (HBM counter scale)")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "this script with --calib-copy-mb into the traffic summary under profiles/")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="duration of emitted traffic in the serving phase (0 = skip)")
    ap.add_argument("--serve-streams", type=int, default=64)
    ap.add_argument("--serve-period-ms", type=float, default=10.0, help="mean block period per stream")
    ap.add_argument("--serve-light-period-ms", type=float, default=30.0,
                    help="a second, lighter serving load (0 = skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=4.0, help="HBM budget of in-flight work")
    ap.add_argument("--serve-lanes", type=int, default=2,
                    help="batches in flight at once (library context + HIP stream each)")
    ap.add_argument("--k-update-every", type=int, default=1)
    ap.add_argument("--k-lag", type=int, default=1, choices=[0, 1],
                    help="serving: block n reads the K of blocks <= n - 1 - k_lag")
    ap.add_argument("--uneven-blocks", type=int, default=512,
                    help="blocks of the uneven-shape batch (0 = skip)")
    ap.add_argument("--uneven-steps", type=int, default=5)
    ap.add_argument("--bidiag-steps", type=int, default=3,
                    help="batch steps timed with the bidiagonal-QR SVD backend, 0 = skip")
    ap.add_argument("--gevd-steps", type=int, default=5,
                    help="batch steps timed in GEVD-MUSIC mode, 0 = skip")
    ap.add_argument("--stream-frames", type=int, default=50,
                    help="frame-rate localizations of one 60-channel stream (eq.3 window), 0 = skip")
    ap.add_argument("--serve-mixed", default="bf16",
                    help="a second batched serving leg at this MFMA input type ('' = skip)")
    ap.add_argument("--serve-fp32-seconds", type=float, default=1.0,
                    help="emission window of the FP32 one-block-per-call serving comparison (0 = skip)")
    ap.add_argument("--serve-inproc", action="store_true",
                    help="run the serving phase in this process instead of a fresh child")
    ap.add_argument("--serve-child", metavar="VARIANTS_JSON", default=None,
                    help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.serve_child is not None:
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 1
        print(json.dumps(serving_phase(args, json.loads(args.serve_child))), flush=True)
        return 0

    if args.pmc_summarize:
        return pmc_summarize(args.pmc_summarize[0], args.pmc_summarize[1], args.calib_copy_mb,
                             args.batch)
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the localization path shards by stream/block with no "
              f"collective, so --gpus {args.gpus} is not run here", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2504_03373_amd as S
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = "cuda:0"
    S.lib()
    PREC = {"fp32": S.SSL_FP32, "bf16": S.SSL_BF16, "fp16": S.SSL_FP16}

    w = synth.workload_paper(n_blocks=1000)
    F, T, M, Ns, D = w.F, w.T, w.M, w.Ns, w.D
    B = args.batch
    t0 = time.time()
    Xs = torch.stack([torch.from_numpy(w.block(b)[0]) for b in range(B)]).to(dev)
    H32 = torch.from_numpy(w.steering_table()).to(dev)

    def table(name):
        if name == "fp32":
            return H32
        # interleaved (re, im) 16-bit pairs, [F][D][2M]
        return torch.view_as_real(H32).reshape(F, D, 2 * M).to(
            torch.bfloat16 if name == "bf16" else torch.float16).contiguous()

    Xn = torch.from_numpy(w.noise_frames()).to(dev)
    gen_s = time.time() - t0

    if args.calib_copy_mb > 0:
        # one plain streaming kernel of known traffic (reads and writes calib MiB once each): the
        # scale of the HBM counters (FETCH_SIZE / WRITE_SIZE) in the same profiled run
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    ctx = S.ssl_ctx_create(0, 0)
    Kd = torch.zeros((F, M, M), dtype=torch.complex128, device=dev)
    S.ssl_corr_accum(ctx, Xn, 1.0 / Xn.shape[1], 0, S.SSL_FP64, Kd)
    noise = S.ssl_noise_create(ctx, F, M)
    kst = torch.zeros(F, dtype=torch.int32, device=dev)
    S.ssl_noise_set(noise, Kd, S.SSL_FP64, kst)

    pk = torch.zeros((B, Ns), dtype=torch.int32, device=dev)
    pv = torch.zeros((B, Ns), dtype=torch.float32, device=dev)
    Pbar = torch.zeros((B, D), dtype=torch.float32, device=dev)
    st = torch.zeros((B, F), dtype=torch.int32, device=dev)

    tuning = {}

    def measure(name: str, with_h2d: bool, conv: bool = True) -> dict:
        prec = PREC[name]
        H = table(name)
        # Ns <= 3: eq.5 through the signal subspace (the library's default projection, any table
        # precision)
        sig = 1 <= Ns <= 3
        R = torch.zeros((F, M, M), dtype=torch.complex64, device=dev)
        En = torch.zeros((F, M - Ns, M), dtype=torch.complex64, device=dev)
        conv_t = torch.zeros((F, 3), dtype=torch.int32, device=dev)
        if not args.no_autotune:
            S.ssl_corr_accum(ctx, Xs[0], 1.0 / T, 0, prec, R)
            S.ssl_gsvd(ctx, R, noise, Ns, En, None, None, conv_t, 0)
            # variants chosen on this workload, each timed in the batched form the step runs: the
            # Jacobi lanes per column pair (once; the SVD is FP32 whatever the input precision)
            # and the projection tile for this precision, B blocks sharing the steering table
            if "jacobi_lanes" not in tuning:
                lanes, jms = S.ssl_autotune_jacobi(ctx, R, noise, Ns, nblocks=B, reps=2)
                tuning["jacobi_lanes"] = lanes
                tuning["jacobi_ms"] = {str(k): round(v, 4) for k, v in jms.items()}
            if not sig:                  # the signal-subspace projection has no tile variants
                waves, sms = S.ssl_autotune_steer(ctx, H, prec, En, Ns, p=2, nblocks=B, reps=3)
                tuning.setdefault("steer_waves", {})[name] = waves
                tuning.setdefault("steer_ms", {})[name] = {str(k): round(v, 4)
                                                           for k, v in sms.items()}
        del R, En
        # Jacobi sweep / rotation counts for the flop model, from one untimed batch step with the
        # per-bin statistics requested (same kernels, same inputs, deterministic: the counts of
        # the timed launches)
        conv_all = []
        if conv:
            cv = torch.zeros((B, F, 3), dtype=torch.int32, device=dev)
            cdescs = [S.block_desc(Xs[b], noise, H, w.grid.n_az, w.grid.n_el, Ns, pk[b], pv[b],
                                   Pbar[b], st[b], cv[b]) for b in range(B)]
            S.ssl_localize_batch(ctx, cdescs, prec, 2)
            conv_all = list(cv.cpu().numpy())
            del cv, cdescs
        jflops = float(sum(jacobi_flops(M, c[:, 0], c[:, 1], c[:, 2], Ns, True, sig)
                           for c in conv_all))
        descs = [S.block_desc(Xs[b], noise, H, w.grid.n_az, w.grid.n_el, Ns, pk[b], pv[b],
                              Pbar[b], st[b]) for b in range(B)]

        def step():
            S.ssl_localize_batch(ctx, descs, prec, 2)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # main timed region: per-kernel events on the launch stream
        S.ssl_ctx_timing_read(ctx, reset=True)
        S.ssl_ctx_timing(ctx, True)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.steps):
            ev[k][0].record()
            step()
            ev[k][1].record()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        S.ssl_ctx_timing(ctx, False)
        kt = S.ssl_ctx_timing_read(ctx, reset=True)
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        status_ok = bool((st.cpu().numpy() == 0).all())
        # graph replay region
        step()                                   # capture (not timed)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        graph_value = args.steps * B / (time.perf_counter() - tg)
        # one block per call
        pk1 = torch.zeros(Ns, dtype=torch.int32, device=dev)
        pv1 = torch.zeros(Ns, dtype=torch.float32, device=dev)
        pb1 = torch.zeros(D, dtype=torch.float32, device=dev)
        st1 = torch.zeros(F, dtype=torch.int32, device=dev)

        def one(k):
            S.ssl_localize(ctx, Xs[k % B], noise, H, prec, w.grid.n_az, w.grid.n_el, Ns, 2, pk1,
                           pv1, pb1, st1)

        for k in range(5):
            one(k)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for k in range(args.per_block_steps):
            one(k)
        torch.cuda.synchronize()
        per_block = args.per_block_steps / (time.perf_counter() - tb)

        avg = {k: ms / max(n, 1) for k, (n, ms) in kt.items() if n}
        ms = lambda k: avg[k] * 1e-3
        # algorithmic work per launch (B blocks): bytes or flops the method must move or compute
        sH = 8 if name == "fp32" else 4
        w_corr = B * (8.0 * F * T * M + 8.0 * F * M * M)
        w_white = B * 8.0 * F * M ** 3
        # projection: |E_n^H h|^2 (M - Ns noise vectors, MFMA at the table's precision), or
        # through the signal subspace |E_s^H h|^2 (Ns vectors, FP64 MFMA)
        w_steer = B * 8.0 * F * D * M * (Ns if sig else M - Ns)
        w_bins = B * (4.0 * F * D + 4.0 * D)
        rl = {
            "corr": {"bound": "hbm", "unit": "GB/s", "bytes_per_launch": w_corr,
                     "achieved": w_corr / ms("corr") / 1e9, "peak": PEAK_HBM_GBS},
            "whiten": {"bound": "mfma", "mfma_dtype": "f64", "unit": "TFLOP/s",
                       "flops_per_launch": w_white,
                       "achieved": w_white / ms("whiten") / 1e12, "peak": PEAK_FP64_TFLOPS},
            "jacobi": {"bound": "alu", "unit": "TFLOP/s", "flops_per_launch": jflops,
                       "achieved": jflops / ms("jacobi") / 1e12, "peak": PEAK_FP32_VECTOR_TFLOPS},
            "steer": {"bound": "mfma", "mfma_dtype": "f64" if sig else name, "unit": "TFLOP/s",
                      "flops_per_launch": w_steer,
                      "achieved": w_steer / ms("steer") / 1e12,
                      "peak": PEAK_FP64_TFLOPS if sig else PEAK_MFMA_TFLOPS[name],
                      "form": "signal subspace" if sig else "noise vectors",
                      "table_bytes_per_element": sH},
            "binsum": {"bound": "hbm", "unit": "GB/s", "bytes_per_launch": w_bins,
                       "achieved": w_bins / ms("binsum") / 1e9, "peak": PEAK_HBM_GBS},
        }
        for v in rl.values():
            v["frac"] = round(v["achieved"] / v["peak"], 4)
            v["achieved"] = round(v["achieved"], 3)
        out = {"value": args.steps * B / elapsed, "elapsed": elapsed, "graph_value": graph_value,
               "per_block": per_block, "lat": lat, "kt": kt, "avg": avg, "rl": rl,
               "jflops": jflops, "conv": conv_all, "status_ok": status_ok}
        if with_h2d:
            # X of every block from pinned host memory: (a) copy then compute on one stream;
            # (b) double-buffered, the copy of step k+1 on a side stream under step k
            Xh = Xs.cpu().pin_memory()
            Xs2 = torch.empty_like(Xs)
            descs2 = [S.block_desc(Xs2[b], noise, H, w.grid.n_az, w.grid.n_el, Ns, pk[b], pv[b],
                                   Pbar[b], st[b]) for b in range(B)]
            main_st = torch.cuda.current_stream()
            torch.cuda.synchronize()
            th = time.perf_counter()
            for _ in range(args.steps):
                Xs.copy_(Xh, non_blocking=True)
                step()
            torch.cuda.synchronize()
            out["h2d_serial"] = args.steps * B / (time.perf_counter() - th)
            cs = torch.cuda.Stream(device=dev)
            bufs, bdescs = (Xs, Xs2), (descs, descs2)
            copied = [torch.cuda.Event(), torch.cuda.Event()]
            freed = [torch.cuda.Event(), torch.cuda.Event()]
            for i in range(2):
                S.ssl_localize_batch(ctx, bdescs[i], prec, 2)   # both captured (not timed)
            torch.cuda.synchronize()
            th = time.perf_counter()
            with torch.cuda.stream(cs):
                bufs[0].copy_(Xh, non_blocking=True)
                copied[0].record(cs)
            for k in range(args.steps):
                i = k & 1
                if k + 1 < args.steps:
                    with torch.cuda.stream(cs):
                        if k >= 1:
                            cs.wait_event(freed[1 - i])
                        bufs[1 - i].copy_(Xh, non_blocking=True)
                        copied[1 - i].record(cs)
                main_st.wait_event(copied[i])
                S.ssl_localize_batch(ctx, bdescs[i], prec, 2)
                freed[i].record(main_st)
            torch.cuda.synchronize()
            out["h2d_overlap"] = args.steps * B / (time.perf_counter() - th)
            # hand the pinned staging copy back to the system: kept in torch's pinned-memory
            # cache, it slowed the serving phase's own pinned uploads (about 6200 -> 5000 served
            # blocks/s at the 10 ms load)
            del Xh, Xs2, descs2, bufs, bdescs
            torch._C._host_emptyCache()
        return out

    main_r = measure(args.prec, with_h2d=not args.no_h2d)
    # the headline step's outputs, kept for the comparison with the oracle below
    head_pk, head_pv, head_pbar = pk.cpu().numpy(), pv.cpu().numpy(), Pbar.cpu().numpy()
    compare = [c for c in args.compare.split(",") if c and c != args.prec]
    sec = {c: measure(c, with_h2d=False, conv=False) for c in compare}
    f32 = main_r if args.prec == "fp32" else sec.get("fp32")

    avg = main_r["avg"]
    roofline = {"kernel": "jacobi_persistent", **{k: main_r["rl"]["jacobi"][k] for k in
                                                   ("bound", "achieved", "peak", "unit", "frac")},
                "frac_unpacked": round(main_r["rl"]["jacobi"]["achieved"] / PEAK_FP32_UNPACKED_TFLOPS, 4),
                "traffic": traffic_bytes(B), "avg_launch_ms": round(avg["jacobi"], 4),
                "flops_per_launch": main_r["jflops"], "bins_per_launch": B * F}
    conv_all = main_r["conv"]
    out = {
        "metric": "GSVD-MUSIC blocks/s (60ch, 257 bins, 1368 dirs) + p50/p99 served latency",
        "value": round(main_r["value"], 2),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * main_r["elapsed"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": w.name, "M": M, "F": F, "T": T, "D": D, "Ns": Ns, "p": 2,
                   "blocks_per_step": B, "path": "ssl_localize_batch",
                   "mfma_inputs": args.prec, "whitening": "fp64",
                   "svd": "fp32 one-sided Jacobi (two-QR preconditioned), stopped at the "
                          "signal / noise split",
                   "projection": ("eq.5 through the signal subspace, FP64 MFMA"
                                  if Ns <= 3 else
                                  f"eq.5 over the noise vectors, {args.prec} MFMA")},
        "graph_value": round(main_r["graph_value"], 2),
        "per_block": {"value": round(main_r["per_block"], 2), "unit": "blocks/s",
                      "path": f"ssl_localize, one block per call, {args.prec}"},
        "step_ms": {"p50": round(float(np.percentile(main_r["lat"], 50)), 4),
                    "p99": round(float(np.percentile(main_r["lat"], 99)), 4),
                    "kind": f"device time of one {B}-block step"},
        "dominant_kernel": max(avg, key=lambda k: avg[k]),
        "kernels": {k: {"launches": n, "avg_ms": round(ms / max(n, 1), 4)}
                    for k, (n, ms) in main_r["kt"].items() if n},
        "roofline": roofline,
        "kernel_rooflines": main_r["rl"],
        "jacobi_sweeps": {"mean": round(float(np.mean([c[:, 0].mean() for c in conv_all])), 3),
                          "max": int(max(c[:, 0].max() for c in conv_all)),
                          "mean_rank": round(float(np.mean([c[:, 2].mean() for c in conv_all])), 2)},
        "status_ok": main_r["status_ok"] and all(r["status_ok"] for r in sec.values()),
        "input_gen_s": round(gen_s, 2),
        "tuning": tuning or "defaults (--no-autotune)",
    }
    if args.uneven_blocks > 0:
        out["uneven"] = uneven_phase(args)
    if args.stream_frames > 0:
        out["streaming"] = streaming_phase(args, S, ctx, w, noise, H32, Xs)
    if args.bidiag_steps > 0:
        out["svd_bidiag_qr"] = bidiag_phase(args, S, ctx, w, noise, H32, Xs)
    if args.gevd_steps > 0:
        out["gevd_music"] = gevd_phase(args, S, ctx, w, Kd, H32, Xs)
    if "h2d_serial" in main_r:
        out["h2d"] = {"serial": round(main_r["h2d_serial"], 2),
                      "overlapped": round(main_r["h2d_overlap"], 2),
                      "unit": "blocks/s", "bytes_per_block": F * T * M * 8,
                      "kind": "X from pinned host memory each step (copy then compute; copy of "
                              "the next step on a side stream under the compute)"}
    for c, r in sec.items():
        out[c] = {"value": round(r["value"], 2), "graph_value": round(r["graph_value"], 2),
                  "per_block": round(r["per_block"], 2), "unit": "blocks/s",
                  "ms_per_step": round(1000.0 * r["elapsed"] / args.steps, 4),
                  "kernels": {k: round(v, 4) for k, v in r["avg"].items()},
                  "steer_roofline": r["rl"]["steer"], "corr_roofline": r["rl"]["corr"],
                  "kind": f"{c} MFMA inputs for the correlation (FP32 accumulation) and a {c} "
                          f"steering table for the projection (through the signal subspace, "
                          f"FP64), FP64 whitening, FP32 Jacobi: batched, and one block per call"}
    if f32 is not None:
        best = max([main_r] + list(sec.values()), key=lambda r: r["value"])
        out["speedup_vs_fp32_per_block"] = round(best["value"] / f32["per_block"], 3)

    if args.serve_seconds > 0:
        variants = {"M": M, "Ns": Ns, "jacobi_lanes": tuning.get("jacobi_lanes"),
                    "steer_waves": tuning.get("steer_waves", {})}
        if args.serve_inproc:
            sv = serving_phase(args, variants)
        else:
            # a fresh process, as a serving deployment runs: after the throughput phases above,
            # the same loop in this process served about 20% fewer blocks at the 10 ms load
            import subprocess
            cmd = [sys.executable, os.path.abspath(__file__)] + sys.argv[1:] + [
                "--serve-child", json.dumps(variants)]
            try:
                res = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=600)
                if res.returncode != 0:
                    raise RuntimeError(f"serving process exited with status {res.returncode}")
                sv = json.loads(res.stdout.strip().splitlines()[-1])
            except (RuntimeError, ValueError, IndexError, subprocess.TimeoutExpired) as exc:
                # the throughput results above stand; the line says why serving is missing
                print(f"serving phase failed: {exc}", file=sys.stderr)
                sv = {"serving_error": str(exc)}
        out.update(sv)

    if not args.no_cpu:
        import oracle
        cores = len(os.sched_getaffinity(0))
        Kh = oracle.noise_corr(Xn.cpu().numpy())
        Hh = w.steering_table()
        nb = max(1, min(args.cpu_blocks, B))
        blocks = [w.block(b)[0] for b in range(nb)]
        tc = time.perf_counter()
        refs = [oracle.localize(X, Kh, Hh, w.grid.n_az, w.grid.n_el, Ns, nthreads=cores)
                for X in blocks]
        cpu_s = time.perf_counter() - tc
        rel = [float(np.max(np.abs(head_pbar[b].astype(np.float64) - r["Pbar"]) / r["Pbar"]))
               for b, r in enumerate(refs)]
        out["cpu_baseline"] = {"value": round(nb / cpu_s, 4), "unit": "blocks/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{nb} blocks of the same 60ch/257-bin/1368-dir workload, "
                                         f"FP64 oracle end to end, threads over bins, {cpu_s:.1f} s",
                               "parity": {"blocks": nb, "prec": args.prec,
                                          "pbar_rel_max": float(f"{max(rel):.3g}"),
                                          "peaks_equal": sum(bool(np.array_equal(head_pk[b], r["peaks"]))
                                                             for b, r in enumerate(refs)),
                                          "kind": "the headline step's Pbar and peaks of these "
                                                  "blocks against the oracle's"}}

    S.ssl_noise_destroy(noise)
    S.ssl_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
