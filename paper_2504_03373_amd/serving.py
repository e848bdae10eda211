"""Continuous-batching localization server for many microphone-array streams.

Blocks arrive from array streams of different channel counts.  The scheduler admits them as
lanes and HBM budget free up, packs every admitted block into the next batch on a free lane (a
lane = a library context + a HIP stream, so a batch can be formed and started while another runs
on the device), and records each block's latency from emission to results on the host.  Each
stream's noise correlation K stays resident on the device and is updated by exponential averaging
with the noise-only frames that accompany its blocks (K <- alpha K + (1 - alpha) K_hat, then a
fresh FP64 inverse).  With a lag of L blocks (k_lag), block n runs on the K that includes the
noise of blocks <= n - 1 - L: at L = 0 the update of block n lands before block n + 1 runs; at
L = 1 (the default) it runs beside block n + 1, so the update is off the stream's round trip.
K versions live in a ring of four handles per stream: an update writes a handle no block in
flight reads.  Every dependency between HIP streams is a device-side wait on the producer's event:
a batch waits for the uploads of its blocks and for the updates producing the K versions they
read, an update waits for the upload of the noise-only frames it reads (whichever stream carried
it), and a slot is overwritten only after its previous batch and update (on the host, or by a
device wait when the upload rides on the lane stream).  The host-side readiness checks
(`ready`) are scheduling policy only: they keep a batch from queueing behind work in flight.

Rules: at most `stream_depth` blocks per stream are in flight (an executor attribute, 1 if
absent; the GPU executor allows 1 + k_lag, the most for which the K versions the blocks read are
never being written), and a stream's blocks are submitted in order; a lane's batch never needs more
than its share of the HBM budget; requests wait in arrival order, skipping only blocks of streams
at their in-flight limit (kept as one FIFO per stream, so forming a batch costs O(streams), not
O(queue)).

The executor interface (`lanes`, `cost_bytes`, `submit`, `poll`, `collect`, and optionally
`arrive`, told of each block as it is emitted, `ready`, false while a block's inputs are still
being uploaded, and `stream_depth`) is what the scheduler needs; `GpuExecutor` implements it with
the library's C ABI.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    stream: int
    seq: int
    emit_t: float
    submit_t: float = -1.0
    done_t: float = -1.0
    batch: int = -1
    k_version: int = -1          # EMA updates applied to the stream's K before this block ran
    peaks: np.ndarray = None
    peak_val: np.ndarray = None
    Pbar: np.ndarray = None      # eq.6 spectrum of the block (only with GpuExecutor(keep_pbar=True))


class Server:
    def __init__(self, executor, hbm_budget_bytes: int, max_batch: int = 64,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, poll_s: float = 50e-6):
        self.ex = executor
        self.lane_budget = hbm_budget_bytes // max(1, executor.lanes)
        self.max_batch = max_batch
        self.clock = clock
        self.sleep = sleep
        self.poll_s = poll_s

    def run(self, arrivals: Sequence[tuple]) -> dict:
        """arrivals: (emit time s, stream, seq), sorted by time.  Runs until every block is done."""
        pending = collections.deque(Request(stream=s, seq=q, emit_t=t) for t, s, q in arrivals)
        # ready blocks, one FIFO per stream: the candidates of a batch are the heads of the
        # streams below their in-flight limit, taken in emission order -- the same order as
        # scanning one arrival-ordered queue and skipping streams at the limit, at a cost of
        # O(streams) per batch instead of O(queue)
        queues = collections.defaultdict(collections.deque)
        n_ready = 0
        depth = max(1, int(getattr(self.ex, "stream_depth", 1)))
        in_flight = collections.Counter()
        cost_of = {}
        lanes = [None] * self.ex.lanes          # per lane: list of requests in flight
        done: List[Request] = []
        batches = 0
        max_ready = 0
        host = dict(submit_s=0.0, collect_s=0.0, sleep_s=0.0)   # where the loop's time goes
        arrive = getattr(self.ex, "arrive", None)
        ready = getattr(self.ex, "ready", None)
        t0 = self.clock()
        while pending or n_ready or any(lanes):
            now = self.clock() - t0
            while pending and pending[0].emit_t <= now:
                r = pending.popleft()
                queues[r.stream].append(r)
                n_ready += 1
                if arrive is not None:
                    arrive(r)
            max_ready = max(max_ready, n_ready)
            progressed = False
            for li, reqs in enumerate(lanes):
                if reqs and self.ex.poll(li):
                    tc = self.clock()
                    self.ex.collect(li)
                    host["collect_s"] += self.clock() - tc
                    tdone = self.clock() - t0
                    for r in reqs:
                        r.done_t = tdone
                        in_flight[r.stream] -= 1
                    done.extend(reqs)
                    lanes[li] = None
                    progressed = True
            for li in range(len(lanes)):
                if lanes[li] is not None or not n_ready:
                    continue
                heads = sorted((q[0] for sid, q in queues.items()
                                if q and in_flight[sid] < depth and (ready is None or ready(q[0]))),
                               key=lambda r: (r.emit_t, r.stream, r.seq))
                batch, cost = [], 0
                for r in heads:
                    if len(batch) >= self.max_batch:
                        break
                    if r.stream not in cost_of:
                        cost_of[r.stream] = self.ex.cost_bytes(r.stream)
                    c = cost_of[r.stream]
                    if cost + c <= self.lane_budget:
                        batch.append(r)
                        cost += c
                if not batch:
                    if not any(lanes) and heads and all(cost_of[r.stream] > self.lane_budget
                                                        for r in heads):
                        raise RuntimeError("a single block exceeds the per-lane HBM budget")
                    break
                for r in batch:
                    queues[r.stream].popleft()
                    in_flight[r.stream] += 1
                n_ready -= len(batch)
                tsub = self.clock() - t0
                for r in batch:
                    r.submit_t = tsub
                    r.batch = batches
                self.ex.submit(li, batch)
                host["submit_s"] += self.clock() - t0 - tsub
                lanes[li] = batch
                batches += 1
                progressed = True
            if not progressed:
                nxt = pending[0].emit_t - (self.clock() - t0) if pending else self.poll_s
                ts = self.clock()
                self.sleep(max(0.0, min(self.poll_s, nxt)))
                host["sleep_s"] += self.clock() - ts
        out = summarize(done, batches, max_ready)
        out.update(host, loop_s=self.clock() - t0)
        return out


def summarize(done: List[Request], batches: int, max_ready: int) -> dict:
    lat = np.array([r.done_t - r.emit_t for r in done]) * 1e3
    if len(done) == 0:
        return dict(completed=0)
    span = max(r.done_t for r in done) - min(r.emit_t for r in done)
    return dict(completed=len(done), blocks_per_s=len(done) / span if span > 0 else float("inf"),
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                max_ms=float(lat.max()), batches=batches, mean_batch=len(done) / max(1, batches),
                max_queue=max_ready, requests=done)


# ------------------------------------------------------------------------------------------------
class GpuExecutor:
    """Executes batches with ssl_localize_batch on `lanes` (context, HIP stream) pairs; per-stream
    noise handles, device input slots and pinned host pools of pre-generated blocks.

    streams: objects with M, F, T, Ns, D, grid (n_az, n_el), `pos`, `freqs`, initial_noise_frames()
    and block(seq) -> (X, noise-only frames); `pool` blocks per stream are generated up front and
    reused cyclically (block seq uses pool entry seq % pool).  `configure`, if given, is called
    with each batch context after creation (to apply tuned kernel variants).

    Input staging: each stream owns `slots` device slots (frames X and noise-only frames).  A
    block is uploaded from pinned host memory on a copy stream as soon as it is emitted and a slot
    is free, so uploads overlap the batches on the device; a batch then only waits for its blocks'
    copy events.  A slot frees when its block's K update (or, without one, its batch) has run; a
    block still unstaged when its batch is formed is uploaded on the lane stream, after a device
    wait for the slot's previous readers.  `stage_at_arrival=False` uploads every block that way
    (a test of that path).  `keep_pbar=True` also copies each block's Pbar back to the host.
    """

    def __init__(self, streams, steering, prec=None, p: int = 2, alpha: float = 0.95,
                 k_update_every: int = 1, hbm_budget_bytes: int = 4 << 30, lanes: int = 2,
                 pool: int = 4, device: int = 0, update_contexts: int = 4, configure=None,
                 slots: int = 4, k_lag: int = 1, stage_at_arrival: bool = True,
                 keep_pbar: bool = False):
        import torch

        from . import (SSL_FP32, SSL_FP64, block_desc, ssl_corr_accum, ssl_ctx_create,
                       ssl_noise_create, ssl_noise_set)
        if k_lag not in (0, 1):
            raise ValueError("k_lag must be 0 or 1")
        if slots < 2 + k_lag:
            raise ValueError("need slots >= 2 + k_lag (blocks in flight plus one staged)")
        self.torch = torch
        self.dev = f"cuda:{device}"
        self.prec = SSL_FP32 if prec is None else prec
        self.p = p
        self.alpha = alpha
        self.k_every = max(1, k_update_every)
        self.lanes = lanes
        self.streams = list(streams)
        self.pool = pool
        self._block_desc = block_desc
        self._fp64 = SSL_FP64
        from . import ssl_ctx_use_graphs
        self.ctxs = [ssl_ctx_create(device, hbm_budget_bytes // lanes) for _ in range(lanes)]
        for c in self.ctxs:
            # every batch has a different composition: capture would never be replayed
            ssl_ctx_use_graphs(c, False)
            if configure is not None:          # e.g. apply autotuned kernel variants
                configure(c)
        self.nctx = ssl_ctx_create(device, 0)
        self.tstreams = [torch.cuda.Stream(device=self.dev) for _ in range(lanes)]
        # K updates run on one stream of their own, in submission order (so version v of a
        # stream is complete before v + 1 starts, with no waits between updates); a batch waits
        # only for the updates that produced the K versions its blocks read.  Few streams on
        # purpose: HIP maps streams onto a handful of hardware queues, and a stream's wait on
        # another parked at the head of a shared queue holds back everything behind it.
        self.ustream = torch.cuda.Stream(device=self.dev)
        # steering tables per channel count (shared by streams of the same geometry)
        self.H = {M: t for M, t in steering.items()}
        self.noise, self.X_slot, self.Xn_slot, self.X_pool, self.Xn_pool = [], [], [], [], []
        # K versions: version v (v updates applied) lives in handle v % NH of the stream; an
        # update reads version v and writes v + 1.  With at most 1 + k_lag blocks of a stream in
        # flight, reading versions >= v - 1 - k_lag, the handle of v + 1 (that of v + 1 - NH) is
        # read by none of them.  k_version = updates launched, k_done[v % NH] = (event
        # completing version v, update call number), None for the initial version
        self.k_lag = k_lag
        self.stream_depth = 1 + k_lag
        self.k_version = [0] * len(self.streams)
        self.NH = 4
        self.k_done = [[None] * self.NH for _ in self.streams]
        self.n_updates = 0
        # update calls go round-robin over a few library contexts: a call waits (on the host) for
        # its context's previous descriptor upload, which sits behind that call's batch
        self.uctx = [ssl_ctx_create(device, 0) for _ in range(max(1, update_contexts))]
        self.next_uctx = 0
        for s in self.streams:
            Xn0 = torch.from_numpy(s.initial_noise_frames()).to(self.dev)
            K0 = torch.zeros((s.F, s.M, s.M), dtype=torch.complex128, device=self.dev)
            ssl_corr_accum(self.nctx, Xn0, 1.0 / Xn0.shape[1], 0, SSL_FP64, K0)
            ring = []
            for _ in range(self.NH):
                n = ssl_noise_create(self.nctx, s.F, s.M)
                ssl_noise_set(n, K0, SSL_FP64)
                ring.append(n)
            self.noise.append(ring)
            xs, xns = [], []
            for q in range(pool):
                X, Xn = s.block(q)
                xs.append(torch.from_numpy(X).pin_memory())
                xns.append(torch.from_numpy(Xn).pin_memory())
            self.X_pool.append(xs)
            self.Xn_pool.append(xns)
            self.X_slot.append([torch.empty((s.F, s.T, s.M), dtype=torch.complex64, device=self.dev)
                                for _ in range(slots)])
            self.Xn_slot.append([torch.empty((s.F, s.T, s.M), dtype=torch.complex64, device=self.dev)
                                 for _ in range(slots)])
        torch.cuda.synchronize()
        # staging state per stream: slot owners (request staged into it, until collected), the
        # events after which a released slot may be overwritten (its batch, its K update), blocks
        # waiting for a slot
        self.cstream = torch.cuda.Stream(device=self.dev)
        self.nslot = slots
        self.slot_owner = [[None] * slots for _ in self.streams]
        self.slot_free = [[()] * slots for _ in self.streams]
        self.waiting = [collections.deque() for _ in self.streams]
        self.to_pump = set()
        self.staged = {}          # (stream, seq) -> (slot, copy event or None, staging number)
        self.n_staged = 0
        nmax = 4096
        self.pk = [torch.zeros((nmax, 3), dtype=torch.int32, device=self.dev) for _ in range(lanes)]
        self.pv = [torch.zeros((nmax, 3), dtype=torch.float32, device=self.dev) for _ in range(lanes)]
        self.pk_h = [torch.zeros((nmax, 3), dtype=torch.int32).pin_memory() for _ in range(lanes)]
        self.pv_h = [torch.zeros((nmax, 3), dtype=torch.float32).pin_memory() for _ in range(lanes)]
        self.stage_at_arrival = stage_at_arrival
        self.keep_pbar = keep_pbar
        if keep_pbar:
            nb, dmax = 512, max(s.D for s in self.streams)
            self.pb = [torch.zeros((nb, dmax), dtype=torch.float32, device=self.dev)
                       for _ in range(lanes)]
            self.pb_h = [torch.zeros((nb, dmax), dtype=torch.float32).pin_memory()
                         for _ in range(lanes)]
        self.inflight = [None] * lanes

    def cost_bytes(self, sid: int) -> int:
        """Device bytes a block holds while in flight: its batch workspace slices (the same sizes
        ssl_localize_batch reserves) plus its input slots."""
        s = self.streams[sid]
        a = lambda n: (n + 255) // 256 * 256
        F, M, D, Nn = s.F, s.M, s.D, s.M - s.Ns
        ws = (2 * a(F * M * M * 8) + a(F * Nn * M * 8) + a(F * D * 4) + a(-(-F // 16) * D * 4)
              + a(F * 4) + a(D * 4))
        return ws + 2 * F * s.T * M * 8

    def _stage(self, r: "Request", k: int, st) -> None:
        """Upload block r into slot k of its stream on HIP stream st.  On the copy stream the
        caller has seen the slot's previous readers complete; on a lane stream the copy waits for
        them on the device.  Records the upload's completion event: (slot, event, staging number
        on the copy stream or -1 on a lane stream)."""
        torch = self.torch
        sid = r.stream
        self.slot_owner[sid][k] = r
        with torch.cuda.stream(st):
            if st is not self.cstream:
                for e in self.slot_free[sid][k]:
                    st.wait_event(e)
            self.slot_free[sid][k] = ()
            self.X_slot[sid][k].copy_(self.X_pool[sid][r.seq % self.pool], non_blocking=True)
            self.Xn_slot[sid][k].copy_(self.Xn_pool[sid][r.seq % self.pool], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
            num = -1
            if st is self.cstream:               # copies complete in staging order
                self.n_staged += 1
                num = self.n_staged
        self.staged[(sid, r.seq)] = (k, ev, num)

    def _free_slot(self, sid: int, ready_only: bool):
        """A released slot (whose readers have completed, if ready_only)."""
        for k in range(self.nslot):
            if self.slot_owner[sid][k] is None:
                if not ready_only or all(e.query() for e in self.slot_free[sid][k]):
                    return k
        return None

    def _pump(self, sid: int) -> None:
        q = self.waiting[sid]
        while q:
            k = self._free_slot(sid, ready_only=True)
            if k is None:
                self.to_pump.add(sid)
                return
            self._stage(q.popleft(), k, self.cstream)
        self.to_pump.discard(sid)

    def arrive(self, r: "Request") -> None:
        if not self.stage_at_arrival:
            return
        self.waiting[r.stream].append(r)
        self._pump(r.stream)

    def ready(self, r: "Request") -> bool:
        """Scheduling policy, not ordering: false while r's upload on the copy stream or the K
        update producing the K version it will read is in flight, so that a batch is not queued
        behind them (a block not staged yet is uploaded on the lane stream at submission, in
        order with its batch)."""
        st = self.staged.get((r.stream, r.seq))
        if st is not None and st[2] >= 0 and not st[1].query():
            return False
        kd = self.k_done[r.stream][max(0, self.k_version[r.stream] - self.k_lag) % self.NH]
        return kd is None or kd[0].query()

    def submit(self, lane: int, reqs: List["Request"]) -> None:
        from . import ssl_localize_batch
        torch = self.torch
        st = self.tstreams[lane]
        if self.keep_pbar and len(reqs) > self.pb[lane].shape[0]:
            raise ValueError(f"keep_pbar holds at most {self.pb[lane].shape[0]} blocks per batch")
        descs = []
        with torch.cuda.stream(st):
            last_update = None                    # updates complete in call order
            for r in reqs:
                if (r.stream, r.seq) not in self.staged:
                    # not uploaded yet (no slot was free, or the scheduler was not told): it is the
                    # oldest block of its stream not yet submitted, so only the stream's blocks in
                    # flight (fewer than stream_depth <= slots) own slots; the others are released
                    # and their last readers are waited for on the device (_stage)
                    q = self.waiting[r.stream]
                    if q and q[0] is r:
                        q.popleft()
                    k = self._free_slot(r.stream, ready_only=True)
                    if k is None:
                        k = self._free_slot(r.stream, ready_only=False)
                    self._stage(r, k, st)
                r.k_version = max(0, self.k_version[r.stream] - self.k_lag)
                kd = self.k_done[r.stream][r.k_version % self.NH]
                if kd is not None and (last_update is None or kd[1] > last_update[1]):
                    last_update = kd
            # device-side waits for every producer on another stream: the copy stream runs in
            # staging order, so its last upload among the batch's blocks covers all of them; the
            # update stream runs in call order, so the latest K version read covers the others
            cp = [self.staged[(r.stream, r.seq)] for r in reqs]
            cp = [t for t in cp if t[2] >= 0]
            if cp:
                st.wait_event(max(cp, key=lambda t: t[2])[1])
            if last_update is not None:
                st.wait_event(last_update[0])
            for i, r in enumerate(reqs):
                s = self.streams[r.stream]
                k = self.staged[(r.stream, r.seq)][0]
                pb = self.pb[lane][i] if self.keep_pbar else None
                descs.append(self._block_desc(self.X_slot[r.stream][k],
                                              self.noise[r.stream][r.k_version % self.NH],
                                              self.H[s.M], s.grid.n_az, s.grid.n_el, s.Ns,
                                              self.pk[lane][i], self.pv[lane][i], pb))
            ssl_localize_batch(self.ctxs[lane], descs, self.prec, self.p, stream=st)
            n = len(reqs)
            self.pk_h[lane][:n].copy_(self.pk[lane][:n], non_blocking=True)
            self.pv_h[lane][:n].copy_(self.pv[lane][:n], non_blocking=True)
            if self.keep_pbar:
                self.pb_h[lane][:n].copy_(self.pb[lane][:n], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        self.inflight[lane] = (reqs, ev, self._launch_updates(reqs, ev))

    def _launch_updates(self, reqs: List["Request"], ev):
        """K EMA updates of the blocks of a batch, launched with it: one library call on the
        update stream (updates run in launch order there), all their bins in one launch pair per
        channel class.  Returns the completion event (None if no block of the batch updates K)."""
        from . import ssl_noise_update_frames_from
        torch = self.torch
        ups = [r for r in reqs if (r.seq + 1) % self.k_every == 0]
        if not ups:
            return None
        i = self.next_uctx
        self.next_uctx = (i + 1) % len(self.uctx)
        ns = self.ustream
        with torch.cuda.stream(ns):
            # no wait on the batch: the update writes a handle no block in flight reads.  Its
            # inputs: the source K version, produced earlier on this stream; the noise-only frames,
            # whose upload it waits for on the device (the copy stream's last one among these
            # blocks covers the others there; every upload that rode on a lane stream separately)
            stg = [self.staged[(r.stream, r.seq)] for r in ups]
            cp = [t for t in stg if t[2] >= 0]
            if cp:
                ns.wait_event(max(cp, key=lambda t: t[2])[1])
            for t in stg:
                if t[2] < 0:
                    ns.wait_event(t[1])
            v = [self.k_version[r.stream] for r in ups]
            ssl_noise_update_frames_from(
                self.uctx[i], [self.noise[r.stream][(vv + 1) % self.NH] for r, vv in zip(ups, v)],
                [self.noise[r.stream][vv % self.NH] for r, vv in zip(ups, v)],
                [self.Xn_slot[r.stream][self.staged[(r.stream, r.seq)][0]] for r in ups],
                self.alpha, stream=ns)
            done = torch.cuda.Event()
            done.record(ns)
        self.n_updates += 1
        for r in ups:
            self.k_version[r.stream] += 1
            self.k_done[r.stream][self.k_version[r.stream] % self.NH] = (done, self.n_updates)
        return done

    def poll(self, lane: int) -> bool:
        for sid in list(self.to_pump):
            self._pump(sid)
        return self.inflight[lane][1].query()

    def collect(self, lane: int) -> None:
        reqs, ev, done = self.inflight[lane]
        ev.synchronize()
        pk, pv = self.pk_h[lane].numpy(), self.pv_h[lane].numpy()
        for i, r in enumerate(reqs):
            ns = self.streams[r.stream].Ns
            r.peaks = pk[i, :ns].copy()
            r.peak_val = pv[i, :ns].copy()
            if self.keep_pbar:
                r.Pbar = self.pb_h[lane][i, :self.streams[r.stream].D].numpy().copy()
        for r in reqs:                            # release the slots, reusable after their readers
            k = self.staged.pop((r.stream, r.seq))[0]
            self.slot_owner[r.stream][k] = None
            self.slot_free[r.stream][k] = (ev, done) if (r.seq + 1) % self.k_every == 0 else (ev,)
            if self.waiting[r.stream]:
                self.to_pump.add(r.stream)
        self.inflight[lane] = None

    def close(self) -> None:
        from . import ssl_ctx_destroy, ssl_noise_destroy
        self.torch.cuda.synchronize()
        for ring in self.noise:
            for n in ring:
                ssl_noise_destroy(n)
        for c in self.ctxs + self.uctx:
            ssl_ctx_destroy(c)
        ssl_ctx_destroy(self.nctx)
