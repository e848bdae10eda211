"""Serving scheduler on the CPU: a fake executor with a latency model and a simulated clock.

Checks admission by HBM budget, the per-stream in-flight limit, per-stream order,
continuous batching (a batch starts on a free lane while another runs), latency bookkeeping and the
oversize-block error.  No GPU and no HIP library involved.
"""
import numpy as np
import pytest

from paper_2504_03373_amd.serving import Server
import synth


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Batch of n blocks takes a + b * n seconds; records what the scheduler asked for."""

    def __init__(self, clock, costs, lanes=2, a=2e-3, b=1e-4, depth=1):
        self.clock, self.costs, self.lanes, self.a, self.b = clock, costs, lanes, a, b
        self.inflight = [None] * lanes
        self.log = []
        self.max_bytes = 0
        self.max_depth = 0
        if depth != 1:
            self.stream_depth = depth

    def cost_bytes(self, sid):
        return self.costs[sid]

    def submit(self, lane, reqs):
        assert self.inflight[lane] is None
        assert len({r.stream for r in reqs}) == len(reqs)
        n = {}
        for x in self.inflight:
            for r in (x[0] if x else []):
                n[r.stream] = n.get(r.stream, 0) + 1
        for r in reqs:
            n[r.stream] = n.get(r.stream, 0) + 1
        self.max_depth = max([self.max_depth] + list(n.values()))
        assert self.max_depth <= getattr(self, "stream_depth", 1), "too many blocks of a stream in flight"
        self.inflight[lane] = (reqs, self.clock() + self.a + self.b * len(reqs))
        self.log.append((self.clock(), lane, [(r.stream, r.seq) for r in reqs]))
        used = sum(self.costs[r.stream] for x in self.inflight if x for r in x[0])
        self.max_bytes = max(self.max_bytes, used)

    def poll(self, lane):
        return self.clock() >= self.inflight[lane][1]

    def collect(self, lane):
        for r in self.inflight[lane][0]:
            r.peaks = np.array([r.stream, r.seq])
        self.inflight[lane] = None


def run(arrivals, costs, budget, lanes=2, max_batch=64, a=2e-3, b=1e-4, depth=1):
    clk = FakeClock()
    ex = FakeExecutor(clk, costs, lanes, a, b, depth)
    srv = Server(ex, budget, max_batch=max_batch, clock=clk, sleep=clk.sleep, poll_s=1e-4)
    return srv.run(arrivals), ex


def test_everything_completes_in_stream_order():
    arr = synth.poisson_arrivals(16, 0.2, 0.010, seed=1)
    st, ex = run(arr, [100] * 16, budget=10_000)
    assert st["completed"] == len(arr)
    order = {}
    for _, _, items in ex.log:
        for s, q in items:
            assert q == order.get(s, -1) + 1, "per-stream order broken"
            order[s] = q
    for r in st["requests"]:
        assert r.done_t >= r.submit_t >= r.emit_t
        assert r.peaks.tolist() == [r.stream, r.seq]


def test_budget_respected():
    arr = synth.poisson_arrivals(32, 0.1, 0.005, seed=2)
    costs = [300 if s % 3 == 0 else 100 for s in range(32)]
    st, ex = run(arr, costs, budget=2000)
    assert st["completed"] == len(arr)
    assert ex.max_bytes <= 2000
    # no batch exceeds a lane's share
    for _, _, items in ex.log:
        assert sum(costs[s] for s, _ in items) <= 1000


def test_continuous_batching_overlaps_lanes():
    """With blocks arriving steadily, the second lane starts batches while the first is busy."""
    arr = synth.poisson_arrivals(64, 0.2, 0.010, seed=3)
    st, ex = run(arr, [10] * 64, budget=1 << 20, a=5e-3, b=2e-4)
    starts = [(t, lane) for t, lane, _ in ex.log]
    overlapped = 0
    for i in range(1, len(starts)):
        if starts[i][1] != starts[i - 1][1]:
            overlapped += 1
    assert overlapped > 0.3 * len(starts)
    assert st["mean_batch"] > 1.0


def test_latency_arithmetic_single_lane():
    """One stream, one lane, arrivals far apart: latency = a + b exactly (plus polling slack)."""
    arr = [(0.1 * k, 0, k) for k in range(10)]
    st, ex = run(arr, [1], budget=10, lanes=1, a=3e-3, b=1e-3)
    lat = np.array([r.done_t - r.emit_t for r in st["requests"]])
    assert np.all(lat >= 4e-3 - 1e-9) and np.all(lat <= 4e-3 + 3e-4)
    assert abs(st["p50_ms"] - np.percentile(lat, 50) * 1e3) < 1e-9
    assert st["batches"] == 10


def test_oversize_block_rejected():
    with pytest.raises(RuntimeError):
        run([(0.0, 0, 0)], [5000], budget=1000)


def test_max_batch_cap():
    arr = [(0.0, s, 0) for s in range(40)]
    st, ex = run(arr, [1] * 40, budget=1 << 20, max_batch=8)
    assert all(len(items) <= 8 for _, _, items in ex.log)
    assert st["completed"] == 40


def test_stream_depth_two():
    """With two blocks per stream allowed in flight, a backlogged stream gets its next block into
    the other lane while the first runs; submission order per stream is kept."""
    arr = [(0.0, s, k) for s in range(4) for k in range(6)]
    arr.sort()
    st, ex = run(arr, [1] * 4, budget=1 << 20, lanes=2, depth=2)
    assert st["completed"] == len(arr)
    assert ex.max_depth == 2
    order = {}
    for _, _, items in ex.log:
        for s, q in items:
            assert q == order.get(s, -1) + 1, "per-stream order broken"
            order[s] = q
    st1, ex1 = run(arr, [1] * 4, budget=1 << 20, lanes=2, depth=1)
    assert ex1.max_depth == 1
    assert max(r.done_t for r in st["requests"]) < max(r.done_t for r in st1["requests"])


def test_ready_hook_delays_blocks():
    """A block the executor reports not ready (inputs still uploading) stays out of batches until
    it is; everything completes, per-stream order holds, and no block runs before it is ready."""
    clk = FakeClock()
    ex = FakeExecutor(clk, [1] * 8, lanes=2, a=1e-3, b=1e-4)
    upload_s = 2e-3
    ex.ready = lambda r: clk() >= r.emit_t + upload_s
    seen = []
    orig = ex.submit

    def submit(lane, reqs):
        for r in reqs:
            seen.append(clk() - r.emit_t)
        orig(lane, reqs)
    ex.submit = submit
    arr = synth.poisson_arrivals(8, 0.05, 0.005, seed=5)
    st = Server(ex, 1 << 20, max_batch=16, clock=clk, sleep=clk.sleep, poll_s=1e-4).run(arr)
    assert st["completed"] == len(arr)
    assert min(seen) >= upload_s - 1e-12
    order = {}
    for _, _, items in ex.log:
        for s, q in items:
            assert q == order.get(s, -1) + 1
            order[s] = q
