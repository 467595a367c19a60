"""Server admission and continuous-batching logic with a fake executor (CPU)."""
import threading
import time

import numpy as np
import pytest

from paper_2503_15118_amd import serve


class FakeExecutor:
    """Scripted per-request durations (seconds per chunk) and footprints; can
    raise NeedMemory once to exercise pause / resume."""

    def __init__(self, chunk_s=0.002, fail_once=()):
        self.chunk_s = chunk_s
        self.fail_once = set(fail_once)
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.log = []

    def footprint(self, r):
        return r.peak * 10

    def start(self, r, resume):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.log.append(("start", r.rid, resume is not None))
        return {"r": r, "pos": resume[1] if resume else 0, "n": len(r.circuits[0])}

    def step(self, h, chunk):
        time.sleep(self.chunk_s)
        h["pos"] += 1
        r = h["r"]
        if r.rid in self.fail_once and h["pos"] == 2:
            self.fail_once.discard(r.rid)
            with self.lock:
                self.running -= 1
            raise serve.NeedMemory(checkpoint=["state"], next_op=h["pos"], peak=2 * r.peak)
        return h["pos"] >= h["n"]

    def finish(self, h):
        return ("done", h["r"].rid), 7

    def release(self, h):
        with self.lock:
            self.running -= 1


def _reqs(n, peak=10, gap=0.001, steps=4):
    return [serve.Request(rid=i, arrival=i * gap, kind="c1", circuits=[list(range(steps))], peak=peak)
            for i in range(n)]


def test_all_requests_complete_with_bounded_concurrency():
    ex = FakeExecutor()
    srv = serve.Server(ex, budget_bytes=10_000, max_active=3, chunk_ops=1)
    m = srv.run(_reqs(12))
    assert m["completed"] == 12 and m["failed"] == 0
    assert ex.max_running <= 3
    assert m["entries"] == 12 * 7
    assert m["p99_s"] >= m["p50_s"] > 0


def test_admission_respects_memory_budget():
    ex = FakeExecutor()
    # each request reserves 100 bytes; budget 250 -> at most 2 at once
    srv = serve.Server(ex, budget_bytes=250, max_active=8, chunk_ops=1)
    m = srv.run(_reqs(6, peak=10))
    assert m["completed"] == 6
    assert ex.max_running <= 2
    assert m["peak_reserved_bytes"] <= 250


def test_oversized_request_fails_without_blocking_others():
    ex = FakeExecutor()
    reqs = _reqs(4, peak=10)
    reqs[1].peak = 10_000          # footprint beyond the budget
    srv = serve.Server(ex, budget_bytes=500, max_active=4, chunk_ops=1)
    m = srv.run(reqs)
    assert m["completed"] == 3 and m["failed"] == 1
    assert [r.error is not None for r in sorted(srv.done, key=lambda r: r.rid)] == [False, True, False, False]


def test_misprediction_pauses_and_resumes_with_doubled_reservation():
    ex = FakeExecutor(fail_once={2})
    srv = serve.Server(ex, budget_bytes=10_000, max_active=2, chunk_ops=1)
    m = srv.run(_reqs(5, peak=10))
    assert m["completed"] == 5 and m["resumes"] == 1
    r2 = [r for r in srv.done if r.rid == 2][0]
    assert r2.peak == 20 and r2.reserve == 200
    starts = [e for e in ex.log if e[1] == 2]
    assert starts == [("start", 2, False), ("start", 2, True)]


def test_later_arrivals_join_while_earlier_ones_run():
    ex = FakeExecutor(chunk_s=0.01)
    reqs = _reqs(2, gap=0.0, steps=10) + [serve.Request(rid=9, arrival=0.03, kind="c1",
                                                        circuits=[list(range(2))], peak=10)]
    srv = serve.Server(ex, budget_bytes=10_000, max_active=4, chunk_ops=1)
    m = srv.run(reqs)
    assert m["completed"] == 3
    late = [r for r in srv.done if r.rid == 9][0]
    first = [r for r in srv.done if r.rid == 0][0]
    # admitted while request 0 was still running, and finished before it
    assert late.admitted < first.finished
    assert late.finished < first.finished


def test_percentiles():
    assert serve.percentile([1.0, 2.0, 3.0, 4.0], 50) == 2.5
    assert abs(serve.percentile(list(range(101)), 99) - 99.0) < 1e-12
    assert np.isnan(serve.percentile([], 50))


def test_trace_generator_shape():
    import workloads as wl
    tr = wl.c5_trace(3, rate=200.0, duration=0.2, c4_steps=2, c4_matrix_n=64, hi_bits=16)
    assert len(tr) > 10
    arr = [t.arrival for t in tr]
    assert arr == sorted(arr) and arr[-1] <= 0.2
    for t in tr:
        assert t.kind in ("c1", "c2", "c3", "c4")
        if t.kind in ("c1", "c3"):
            assert t.peak <= 2 ** 18
        if t.kind == "c4":
            assert len(t.circuits) * 64 * 16 == t.peak or len(t.circuits) == 1
