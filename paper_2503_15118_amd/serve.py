"""Serving: a request loop over device-resident simulations on one GPU.

Requests (circuits, or batches of right-hand-side instances that share one op
list) arrive over time.  The server admits them first-in first-out while the
sum of their predicted device footprints (the library's own footprint model at
the request's predicted peak entry count) fits the HBM budget and a slot is
free.  Every admitted request keeps its state resident in its own arena and
runs on its own HIP stream from a worker thread, so requests that arrive while
others are on the GPU start as soon as a slot and memory free up and their
kernels overlap on the device (continuous batching).  Ops run in chunks; the
state stays on the device between chunks.  A request whose state outgrows its
reservation (SS_E_CAPACITY) is checkpointed to host memory, releases its
arena, and is queued again at the front with twice the reservation; when
re-admitted it resumes from the failed op.

The executor is pluggable: ``GpuExecutor`` drives the C ABI; tests use a
fake executor with scripted durations to check admission, back-pressure,
mis-prediction handling and the latency statistics without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Any, Callable, Deque, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the trace
    kind: str
    circuits: list                 # one circuit, or instances sharing one op list
    peak: int                      # predicted peak entries (all instances)
    # filled by the server
    reserve: int = 0               # admitted footprint in bytes
    admitted: float = -1.0
    finished: float = -1.0
    resumes: int = 0
    result: Any = None
    entries: int = 0
    entries_before: int = 0        # entries updated by runs that ended in a checkpoint
    error: Optional[str] = None


class NeedMemory(Exception):
    """Raised by an executor when a request's state outgrew its reservation."""

    def __init__(self, checkpoint, next_op: int, peak: int):
        super().__init__("capacity")
        self.checkpoint = checkpoint
        self.next_op = next_op
        self.peak = peak


def percentile(xs: List[float], q: float) -> float:
    """q-th percentile with linear interpolation between closest ranks."""
    if not xs:
        return float("nan")
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


class Server:
    """Admission by predicted footprint + continuous batching over worker slots."""

    def __init__(self, executor, budget_bytes: int, max_active: int = 8, chunk_ops: int = 128,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk_ops = int(chunk_ops)
        self.clock = clock
        self.lock = threading.Condition()
        self.queue: Deque[Request] = collections.deque()
        self.used = 0
        self.active = 0
        self.peak_used = 0
        self.done: List[Request] = []
        self.resume_state: Dict[int, Any] = {}

    # -- admission ----------------------------------------------------------
    def _admit_locked(self, now: float) -> List[Request]:
        out = []
        while self.queue and self.active < self.max_active:
            r = self.queue[0]
            fp = self.ex.footprint(r)
            if fp > self.budget:
                # can never fit: fail it rather than block the queue
                self.queue.popleft()
                r.error = f"footprint {fp} exceeds the budget {self.budget}"
                r.finished = now
                self.done.append(r)
                continue
            if self.used + fp > self.budget:
                break                      # FIFO: wait for memory to free up
            self.queue.popleft()
            r.reserve = fp
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)
            self.active += 1
            if r.admitted < 0:
                r.admitted = now
            out.append(r)
        return out

    def _worker(self, r: Request, t0: float):
        resume = self.resume_state.pop(r.rid, None)
        try:
            h = self.ex.start(r, resume)
            while not self.ex.step(h, self.chunk_ops):
                pass
            r.result, r.entries = self.ex.finish(h)
            self.ex.release(h)
            fin = self.clock() - t0
            with self.lock:
                r.finished = fin
                self.used -= r.reserve
                self.active -= 1
                self.done.append(r)
                self.lock.notify_all()
        except NeedMemory as nm:
            # checkpointed by the executor; queue again at the front with a
            # doubled reservation and resume from the failed op
            with self.lock:
                self.used -= r.reserve
                self.active -= 1
                r.resumes += 1
                r.peak = max(2 * r.peak, nm.peak)
                self.resume_state[r.rid] = (nm.checkpoint, nm.next_op)
                self.queue.appendleft(r)
                self.lock.notify_all()
        except Exception as e:  # noqa: BLE001  (reported per request)
            with self.lock:
                r.error = repr(e)
                r.finished = self.clock() - t0
                self.used -= r.reserve
                self.active -= 1
                self.done.append(r)
                self.lock.notify_all()

    def run(self, requests: List[Request]) -> Dict[str, Any]:
        """Replay `requests` (arrival times relative to now); returns metrics."""
        pending = sorted(requests, key=lambda r: r.arrival)
        n = len(pending)
        t0 = self.clock()
        threads = []
        i = 0
        with self.lock:
            while len(self.done) < n:
                now = self.clock() - t0
                while i < n and pending[i].arrival <= now:
                    self.queue.append(pending[i])
                    i += 1
                for r in self._admit_locked(now):
                    th = threading.Thread(target=self._worker, args=(r, t0), daemon=True)
                    th.start()
                    threads.append(th)
                wait = 0.05
                if i < n:
                    wait = max(0.0, min(wait, pending[i].arrival - now))
                self.lock.wait(timeout=wait)
        for th in threads:
            th.join()
        wall = self.clock() - t0
        ok = [r for r in self.done if r.error is None]
        lat = [r.finished - r.arrival for r in ok]
        return {
            "requests": n,
            "completed": len(ok),
            "failed": n - len(ok),
            "wall_s": wall,
            "p50_s": percentile(lat, 50),
            "p99_s": percentile(lat, 99),
            "mean_s": float(np.mean(lat)) if lat else float("nan"),
            "requests_per_s": len(ok) / wall if wall > 0 else float("nan"),
            "entries": int(sum(r.entries for r in ok)),
            "entries_per_s": sum(r.entries for r in ok) / wall if wall > 0 else float("nan"),
            "peak_reserved_bytes": self.peak_used,
            "resumes": int(sum(r.resumes for r in self.done)),
        }


class GpuExecutor:
    """Runs requests through the C ABI, each in its own arena on its own stream."""

    def __init__(self, device="cuda:0", tile_order: int = 0):
        import torch
        from . import _abi
        self.torch = torch
        self.abi = _abi
        self.device = torch.device(device)
        # several states run at once on one GPU: one ticket counter per launch
        self.tile_order = tile_order

    def footprint(self, r: Request) -> int:
        c = r.circuits[0]
        tb = sum(max(256, len(t.values) * 8) for t in c.tables) + 4096
        return self.abi.required_bytes(c.regs, len(r.circuits), max(1024, r.peak), tb)

    def start(self, r: Request, resume):
        torch = self.torch
        c = r.circuits[0]
        stream = torch.cuda.Stream(device=self.device)
        tb = sum(max(256, len(t.values) * 8) for t in c.tables) + 4096
        with torch.cuda.stream(stream):
            st = self.abi.State(c.regs, ninst=len(r.circuits), eps=c.eps, cap_entries=max(1024, r.peak),
                                table_bytes=tb, device=self.device, stream=stream)
        st.set_option("tile_order", self.tile_order)
        for t in c.tables:
            st.load_qram(t)
        next_op = 0
        if resume is None:
            for i, ci in enumerate(r.circuits):
                if ci.init_values is not None:
                    st.set_entries(i, ci.init_values, ci.init_amps)
        else:
            ckpt, next_op = resume
            for i, (vals, amps) in enumerate(ckpt):
                st.set_entries(i, vals, amps)
        ops = self.abi.to_ss_ops(c.ops)
        return {"st": st, "ops": ops, "pos": next_op, "req": r, "stream": stream,
                "e0": st.stats()["entries_updated"]}

    def _checkpoint(self, h):
        st = h["st"]
        out = []
        r = h["req"]
        for i in range(len(r.circuits)):
            keys, amps = st.export(i)
            out.append((self._unpack(st, r.circuits[0].regs, keys), amps))
        return out

    @staticmethod
    def _unpack(st, regs, keys):
        vals = np.zeros((len(keys), len(regs)), dtype=np.uint64)
        for j in range(len(regs)):
            w, off, width = st.layout(j)
            mask = np.uint64((1 << width) - 1) if width < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
            vals[:, j] = (keys[:, w] >> np.uint64(off)) & mask
        return vals

    def step(self, h, chunk: int) -> bool:
        ops = h["ops"]
        a, b = h["pos"], min(len(ops), h["pos"] + chunk)
        if a < b:
            res = h["st"].apply(ops[a:b], raise_on_error=False)
            if res.status == self.abi.SS_E_CAPACITY:
                ck = self._checkpoint(h)
                nxt = a + int(res.failed_op)
                # the work done so far counts once the request completes
                h["req"].entries_before += h["st"].stats()["entries_updated"] - h["e0"]
                cap = h["st"].capacity
                h["st"].close()
                h["st"] = None
                raise NeedMemory(ck, nxt, 2 * cap)
            if res.status != 0:
                raise self.abi.SSError(res.status, "ss_apply_ops")
        h["pos"] = b
        return b >= len(ops)

    def finish(self, h):
        st = h["st"]
        r = h["req"]
        res = [st.export(i) for i in range(len(r.circuits))]
        entries = r.entries_before + st.stats()["entries_updated"] - h["e0"]
        return res, entries

    def release(self, h):
        h["st"].close()
        h["st"] = None


def plain_sequential(requests: List[Request], executor, clock=time.perf_counter) -> Dict[str, Any]:
    """The same trace served one request at a time, first come first served:
    each request starts at max(its arrival, the previous finish)."""
    pending = sorted(requests, key=lambda r: r.arrival)
    t0 = clock()
    lat, entries = [], 0
    for r in pending:
        now = clock() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        h = executor.start(r, None)
        while not executor.step(h, 1 << 30):
            pass
        r.result, r.entries = executor.finish(h)
        executor.release(h)
        r.finished = clock() - t0
        lat.append(r.finished - r.arrival)
        entries += r.entries
    wall = clock() - t0
    return {"requests": len(pending), "wall_s": wall, "p50_s": percentile(lat, 50),
            "p99_s": percentile(lat, 99), "requests_per_s": len(pending) / wall,
            "entries": entries, "entries_per_s": entries / wall}
