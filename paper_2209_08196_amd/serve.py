"""Continuous-batching encode server over many sensor streams.

Scans arrive from many sensors at their own rates.  A producer thread
releases each scan at its arrival time on the wall clock; the serving loop
admits it, and whenever one of its step contexts is free it submits the
scans that have arrived -- at most one per stream, oldest first -- as one
asynchronous batched step (jiffy_step_submit) on that context's own HIP
stream, then goes on admitting arrivals and submitting to the other context
while the first runs.  A finished step's records come back to the host in
one copy; a scan's latency is the time its records are on the host minus its
arrival time.  Each stream predicts from its own resident previous scan
(Sec. III-D), so a stream's records are exactly those of encoding its scan
sequence alone.

Device memory is bounded by a budget fixed at start: the step contexts'
workspaces and packed output buffers are allocated once; the rest is a pool
from which each admitted stream's resident state is carved
(jiffy_stream_create_at).  A scan of a stream that is not admitted is
admitted when its state fits in the pool, else dropped (counted).  A stream
idle for longer than `idle_s` is closed and its state returned to the pool,
where later arrivals reuse it; its next scan starts a new session (an
I-scan).  Nothing is allocated on the device while serving.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np

_ALIGN = 256


def _al(x):
    return (x + _ALIGN - 1) // _ALIGN * _ALIGN


@dataclasses.dataclass(frozen=True)
class StreamSpec:
    height: int
    width: int
    widths: tuple
    precisions: tuple

    @property
    def records(self):
        return len(self.widths)

    @property
    def samples(self):
        return self.height * self.width * len(self.widths)


class Pool:
    """First-fit allocator over [0, capacity) in 256-byte units, with
    coalescing frees.  Offsets only: the memory itself is the backend's."""

    def __init__(self, capacity):
        self.capacity = int(capacity) // _ALIGN * _ALIGN
        self.free = [(0, self.capacity)] if self.capacity > 0 else []  # sorted (offset, size)
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes):
        n = _al(max(int(nbytes), 1))
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                if s == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, s - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return o
        return None

    def release(self, offset, nbytes):
        n = _al(max(int(nbytes), 1))
        self.used -= n
        self.free.append((offset, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged


@dataclasses.dataclass
class ServeStats:
    scans_done: int = 0
    scans_dropped: int = 0
    admissions: int = 0
    evictions: int = 0
    streams_seen: int = 0
    steps: int = 0
    points: int = 0
    wall_s: float = 0.0
    busy_s: float = 0.0
    overlap_steps: int = 0
    pool_bytes: int = 0
    pool_peak_bytes: int = 0
    fixed_bytes: int = 0
    latencies_s: list = dataclasses.field(default_factory=list)
    batch_sizes: list = dataclasses.field(default_factory=list)

    def summary(self):
        lat = np.asarray(self.latencies_s) if self.latencies_s else np.zeros(1)
        return {
            "scans": self.scans_done, "dropped_scans": self.scans_dropped,
            "admissions": self.admissions, "evictions": self.evictions,
            "steps": self.steps, "steps_submitted_while_another_ran": self.overlap_steps,
            "mean_batch": round(float(np.mean(self.batch_sizes)) if self.batch_sizes else 0, 2),
            "max_batch": int(max(self.batch_sizes)) if self.batch_sizes else 0,
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "max_ms": round(1e3 * float(lat.max()), 3),
            "points_per_s": round(self.points / self.wall_s, 1) if self.wall_s else 0.0,
            "points_per_s_busy": round(self.points / self.busy_s, 1) if self.busy_s else 0.0,
            "wall_s": round(self.wall_s, 3),
            "device_bytes_fixed": self.fixed_bytes, "state_pool_bytes": self.pool_bytes,
            "state_pool_peak_bytes": self.pool_peak_bytes,
        }


class Server:
    """budget_bytes: device bytes the server may use in all.  backend: the
    encoder (GpuBackend over libjiffy, or a stand-in for host-logic tests)
    exposing state_bytes(spec), record_bound(spec), setup(slots, max_records,
    max_samples, out_capacity, pool_bytes) -> fixed device bytes,
    open(sid, spec, offset), close(sid), submit(slot, sids, scans),
    done(slot) -> bool, finish(slot) -> one bytes-like object of records per
    stream (read before the slot's next step).
    Steps hold at most max_records records, max_samples samples and
    out_capacity bytes of records."""

    def __init__(self, specs: dict, budget_bytes: int, backend, slots: int = 2, max_records: int = 256,
                 max_samples: int = 16 << 20, idle_s: float = 0.5):
        self.specs = specs
        self.backend = backend
        self.slots = slots
        self.max_records = max_records
        self.max_samples = max_samples
        self.idle_s = idle_s
        self.budget = int(budget_bytes)
        # the largest single scan must fit a step
        big = max(specs.values(), key=lambda s: s.samples)
        self.max_samples = max(self.max_samples, big.samples)
        self.out_capacity = max(backend.record_bound(s) for s in specs.values())
        self.out_capacity = max(self.out_capacity, int(self.max_samples * 4.25) + 4096)
        self.fixed = backend.step_bytes(self.max_records, self.max_samples, self.out_capacity) * slots
        if self.fixed >= self.budget:
            # shrink the steps to a quarter of the budget, down to one scan of the largest stream
            per = self.budget // (4 * slots)
            s = big.samples
            while s * 2 <= self.max_samples and backend.step_bytes(
                    self.max_records, s * 2, int(s * 2 * 4.25) + 4096) <= per:
                s *= 2
            self.max_samples = s
            self.out_capacity = max(max(backend.record_bound(x) for x in specs.values()), int(s * 4.25) + 4096)
            self.fixed = backend.step_bytes(self.max_records, self.max_samples, self.out_capacity) * slots
        if self.fixed >= self.budget:
            raise ValueError(f"a budget of {self.budget} bytes cannot hold {slots} steps of one scan "
                             f"({self.fixed} bytes)")
        self.pool = Pool(self.budget - self.fixed)
        backend.setup(slots, self.max_records, self.max_samples, self.out_capacity, self.pool.capacity)
        self.open = {}       # sid -> pool offset of its state
        self.last_use = {}   # sid -> time of its last scan's arrival or completion
        self.session = collections.defaultdict(int)  # sid -> sessions opened so far
        self.results = collections.defaultdict(list)  # sid -> [(session, scan index, record bytes), ...]

    # -- admission --------------------------------------------------------
    def _admit(self, sid, st):
        if sid in self.open:
            return True
        spec = self.specs[sid]
        off = self.pool.alloc(self.backend.state_bytes(spec))
        if off is None:
            return False
        self.backend.open(sid, spec, off)
        self.open[sid] = off
        self.session[sid] += 1
        st.admissions += 1
        return True

    def _evict(self, sid, st):
        self.backend.close(sid)
        self.pool.release(self.open.pop(sid), self.backend.state_bytes(self.specs[sid]))
        st.evictions += 1

    def _choose(self, pending, busy):
        """Streams for the next step: heads of the pending queues, oldest
        first, one per stream, within the step limits."""
        heads = sorted((dq[0][0], sid) for sid, dq in pending.items() if dq and sid not in busy)
        batch, recs, samples, out = [], 0, 0, 0
        for _, sid in heads:
            s = self.specs[sid]
            rb = self.backend.record_bound(s)
            if batch and (recs + s.records > self.max_records or samples + s.samples > self.max_samples
                          or out + rb > self.out_capacity):
                break
            batch.append(sid)
            recs += s.records
            samples += s.samples
            out += rb
        return batch

    def run(self, arrivals, scan_of, speed: float = 1.0, keep_results=False):
        """arrivals: time-sorted (t, stream id, scan index), t in seconds of
        the sensors' clock; they are released at t / speed of wall time.
        scan_of(sid, k) returns the scan's per-attribute tensors (or a
        jiffy.PreparedScan of them), resident on the device before the run.
        keep_results: True, or a set of stream ids whose records are kept in
        self.results.  Returns ServeStats."""
        st = ServeStats(fixed_bytes=self.fixed, pool_bytes=self.pool.capacity)
        q = collections.deque()
        cv = threading.Condition()
        state = {"done": False}
        t0 = time.perf_counter() + 0.01

        def producer():
            for t, sid, k in arrivals:
                if state.get("stop"):
                    break
                due = t0 + t / speed
                d = due - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                with cv:
                    q.append((due, sid, k))
                    cv.notify()
            with cv:
                state["done"] = True
                cv.notify()

        if hasattr(self.backend, "begin"):
            self.backend.begin()
        th = threading.Thread(target=producer, daemon=True)
        th.start()
        pending = collections.OrderedDict()  # sid -> deque of (due, k)
        busy = set()
        inflight = collections.deque()       # (slot, [(sid, due, k, session)], t_submit)
        free = list(range(self.slots))
        seen = set()
        self._busy_until = t0
        try:
            while True:
                with cv:
                    incoming = list(q)
                    q.clear()
                    prod_done = state["done"]
                now = time.perf_counter()
                for due, sid, k in incoming:
                    seen.add(sid)
                    if not self._admit(sid, st):
                        st.scans_dropped += 1
                        continue
                    pending.setdefault(sid, collections.deque()).append((due, k))
                    self.last_use[sid] = due
                # idle streams give their state back
                for sid in [s for s in self.open if s not in busy and not pending.get(s)
                            and now - self.last_use.get(s, now) > self.idle_s]:
                    self._evict(sid, st)
                # the oldest step in flight, if it is done
                if inflight and self.backend.done(inflight[0][0]):
                    self._complete(inflight.popleft(), busy, free, st, keep_results)
                    continue
                if free:
                    batch = self._choose(pending, busy)
                    if batch:
                        slot = free.pop()
                        items = []
                        for sid in batch:
                            due, k = pending[sid].popleft()
                            items.append((sid, due, k, self.session[sid]))
                        t_sub = time.perf_counter()
                        if inflight:
                            st.overlap_steps += 1
                        self.backend.submit(slot, [i[0] for i in items], [scan_of(i[0], i[2]) for i in items])
                        busy.update(batch)
                        inflight.append((slot, items, t_sub))
                        st.batch_sizes.append(len(batch))
                        st.steps += 1
                        continue
                if inflight:
                    if not free:  # both contexts busy: wait for the oldest step
                        self._complete(inflight.popleft(), busy, free, st, keep_results)
                    else:         # a context is free but nothing can go yet: wait briefly for either
                        with cv:
                            if not q:
                                cv.wait(timeout=0.0002)
                    continue
                if prod_done and not any(pending.values()):
                    with cv:
                        if not q:
                            break
                    continue
                with cv:
                    if not q and not state["done"]:
                        cv.wait(timeout=0.002)
        finally:
            state["stop"] = True
            th.join()
            for slot, _, _ in inflight:
                self.backend.finish(slot)
        st.wall_s = time.perf_counter() - t0
        st.streams_seen = len(seen)
        st.pool_peak_bytes = self.pool.peak
        return st

    def _complete(self, entry, busy, free, st, keep_results):
        slot, items, t_sub = entry
        recs = self.backend.finish(slot)
        t_done = time.perf_counter()
        start = max(t_sub, self._busy_until)  # busy time: the union of the steps' submit-to-done spans
        if t_done > start:
            st.busy_s += t_done - start
        self._busy_until = max(self._busy_until, t_done)
        free.append(slot)
        for (sid, due, k, sess), r in zip(items, recs):
            busy.discard(sid)
            st.latencies_s.append(t_done - due)
            st.scans_done += 1
            st.points += self.specs[sid].samples
            self.last_use[sid] = t_done
            if keep_results is True or (keep_results and sid in keep_results):
                self.results[sid].append((sess, k, bytes(r)))

    def close(self):
        for sid in list(self.open):
            self.backend.close(sid)
            self.pool.release(self.open.pop(sid), self.backend.state_bytes(self.specs[sid]))
        self.backend.shutdown()

    @staticmethod
    def gpu(specs: dict, budget_bytes: int, **kw):
        """A server over libjiffy (GpuBackend)."""
        return Server(specs, budget_bytes, GpuBackend(), **kw)


class GpuBackend:
    """libjiffy: one jiffy_step per slot on its own HIP stream, a packed
    output buffer and a pinned host buffer per slot, and one device pool for
    the streams' resident states -- all allocated in setup()."""

    def state_bytes(self, spec):
        from . import jiffy
        return jiffy.stream_state_bytes(spec.height, spec.width, spec.widths)

    def record_bound(self, spec):
        from . import jiffy
        lay = jiffy.make_layout(spec.height, spec.width, spec.widths, spec.precisions)
        return jiffy.encode_bound(lay, 1) - (20 + 8 * lay.n_attrs + 4 * lay.n_attrs)

    def step_bytes(self, max_records, max_samples, out_capacity):
        from . import jiffy
        return jiffy.step_workspace_bytes(max_records, max_samples) + _al(out_capacity)

    def setup(self, slots, max_records, max_samples, out_capacity, pool_bytes):
        import torch

        from . import jiffy
        self.jiffy = jiffy
        self.steps = [jiffy.Step(max_records, max_samples) for _ in range(slots)]
        self.outs = [torch.empty(out_capacity, dtype=torch.uint8, device="cuda") for _ in range(slots)]
        self.host = [torch.empty(out_capacity, dtype=torch.uint8, pin_memory=True) for _ in range(slots)]
        self.hip = [torch.cuda.Stream() for _ in range(slots)]
        self.pool = torch.empty(max(pool_bytes, _ALIGN), dtype=torch.uint8, device="cuda")
        self.streams = {}
        self.inflight = {}

    def open(self, sid, spec, offset):
        n = self.state_bytes(spec)
        self.streams[sid] = self.jiffy.Stream(spec.height, spec.width, spec.widths, spec.precisions,
                                              state=self.pool[offset:offset + n])

    def close(self, sid):
        self.streams.pop(sid).close()

    def begin(self):
        # the scans are resident before serving starts (written on other streams): one wait here,
        # none per step
        import torch
        torch.cuda.synchronize()

    def submit(self, slot, sids, scans):
        self.steps[slot].submit([self.streams[s] for s in sids], scans, self.outs[slot], stream=self.hip[slot])
        self.inflight[slot] = len(sids)

    def done(self, slot):
        return self.hip[slot].query()

    def finish(self, slot):
        """Waits for the step; its records are then in the slot's pinned host
        buffer.  Returns one view per stream (valid until the slot's next
        step; bytes(view) keeps a copy)."""
        lens, _ = self.steps[slot].finish()
        total = int(sum(lens))
        host = self.host[slot]
        with __import__("torch").cuda.stream(self.hip[slot]):
            host[:total].copy_(self.outs[slot][:total], non_blocking=True)
        self.hip[slot].synchronize()
        buf = memoryview(host.numpy())
        out, p = [], 0
        for n in lens:
            out.append(buf[p:p + n])
            p += n
        self.inflight.pop(slot, None)
        return out

    def shutdown(self):
        for s in self.streams.values():
            s.close()
        self.streams.clear()
        for st in getattr(self, "steps", []):
            st.close()
