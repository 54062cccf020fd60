"""Host logic of the serving loop (no GPU): admission by the device-memory
budget with a state pool, one scan per stream per step in arrival order,
two steps in flight at once, idle streams closed and their memory reused,
wall-clock latencies.  The backend is a stand-in that records what it was
given and completes each step after a fixed delay."""
import threading
import time

import pytest

from paper_2209_08196_amd import serve
from paper_2209_08196_amd.serve import Pool, Server, StreamSpec


class FakeBackend:
    def __init__(self, delay=0.0):
        self.delay = delay
        self.log = []            # (slot, [(sid, k)], t_submit)
        self.opened = {}         # sid -> (offset, bytes)
        self.open_log = []       # (sid, offset)
        self.pending = {}
        self.max_pending = 0
        self.lock = threading.Lock()

    def state_bytes(self, spec):
        return spec.samples * 2 + 1000

    def record_bound(self, spec):
        return spec.samples * 4 + 100

    def step_bytes(self, max_records, max_samples, out_capacity):
        return max_samples * 5 + out_capacity

    def setup(self, slots, max_records, max_samples, out_capacity, pool_bytes):
        self.slots, self.limits, self.pool_bytes = slots, (max_records, max_samples, out_capacity), pool_bytes

    def open(self, sid, spec, offset):
        n = self.state_bytes(spec)
        assert sid not in self.opened
        assert offset + n <= self.pool_bytes
        for o, m in self.opened.values():  # states never overlap
            assert offset + n <= o or o + m <= offset
        self.opened[sid] = (offset, n)
        self.open_log.append((sid, offset))

    def close(self, sid):
        del self.opened[sid]

    def submit(self, slot, sids, scans):
        assert slot not in self.pending
        assert len(set(sids)) == len(sids)
        for s in sids:
            assert s in self.opened
        self.pending[slot] = (list(zip(sids, scans)), time.perf_counter())
        self.max_pending = max(self.max_pending, len(self.pending))
        self.log.append((slot, list(zip(sids, scans))))

    def done(self, slot):
        return time.perf_counter() - self.pending[slot][1] >= self.delay

    def finish(self, slot):
        items, t = self.pending.pop(slot)
        d = t + self.delay - time.perf_counter()
        if d > 0:
            time.sleep(d)
        return [f"{sid}:{k}".encode() for sid, k in items]

    def shutdown(self):
        pass


def _specs(n, shape=(16, 64), widths=(4, 2)):
    return {s: StreamSpec(shape[0], shape[1], widths, (1,) * len(widths)) for s in range(n)}


def test_pool_first_fit_and_coalescing():
    p = Pool(4096)
    a, b, c = p.alloc(1000), p.alloc(256), p.alloc(1)
    assert (a, b, c) == (0, 1024, 1280)
    p.release(b, 256)
    assert p.alloc(200) == 1024           # the hole is reused
    p.release(a, 1000)
    p.release(1024, 200)
    assert p.alloc(1280) == 0             # the two holes merged
    assert p.alloc(4096) is None
    assert p.peak <= 4096


def test_admission_by_budget_drops_what_does_not_fit():
    specs = _specs(6)
    fb = FakeBackend()
    one = fb.state_bytes(specs[0])
    # a budget with room for the steps and three stream states
    probe = Server(_specs(1), 1 << 40, FakeBackend())
    fixed = probe.fixed
    srv = Server(specs, fixed + 3 * serve._al(one) + 100, fb)
    arrivals = sorted([(0.002 * s + 0.004 * k, s, k) for s in range(6) for k in range(4)])
    st = srv.run(arrivals, lambda sid, k: k, keep_results=True)
    assert st.admissions == 3 and set(srv.results) == {0, 1, 2}
    assert st.scans_done == 12 and st.scans_dropped == 12
    for sid in range(3):  # every admitted scan, in order, exactly once
        assert [r for _, _, r in srv.results[sid]] == [f"{sid}:{k}".encode() for k in range(4)]
    assert st.pool_peak_bytes <= srv.pool.capacity <= srv.budget - srv.fixed
    srv.close()


def test_one_scan_per_stream_per_step_in_arrival_order():
    specs = _specs(3)
    fb = FakeBackend(delay=0.02)
    arrivals = [(0.0, 0, 0), (0.0, 0, 1), (0.0, 1, 0), (0.0, 2, 0), (0.0, 0, 2)]
    srv = Server(specs, 1 << 40, fb)
    st = srv.run(arrivals, lambda sid, k: k, keep_results=True)
    seq0 = [k for _, items in fb.log for s, k in items if s == 0]
    assert seq0 == [0, 1, 2]
    assert st.scans_done == 5 and sum(st.batch_sizes) == 5
    assert [r for _, _, r in srv.results[0]] == [b"0:0", b"0:1", b"0:2"]
    assert all(x >= 0 for x in st.latencies_s)
    srv.close()


def test_two_steps_in_flight_and_wall_clock_latency():
    """Steps take 20 ms; arrivals every 5 ms from four streams: while one
    step runs the next is submitted on the other context, never more than
    two are in flight, and latencies include the step time."""
    specs = _specs(4)
    fb = FakeBackend(delay=0.02)
    arrivals = sorted([(0.005 * i, i % 4, i // 4) for i in range(40)])
    srv = Server(specs, 1 << 40, fb, slots=2)
    st = srv.run(arrivals, lambda sid, k: k)
    assert st.scans_done == 40 and st.scans_dropped == 0
    assert fb.max_pending == 2
    assert st.overlap_steps > 0
    assert min(st.latencies_s) >= 0.02 * 0.9
    assert st.wall_s >= 0.2
    s = st.summary()
    assert s["mean_batch"] > 1 and 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    srv.close()


def test_idle_streams_give_their_memory_to_later_arrivals():
    """Two groups of streams in turn, with a budget for two states: the
    first group goes idle, is closed, and the second reuses its memory."""
    specs = _specs(4)
    fb = FakeBackend()
    probe = Server(_specs(1), 1 << 40, FakeBackend())
    one = serve._al(fb.state_bytes(specs[0]))
    srv = Server(specs, probe.fixed + 2 * one + 100, fb, idle_s=0.03)
    first = [(0.005 * k, s, k) for s in (0, 1) for k in range(3)]
    second = [(0.15 + 0.005 * k, s, k) for s in (2, 3) for k in range(3)]
    third = [(0.30, 0, 3)]  # stream 0 comes back: a new session
    st = srv.run(sorted(first + second + third), lambda sid, k: k, keep_results=True)
    assert st.scans_dropped == 0 and st.scans_done == 13
    assert st.evictions >= 2 and st.admissions == 5
    offs = {}
    for sid, off in fb.open_log:
        offs.setdefault(off, []).append(sid)
    assert any(len(v) > 1 for v in offs.values())  # a freed state was handed to another stream
    assert srv.session[0] == 2 and [(s, k) for s, k, _ in srv.results[0]] == [(1, 0), (1, 1), (1, 2), (2, 3)]
    srv.close()


def test_budget_too_small_for_one_step_is_refused():
    with pytest.raises(ValueError):
        Server(_specs(2), 1000, FakeBackend())
