"""Continuous-batching encode server over many sensor streams.

Scans arrive from many sensors at their own rates; every step the server
encodes the scans that have arrived, at most one per stream, in one batched
call (jiffy_batch_encode_step), each stream predicting from its own resident
previous scan (Sec. III-D).  A stream's records are therefore exactly those
of encoding its scan sequence alone.

Device memory is bounded by a budget: a stream is admitted when its
resident state (two halves of quantized samples and valid words, and its
output buffer) fits next to the streams already admitted and the encoder
workspace reserved for one step; a stream that does not fit is rejected and
its scans are counted as dropped.  Steps take arrived scans in arrival
order while their encoder workspace fits the reserve.

Time is virtual: arrivals follow their timestamps, and each step advances
the clock by its measured duration (submit to records on the host), so the
reported latency (completion minus arrival) is what a server with this
throughput would show under that arrival process.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

_SLOT_BYTES = 576      # device bytes per frame slot of the encoder
_FRAME = 128
_FTILE = 8192
_ALIGN = 256
_WS_GROWTH = 1.25      # the library grows its workspace by a quarter over the need


def _al(x):
    return (x + _ALIGN - 1) // _ALIGN * _ALIGN


def state_bytes(height, width, widths):
    """Device bytes a stream keeps resident: two halves of quantized
    samples (each padded by 16 bytes) and of 64-pixel valid words."""
    npx = height * width
    nwords = (npx + 63) // 64
    return sum(2 * (npx * w + 16) + 2 * 8 * nwords for w in widths)


def record_bound(height, width, widths):
    """Worst-case bytes of one scan's records (the output buffer)."""
    npx = height * width
    nm = (npx + 7) // 8
    nb = (npx + _FRAME - 1) // _FRAME
    total = 0
    for w in widths:
        frame = 16 + nm + 4 * (nm // 131072 + 1)
        total += 12 + frame + 3 + 4 + 3 * nb + 3 + nb * 16 * 8 * w + 3
    return total


def workspace_bytes(height, width, widths):
    """Encoder workspace of one scan (all its attributes) in a batched step."""
    npx = height * width
    nwords = (npx + 63) // 64
    maxnb = (npx + _FRAME - 1) // _FRAME
    nm = (npx + 7) // 8
    nft = (npx + _FTILE - 1) // _FTILE
    per_attr = (_al(16 * maxnb + 4 * nft) + _al(8 * nft + 4) + _al(_SLOT_BYTES * maxnb)
                + _al(16 + nm + 4 * (nm // 131072 + 1)) + _al(8 * (nm // 4 + 4)) + _al(8 * nwords) + 512 + 8 * (nft + 1))
    return len(widths) * per_attr + 1024


@dataclasses.dataclass
class StreamSpec:
    height: int
    width: int
    widths: tuple
    precisions: tuple


@dataclasses.dataclass
class ServeStats:
    scans_done: int = 0
    scans_dropped: int = 0
    streams_admitted: int = 0
    streams_rejected: int = 0
    steps: int = 0
    points: int = 0
    busy_s: float = 0.0
    sim_end_s: float = 0.0
    resident_bytes: int = 0
    latencies_s: list = dataclasses.field(default_factory=list)
    batch_sizes: list = dataclasses.field(default_factory=list)

    def summary(self):
        lat = np.asarray(self.latencies_s) if self.latencies_s else np.zeros(1)
        return {
            "scans": self.scans_done, "dropped_scans": self.scans_dropped,
            "streams_admitted": self.streams_admitted, "streams_rejected": self.streams_rejected,
            "steps": self.steps, "mean_batch": round(float(np.mean(self.batch_sizes)) if self.batch_sizes else 0, 2),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "max_ms": round(1e3 * float(lat.max()), 3),
            "points_per_s_busy": round(self.points / self.busy_s, 1) if self.busy_s else 0.0,
            "points_per_s_offered": round(self.points / self.sim_end_s, 1) if self.sim_end_s else 0.0,
            "resident_bytes": self.resident_bytes,
        }


class Server:
    """budget_bytes: device bytes the server may use (resident stream
    states, output buffers, the encoder workspace of one step).
    encode_step(stream_ids, scans) -> list of bytes objects (one per stream)
    is the batched encoder; Server.gpu() builds the one over libjiffy."""

    def __init__(self, specs: dict, budget_bytes: int, encode_step, max_batch: int = 256, on_admit=None):
        self.specs = specs
        self.on_admit = on_admit  # called with a stream id when it is admitted (resident state set up)
        self.budget = int(budget_bytes)
        self.encode_step = encode_step
        self.max_batch = max_batch
        self.admitted = set()
        self.rejected = set()
        self.resident = 0
        # the workspace reserve: the largest single scan's need, grown as the library grows
        self.ws_reserve = int(_WS_GROWTH * max(workspace_bytes(s.height, s.width, s.widths)
                                              for s in specs.values()))
        self.results = collections.defaultdict(list)  # stream id -> list of record bytes

    def _stream_cost(self, sid):
        s = self.specs[sid]
        return state_bytes(s.height, s.width, s.widths) + record_bound(s.height, s.width, s.widths)

    def admit(self, sid):
        if sid in self.admitted:
            return True
        if sid in self.rejected:
            return False
        need = self._stream_cost(sid)
        if self.resident + need + self.ws_reserve <= self.budget:
            self.admitted.add(sid)
            self.resident += need
            if self.on_admit:
                self.on_admit(sid)
            return True
        self.rejected.add(sid)
        return False

    def _ws_available(self):
        return max(0, int((self.budget - self.resident) / _WS_GROWTH))

    def run(self, arrivals, scan_of, keep_results=False):
        """arrivals: time-sorted (t, stream id, scan index); scan_of(sid, k)
        returns the scan's per-attribute device tensors.  keep_results: True,
        or a set of stream ids whose records are kept in self.results.
        Returns ServeStats."""
        st = ServeStats()
        pending = collections.OrderedDict()  # sid -> deque of (t, k)
        queue = collections.deque(arrivals)
        clock = 0.0
        while queue or any(pending.values()):
            if not any(pending.values()):
                clock = max(clock, queue[0][0])
            while queue and queue[0][0] <= clock:
                t, sid, k = queue.popleft()
                if not self.admit(sid):
                    st.scans_dropped += 1
                    continue
                pending.setdefault(sid, collections.deque()).append((t, k))
            # one scan per stream, oldest arrivals first, while the workspace fits
            heads = sorted((dq[0][0], sid) for sid, dq in pending.items() if dq)
            ws_left = self._ws_available()
            batch = []
            for t, sid in heads:
                s = self.specs[sid]
                w = workspace_bytes(s.height, s.width, s.widths)
                if batch and (w > ws_left or len(batch) >= self.max_batch):
                    break
                ws_left -= w
                batch.append(sid)
            if not batch:  # every scan that arrived was dropped
                continue
            items = [(sid, pending[sid].popleft()) for sid in batch]
            t0 = time.perf_counter()
            recs = self.encode_step(batch, [scan_of(sid, k) for sid, (t, k) in items])
            d = time.perf_counter() - t0
            clock += d
            st.busy_s += d
            st.steps += 1
            st.batch_sizes.append(len(batch))
            for (sid, (t, k)), r in zip(items, recs):
                st.latencies_s.append(clock - t)
                st.scans_done += 1
                s = self.specs[sid]
                st.points += s.height * s.width * len(s.widths)
                if keep_results is True or (keep_results and sid in keep_results):
                    self.results[sid].append(r)
        st.sim_end_s = max(clock, arrivals[-1][0] if arrivals else 0.0)
        st.streams_admitted = len(self.admitted)
        st.streams_rejected = len(self.rejected)
        st.resident_bytes = self.resident
        return st

    @staticmethod
    def gpu(specs: dict, budget_bytes: int, max_batch: int = 256):
        """A server over libjiffy: one jiffy_stream per admitted stream and a
        device output buffer each; records are copied to the host."""
        import torch

        from . import jiffy
        streams, outs = {}, {}

        def on_admit(sid):  # the stream's resident state and output buffer
            s = specs[sid]
            streams[sid] = jiffy.Stream(s.height, s.width, s.widths, s.precisions)
            outs[sid] = torch.empty(streams[sid].record_bound(), dtype=torch.uint8, device="cuda")

        def encode_step(sids, scans):
            lens, _ = jiffy.batch_encode_step([streams[s] for s in sids], scans, [outs[s] for s in sids])
            host = [outs[s][:n].to("cpu", non_blocking=True) for s, n in zip(sids, lens)]
            torch.cuda.synchronize()
            return [h.numpy().tobytes() for h in host]

        srv = Server(specs, budget_bytes, encode_step, max_batch, on_admit)
        srv._streams = streams
        return srv

    def close(self):
        for s in getattr(self, "_streams", {}).values():
            s.close()
