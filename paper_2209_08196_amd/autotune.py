"""Autotuner of the batched encoder's launch configuration.

Candidates are the chain of kernels and the fused persistent launch at
1 .. N workgroups per compute unit (N: what one compute unit holds of the
fused kernel).  Each candidate encodes the same steps of the same streams
from the same starting state through a HIP-graph batch (jiffy_batch);
every candidate's records must equal the kernel chain's byte for byte, or
the candidate is rejected.  The fastest candidate (median step time) is
applied with jiffy_set_tuning and the result is kept in a JSON cache keyed
by the device and the batch's shape (stream sizes and widths), so that a
later process with the same batch skips the search.
"""
from __future__ import annotations

import json
import os
import statistics
import time

from . import jiffy

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "jiffy", "autotune.json")


def candidates(max_wgs_per_cu):
    out = [{"fused": 0, "wgs_per_cu": 0}]
    for w in range(1, max(1, max_wgs_per_cu) + 1):
        out.append({"fused": 1, "wgs_per_cu": w})
    return out


def signature(streams):
    """The batch's shape: every stream's height, width, sample widths and precisions."""
    parts = []
    for s in streams:
        lay = s.layout
        parts.append(f"{lay.height}x{lay.width}:" + ",".join(
            f"{lay.width_bytes[a]}/{lay.precision[a]}" for a in range(lay.n_attrs)))
    return ";".join(parts)


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _run(make_streams, scans, steps, tuning):
    """Encodes `steps` steps with `tuning`; -> (step seconds list, records
    per step as bytes)."""
    import torch
    jiffy.set_tuning(**tuning)
    streams = make_streams()
    outs = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in streams]
    batch = jiffy.Batch(streams, scans[0], outs)
    times, recs = [], []
    try:
        for t in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lens, _ = batch.run(scans[t])
            times.append(time.perf_counter() - t0)
            recs.append(b"".join(o[:n].cpu().numpy().tobytes() for o, n in zip(outs, lens)))
    finally:
        batch.close()
        for s in streams:
            s.close()
    return times, recs


def tune(make_streams, scans, steps=None, cache=DEFAULT_CACHE, force=False, log=None):
    """make_streams() -> a fresh list of jiffy.Stream (same layouts each
    call); scans[t][i] -> stream i's scan of step t (prepared scans or
    tensor lists).  Returns the report dict; the best tuning is applied."""
    import torch
    steps = steps or len(scans)
    probe = make_streams()
    sig = signature(probe)
    for s in probe:
        s.close()
    dev = _device_name()
    key = f"{dev}|{sig}"
    db = {}
    if cache and os.path.exists(cache):
        try:
            db = json.load(open(cache))
        except (OSError, ValueError):
            db = {}
    if not force and key in db:
        best = db[key]["best"]
        jiffy.set_tuning(**best)
        return dict(db[key], cached=True)
    _, max_wgs = jiffy.get_tuning()
    ref = None
    results = []
    for cand in candidates(max_wgs):
        times, recs = _run(make_streams, scans, steps, cand)
        same = ref is None or recs == ref
        if ref is None:
            ref = recs
        med = statistics.median(times[1:] if len(times) > 1 else times)
        results.append({"tuning": cand, "median_ms": round(1e3 * med, 4), "byte_identical": same})
        if log:
            log(f"autotune {cand}: {1e3 * med:.3f} ms/step, byte-identical {same}")
    ok = [r for r in results if r["byte_identical"]]
    best = min(ok, key=lambda r: r["median_ms"])["tuning"]
    jiffy.set_tuning(**best)
    torch.cuda.synchronize()
    report = {"device": dev, "signature_streams": len(sig.split(";")), "steps": steps, "candidates": results,
              "best": best}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db[key] = report
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return dict(report, cached=False)
