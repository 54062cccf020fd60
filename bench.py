#!/usr/bin/env python3
"""Encode+decode throughput of the Jiffy codec on one MI355X.

Headline workload (the largest configuration that fits one GPU): the
stress set, 32 independent sensor streams of 200 scans of 128x4096 range
samples (u32, millimetres, precision 1 mm), 60% zero samples in blobs,
drone-like motion of 5-15 degrees per scan and a scene cut every 20 scans,
seeded synthetic data standing in for the paper's recordings.  Each
stream's first 20-scan scene period is generated on the host and replayed
ten times on the device (scan 20k+i equals scan i; every 20th scan still
follows a different view, so it is a scene cut).  One step encodes every
stream's 200 scans and decodes every stream back, each in one launch
sequence over all streams (jiffy_encode_many, jiffy_decode_many); inputs
and outputs stay in device memory.  The same step is also timed as one
jiffy_encode and one jiffy_decode_layout call per stream
(`per_stream_calls`), whose streams must be the same bytes.  A point is one pixel of one attribute, as in the paper's points/s
(Sec. IV-F).

Further legs (each skippable):
  batched   the 64-stream batched set (16x1024 .. 128x2048, range at 1 cm
            and signal), one scan of every stream per step: the plain
            one-scan-per-launch codec, the batched step and the
            graph-replayed batch, byte-identical records required, with the
            batched step's own roofline;
  serving   the 256-stream serving set under device-memory budgets;
  cpu       the oracle on a bounded sample of the headline workload, one
            thread and all host cores, its streams compared byte for byte
            with the ones the timed GPU encoder wrote.

Prints one JSON line.  `roofline`: the dominant kernel's algorithmic bytes
per launch (input samples, previous scans of P-records, compressed bytes)
over its mean launch time (HIP events on the launch stream) against the
8 TB/s HBM peak; `traffic` is the HBM bytes measured with rocprofv3 counters
for the same kernel source and workload (or null).
"""
import argparse
import hashlib
import json
import os
import struct
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encode+decode points/sec & HBM GB/s fraction at byte-identical output"
HBM_PEAK_GBS = 8000.0
HEAD_CID = 5       # the stress set: 32 streams x 200 scans of 128x4096
SCENE_PERIOD = 20  # scans per scene of the stress set (the part that is generated)
SERVING_CYCLE = 4  # distinct synthetic scans per serving stream (cycled)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2209_08196_amd", "csrc", f)
                  for f in ("jiffy_encode.hip", "jiffy_decode.hip", "jiffy_standardize.hip", "jiffy_device.h",
                            "jiffy_internal.h")]
_STORE = {1: np.uint8, 2: np.int16, 4: np.int32}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def pool_size():
    """Host threads for the oracle's all-core leg (the GPU machine's share is 16 cores)."""
    return max(1, min(16, os.cpu_count() or 1))


def gen_procs():
    """Processes that generate inputs: at most 8, so that a run under a
    profiler (which initializes the GPU in the parent before the fork) stays
    well below the number of processes that may use one GPU."""
    return max(1, min(8, os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# synthetic inputs (generated in worker processes before the GPU is touched)
# ---------------------------------------------------------------------------
def _gen(job):
    from paper_2209_08196_amd import synth
    cid, sid, t0, t1, *rest = job
    return synth.stream(cid, sid, standing=bool(rest and rest[0])).scans(t0, t1)


def generate(jobs):
    """Scan arrays for (cid, stream, t0, t1) jobs, in a process pool."""
    n = gen_procs()
    if n == 1 or len(jobs) == 1:
        return [_gen(j) for j in jobs]
    return _pool_map(_gen, jobs, min(n, len(jobs)), 1)


def _pool_map(fn, jobs, procs, chunksize):
    """map over forked worker processes that finish normally (close and join:
    a terminated worker would run the signal handlers it inherited, such as
    a profiler's, in the child)."""
    import multiprocessing as mp
    pool = mp.get_context("fork").Pool(procs)
    try:
        out = pool.map(fn, jobs, chunksize=chunksize)
    finally:
        pool.close()
        pool.join()
    return out


def _cloud(args):
    from paper_2209_08196_amd import synth
    t, rng_img, attr_imgs = args
    return synth.cartesian_scan(np.random.default_rng([2, t]), rng_img, attr_imgs)[:2]


def generate_clouds(dual):
    """Cartesian clouds of the dual-return stream's range scans, each point
    carrying signal, reflectivity and near-IR (in a process pool)."""
    T = dual[0].shape[0]
    jobs = [(t, dual[0][t], [dual[2][t], dual[3][t], dual[4][t]]) for t in range(T)]
    return _pool_map(_cloud, jobs, min(gen_procs(), T), 4)


# ---------------------------------------------------------------------------
# stream statistics (from the stream's own headers)
# ---------------------------------------------------------------------------
def stream_stats(s: bytes, widths, npx, precisions):
    A, = struct.unpack_from("<H", s, 6)
    T, = struct.unpack_from("<I", s, 16)
    p = 20 + 8 * A
    lens = struct.unpack_from(f"<{T * A}I", s, p)
    p += 4 * T * A
    st = dict(mask_bytes=0, frame_bytes=0, n_values=0, p_items=0, p_bytes=0, i_items=0, x_bytes=0)
    for r, L in enumerate(lens):
        a = r % A
        mode = s[p + 4]
        flen, = struct.unpack_from("<I", s, p + 8)
        sec = (12 + flen + 3) & ~3
        N, = struct.unpack_from("<I", s, p + sec)
        nb = (N + 127) // 128
        b = np.frombuffer(s, np.uint8, nb, p + sec + 4).astype(np.int64)
        n = np.frombuffer(s, np.uint8, nb, p + sec + 4 + nb).astype(np.int64)
        B = np.frombuffer(s, np.uint8, nb, p + sec + 4 + 2 * nb).astype(np.int64)
        st["frame_bytes"] += int((16 * b + n + (n * (B - b) + 7) // 8).sum())
        st["mask_bytes"] += flen
        st["n_values"] += N
        st["x_bytes"] += widths[a] * npx
        if mode == 1:
            st["p_items"] += 1
            st["p_bytes"] += widths[a] * npx
        else:
            st["i_items"] += 1
        p += L
    st["stream_bytes"] = len(s)
    return st


def add_stats(stats):
    out = {}
    for st in stats:
        for k, v in st.items():
            out[k] = out.get(k, 0) + v
    return out


def split_records(s: bytes):
    """The records of a stream with a record-length table."""
    A, = struct.unpack_from("<H", s, 6)
    T, = struct.unpack_from("<I", s, 16)
    p = 20 + 8 * A
    lens = struct.unpack_from(f"<{T * A}I", s, p)
    p += 4 * T * A
    out = []
    for L in lens:
        out.append(s[p:p + L])
        p += L
    return out


def record_stats(recs, widths, npx, precisions):
    """As stream_stats, for a list of records of one scan each (attribute order)."""
    st = dict(p_items=0, p_bytes=0, i_items=0, x_bytes=0, q_bytes=0, stream_bytes=0)
    for k, r in enumerate(recs):
        a = k % len(widths)
        st["x_bytes"] += widths[a] * npx
        st["stream_bytes"] += len(r)
        if precisions[a] > 1:
            st["q_bytes"] += widths[a] * npx
        if r[4] == 1:
            st["p_items"] += 1
            st["p_bytes"] += widths[a] * npx
        else:
            st["i_items"] += 1
    return st


def kernel_profile(run, reps):
    """Per-kernel mean launch times (HIP events on the launch stream) over
    `reps` calls of run()."""
    import torch
    from paper_2209_08196_amd import jiffy
    torch.cuda.synchronize()
    jiffy.profile_enable(True)
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    prof = jiffy.profile_read()
    jiffy.profile_enable(False)
    return {k: dict(avg_ms=v[0] / v[1], launches=v[1]) for k, v in prof.items()}


def roofline(kernels, alg_per_launch, workload):
    """The roofline object of the dominant kernel: algorithmic bytes per
    launch (encode: samples in + previous scans of P-records + compressed
    bytes out) over its mean launch time."""
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    alg = alg_per_launch(dom)
    avg_s = kernels[dom]["avg_ms"] / 1e3
    achieved = alg / avg_s / 1e9 if alg else None
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        ent = tr.get("workloads", {}).get(workload, {}).get("kernels", {}).get(dom)
        if ent and tr.get("source_sha") == source_sha():
            traffic = ent["fetch_bytes"] + ent["write_bytes"]
    return {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic, "kernel": dom, "alg_bytes_per_launch": alg,
            "avg_launch_ms": round(kernels[dom]["avg_ms"], 4)}


# ---------------------------------------------------------------------------
# headline: the stress set, encode + decode of whole streams
# ---------------------------------------------------------------------------
def headline(args, host_period):
    import torch

    from paper_2209_08196_amd import jiffy, synth
    cfg = synth.CONFIGS[HEAD_CID]
    S = len(host_period) if args.streams is None else min(args.streams, len(host_period))
    T = cfg.scans
    reps = T // SCENE_PERIOD
    g0 = synth.stream(HEAD_CID, 0)
    H, W, widths, precs = g0.H, g0.W, g0.widths, g0.precisions
    A = len(widths)
    npx = H * W
    lay = jiffy.make_layout(H, W, widths, precs)
    bound = jiffy.encode_bound(lay, T)
    dev, outs, decs = [], [], []
    stream = torch.cuda.current_stream()
    for s in range(S):
        per = [torch.from_numpy(p.view(_STORE[p.dtype.itemsize])).cuda() for p in host_period[s]]
        dev.append([p.repeat(reps, 1, 1).contiguous() for p in per])
        outs.append(torch.empty(bound, dtype=torch.uint8, device="cuda"))
        decs.append([torch.empty_like(d) for d in dev[-1]])
    log(f"headline: {S} streams x {T} scans of {H}x{W} resident ({S * T * npx * 4 / 1e9:.1f} GB of samples)")
    points = S * T * npx * A
    # the step: every stream's records in one encode launch sequence, then one decode launch sequence
    encm = jiffy.EncoderMany(dev, precs, outs=outs, stream=stream)
    decm = jiffy.DecoderMany(lay, T, outs, decs, stream=stream)

    def step():
        bs, m = encm()
        decm(encm.lengths)
        return bs, m

    def timed(run_enc, run_dec, steps):
        """Wall time of `steps` steps, and encode / decode time from events on the launch stream."""
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for ev in evs:
            ev[0].record(stream)
            run_enc()
            ev[1].record(stream)
            run_dec()
            ev[2].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return (wall, sum(ev[0].elapsed_time(ev[1]) for ev in evs), sum(ev[1].elapsed_time(ev[2]) for ev in evs))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    wall, enc_ms, dec_ms = timed(encm, lambda: decm(encm.lengths), args.steps)
    ms_per_step = 1e3 * wall / args.steps
    log(f"headline: {args.steps} steps, {ms_per_step:.2f} ms/step")

    # the outputs of the last timed step: lossless round trip (precision 1)
    lens = encm.lengths
    streams_host = [outs[s][:lens[s]].cpu().numpy().tobytes() for s in range(S)]
    modes_all = [encm._modes[s].copy() for s in range(S)]

    def check_round_trip(what):
        for s in range(S):
            for d, x in zip(decs[s], dev[s]):
                if not torch.equal(d, x):
                    raise SystemExit(f"{what}: stream {s}: decode(encode(x)) != x")

    check_round_trip("many-stream calls")
    stats = add_stats(stream_stats(b, widths, npx, precs) for b in streams_host)
    x_bytes = stats["x_bytes"]
    log(f"headline: {stats['stream_bytes']} bytes, ratio {x_bytes / stats['stream_bytes']:.2f}, "
        f"P-records {stats['p_items']} of {stats['p_items'] + stats['i_items']}")

    # the same step as one jiffy_encode and one jiffy_decode_layout call per stream: same bytes
    per_stream = None
    if args.per_stream_steps > 0:
        encs = [jiffy.Encoder(dev[s], precs, out=outs[s], stream=stream) for s in range(S)]
        dcds = [jiffy.Decoder(lay, T, decs[s], stream=stream) for s in range(S)]
        res1 = [None] * S

        def enc1():
            for s in range(S):
                res1[s] = encs[s]()

        def dec1():
            for s in range(S):
                dcds[s](res1[s][0])

        for d in decs:
            for t in d:
                t.zero_()
        enc1()
        dec1()
        w1, e1, d1 = timed(enc1, dec1, args.per_stream_steps)
        for s in range(S):
            if res1[s][0].cpu().numpy().tobytes() != streams_host[s] or not np.array_equal(res1[s][1], modes_all[s]):
                raise SystemExit(f"stream {s}: jiffy_encode and jiffy_encode_many wrote different streams")
        check_round_trip("per-stream calls")
        n1 = args.per_stream_steps
        per_stream = {"points_per_s": round(points / (w1 / n1), 1), "ms_per_step": round(1e3 * w1 / n1, 3),
                      "encode_points_per_s": round(points / (e1 / n1 / 1e3), 1),
                      "decode_points_per_s": round(points / (d1 / n1 / 1e3), 1), "steps": n1,
                      "same_bytes": True}
        log(f"headline per-stream calls: {1e3 * w1 / n1:.2f} ms/step")
        del encs, dcds, res1

    kernels = {}
    if args.profile_steps > 0:
        kernels = kernel_profile(step, args.profile_steps)

    def alg(name):  # per launch: every launch covers every stream's records
        if name.startswith("k_enc") or name.startswith("k_dec"):
            return stats["x_bytes"] + stats["p_bytes"] + stats["stream_bytes"]
        return None

    path_alg = 2 * (x_bytes + stats["p_bytes"] + stats["stream_bytes"])
    result = {
        "metric": METRIC, "value": round(points / (wall / args.steps), 1), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"stress-128x4096-drone-range-1mm: {S} streams x {T} scans of {H}x{W} range u32, "
                               f"precision 1 mm, 60% zeros, 5-15 deg/scan, scene cut every {SCENE_PERIOD} scans "
                               f"(each stream's first {SCENE_PERIOD}-scan period generated and replayed {reps}x); "
                               "encode+decode of every stream per step (one jiffy_encode_many and one "
                               "jiffy_decode_many call)",
                   "streams": S, "scans": T, "height": H, "width": W, "attributes": ["range"], "precision_mm": 1},
        "encode_points_per_s": round(points / (enc_ms / args.steps / 1e3), 1),
        "decode_points_per_s": round(points / (dec_ms / args.steps / 1e3), 1),
        "compression_ratio": round(x_bytes / stats["stream_bytes"], 3),
        "p_records": stats["p_items"], "i_records": stats["i_items"],
        "path_alg_gbps": round(path_alg / (wall / args.steps) / 1e9, 1),
        "path_hbm_frac": round(path_alg / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
    }
    if per_stream:
        result["per_stream_calls"] = per_stream
    if kernels:
        result["roofline"] = roofline(kernels, alg, "stress")
        result["kernels_ms"] = {k: round(v["avg_ms"], 4)
                                for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["avg_ms"])}
    ctx = dict(streams=streams_host, modes=modes_all, S=S, T=T, precs=precs)
    # free the device buffers of this leg before the next
    del dev, outs, decs, encm, decm
    torch.cuda.empty_cache()
    return result, ctx


# ---------------------------------------------------------------------------
# batched: 64 streams, one scan each per step
# ---------------------------------------------------------------------------
def batched_leg(host, steps, warmup):
    """host[s]: stream s's scans (list per attribute of [T, H, W]).  Every
    step encodes one scan of every stream three ways on twin streams:
    one jiffy_batch_encode_step per stream (the plain one-scan-per-launch
    codec), one jiffy_batch_encode_step over all 64, and one replay of the
    batch's HIP graph (jiffy_batch_run).  Records must be identical."""
    import torch

    from paper_2209_08196_amd import jiffy, synth
    cfg = synth.CONFIGS[3]
    gens = [synth.stream(3, s) for s in range(len(host))]
    T = warmup + steps
    scans = [[torch.from_numpy(p[:T].view(_STORE[p.dtype.itemsize])).cuda() for p in h] for h in host]
    # each step's scan tensors checked once (the timed calls pass their pointers)
    prep = [[jiffy.PreparedScan(g.H, g.W, g.widths, [p[t] for p in sc]) for g, sc in zip(gens, scans)]
            for t in range(T)]
    points = sum(g.H * g.W * len(g.widths) for g in gens)
    mk = lambda: [jiffy.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]  # noqa: E731
    # the launch configuration of the batched step: the autotuner's choice on the first steps
    from paper_2209_08196_amd import autotune
    nt = min(T, 6)
    tune = autotune.tune(mk, prep[:nt], cache=None, log=log)
    chain = {"fused": 0, "wgs_per_cu": 0}
    s1, sb, sg = mk(), mk(), mk()
    mko = lambda ss: [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in ss]  # noqa: E731
    o1, ob, og = mko(s1), mko(sb), mko(sg)
    jiffy.set_tuning(**tune["best"])  # the graph captures the tuned configuration
    batch = jiffy.Batch(sg, [[p[0] for p in sc] for sc in scans], og)
    identical = True
    t1 = tb = tg = 0.0
    for t in range(T):
        at = prep[t]
        torch.cuda.synchronize()
        jiffy.set_tuning(**chain)  # the plain codec: the kernel chain, one scan per call
        a = time.perf_counter()
        l1 = [jiffy.batch_encode_step([s1[i]], [at[i]], [o1[i]])[0][0] for i in range(len(gens))]
        b = time.perf_counter()
        jiffy.set_tuning(**tune["best"])
        lb, _ = jiffy.batch_encode_step(sb, at, ob)
        c = time.perf_counter()
        lg, _ = batch.run(at)
        d = time.perf_counter()
        if t >= warmup:
            t1 += b - a
            tb += c - b
            tg += d - c
        for i in range(len(gens)):
            if not (l1[i] == lb[i] == lg[i] and torch.equal(o1[i][:l1[i]], ob[i][:lb[i]])
                    and torch.equal(ob[i][:lb[i]], og[i][:lg[i]])):
                identical = False
    log(f"batched: one-scan-per-launch {1e3 * t1 / steps:.3f} ms, batched {1e3 * tb / steps:.3f} ms, "
        f"graph {1e3 * tg / steps:.3f} ms per step")
    # per-kernel times of the batched step: the same steps again on fresh twin streams, with HIP
    # events around every launch from the first timed step on; the algorithmic bytes of those steps
    # come from their records
    sp = mk()
    op = mko(sp)
    rs = []
    for t in range(T):
        if t == warmup:
            torch.cuda.synchronize()
            jiffy.profile_enable(True)
        lp, _ = jiffy.batch_encode_step(sp, prep[t], op)
        if t >= warmup:
            for i, g in enumerate(gens):
                buf = op[i][:lp[i]].cpu().numpy().tobytes()
                recs, p = [], 0
                for _ in range(len(g.widths)):
                    L, = struct.unpack_from("<I", buf, p)
                    recs.append(buf[p:p + L])
                    p += L
                rs.append(record_stats(recs, g.widths, g.H * g.W, g.precisions))
    torch.cuda.synchronize()
    prof = jiffy.profile_read()
    jiffy.profile_enable(False)
    kernels = {k: dict(avg_ms=v[0] / v[1], launches=v[1]) for k, v in prof.items()}
    st = add_stats(rs)
    # per step: samples in, previous scans of P-records, quantized state of P > 1 attributes, records out
    alg_step = (st["x_bytes"] + st["p_bytes"] + st["q_bytes"] + st["stream_bytes"]) // steps
    rl = roofline(kernels, lambda name: alg_step if name.startswith("k_enc") else None, "batched")
    for s in sp:
        s.close()
    jiffy.set_tuning(**chain)
    batch.close()
    for s in s1 + sb + sg:
        s.close()
    torch.cuda.empty_cache()
    return {"workload": f"{cfg.name}: 64 streams (16 each of 16x1024, 32x2048, 64x1024, 128x2048), range u32 "
                        f"at 1 cm + signal u16, one scan per stream per step, {steps} timed steps",
            "streams": len(gens), "points_per_step": points,
            "batched_points_per_s": round(points * steps / tb, 1), "batched_ms_per_step": round(1e3 * tb / steps, 3),
            "graph_points_per_s": round(points * steps / tg, 1), "graph_ms_per_step": round(1e3 * tg / steps, 3),
            "one_scan_per_launch_points_per_s": round(points * steps / t1, 1),
            "one_scan_per_launch_ms_per_step": round(1e3 * t1 / steps, 3),
            "alg_bytes_per_step": alg_step,
            "path_alg_gbps": round(alg_step * steps / tb / 1e9, 1),
            "byte_identical": identical, "roofline": rl,
            "autotune": {"best": tune["best"], "candidates": tune["candidates"]},
            "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["avg_ms"])}}


# ---------------------------------------------------------------------------
# serving: 256 streams under device-memory budgets
# ---------------------------------------------------------------------------
def serving_leg(host, duration_s, speed_loaded=8.0):
    """256 sensor streams (32x1024 .. 128x2048, range u32 and three u16
    attributes at 1 mm; 10 or 20 Hz each with random phase and Poisson
    jitter), served in real time by continuous batching over two step
    contexts: under 8 GiB at the sensors' rate, under 8 GiB with arrivals
    `speed_loaded` times faster (the server saturated), under 8 GiB with
    every arrival released at once (a burst: full steps back to back, the
    two contexts' steps overlapping on the device), and under 64 MiB with
    sensors connecting for 1-3 s sessions (admission binds, idle streams'
    memory is reused).  host[s]: stream s's distinct synthetic
    scans, cycled.  Stream 0's records from the first run are compared with
    its sequence encoded alone by jiffy_encode."""
    import torch

    from paper_2209_08196_amd import jiffy, serve, synth
    cfg = synth.CONFIGS[4]
    gens = [synth.stream(4, s) for s in range(len(host))]
    ncyc = host[0][0].shape[0]
    dev = [[torch.from_numpy(p.view(_STORE[p.dtype.itemsize])).cuda() for p in h] for h in host]
    specs = {s: serve.StreamSpec(g.H, g.W, tuple(g.widths), tuple(g.precisions)) for s, g in enumerate(gens)}
    # every cycled scan's tensors checked once against its stream's layout
    prepared = [[jiffy.PreparedScan(g.H, g.W, g.widths, [p[k] for p in dev[s]]) for k in range(ncyc)]
                for s, g in enumerate(gens)]
    scan_of = lambda sid, k: prepared[sid][k % ncyc]  # noqa: E731
    out = {"workload": f"{cfg.name}: {len(host)} streams (sizes 32x1024, 64x1024, 64x2048, 128x2048; range u32 + "
                       f"3 x u16 at 1 mm), 10/20 Hz with Poisson(2 ms) jitter, {duration_s} s of arrivals, each "
                       f"stream cycling {ncyc} synthetic scans; real-time serving on two step contexts"}
    runs = [("nominal_8192MiB", 8 << 30, 1.0, None), ("loaded_x%g_8192MiB" % speed_loaded, 8 << 30, speed_loaded, None),
            ("burst_8192MiB", 8 << 30, 1e6, None), ("sessions_64MiB", 64 << 20, 1.0, (1.0, 3.0))]
    for name, budget, speed, sess in runs:
        arrivals = synth.serving_arrivals(len(host), duration_s, session_s=sess)
        keep = {arrivals[0][1]} if name.startswith("nominal") else False
        srv = serve.Server.gpu(specs, budget)
        st = srv.run(arrivals, scan_of, speed=speed, keep_results=keep)
        res = st.summary()
        res["scans_offered"] = len(arrivals)
        res["speed"] = speed
        if keep:
            sid = arrivals[0][1]
            ks = [k for _, s, k in arrivals if s == sid]
            g = gens[sid]
            seq = [torch.stack([dev[sid][a][k % ncyc] for k in ks]).contiguous() for a in range(len(g.widths))]
            alone, _ = jiffy.encode(seq, g.precisions)
            want = split_records(alone.cpu().numpy().tobytes())
            A = len(g.widths)
            got = srv.results[sid]
            res["alone_equal_stream"] = sid
            res["alone_equal"] = len(got) == len(ks) and all(
                r == b"".join(want[i * A:(i + 1) * A]) for i, (_, _, r) in enumerate(got))
        srv.close()
        torch.cuda.synchronize()
        out[name] = res
        log(f"serving {name}: {res}")
    return out


def heuristic_leg(cases):
    """Sec. IV-E's validation of the trial (4 rows) against the brute-force
    choice, on the GPU: per record whether the trial's choice equals the
    brute-force one, the split of the disagreements (I chosen where P was
    smaller, P chosen where I was smaller), the bytes the trial leaves, and
    the throughput of both."""
    import torch

    from paper_2209_08196_amd import jiffy
    out = {}
    for name, host, precs in cases:
        dev = [torch.from_numpy(p.view(_STORE[p.dtype.itemsize])).cuda() for p in host]
        T, H, W = host[0].shape
        lay = jiffy.make_layout(H, W, [p.dtype.itemsize for p in host], precs)
        buf = torch.empty(jiffy.encode_bound(lay, T), dtype=torch.uint8, device="cuda")
        res = {}
        for mode, key in ((jiffy.MODE_AUTO, "trial"), (jiffy.MODE_BRUTE, "brute")):
            jiffy.encode(dev, precs, mode=mode, out=buf)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                s, m = jiffy.encode(dev, precs, mode=mode, out=buf)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            res[key] = (s.numel(), m.copy(), dt)
        mt, mb = res["trial"][1][1:], res["brute"][1][1:]  # scan 0 is an I-scan either way
        n = mt.size
        out[name] = {
            "records_compared": int(n), "agreement": round(float((mt == mb).mean()), 4),
            "suboptimal_i": round(float(((mt == 0) & (mb == 1)).mean()), 4),
            "suboptimal_p": round(float(((mt == 1) & (mb == 0)).mean()), 4),
            "p_fraction_brute": round(float(mb.mean()), 4),
            "trial_bytes_over_brute": round(res["trial"][0] / res["brute"][0] - 1.0, 5),
            "encode_points_per_s_trial": round(T * H * W * len(host) / res["trial"][2], 1),
            "encode_points_per_s_brute": round(T * H * W * len(host) / res["brute"][2], 1)}
        log(f"heuristic {name}: {out[name]}")
        del dev, buf
        torch.cuda.empty_cache()
    return out


def quant_leg(x_host, precisions=(1, 2, 4, 8, 16, 32, 64)):
    """Sec. IV-G / Fig. 4 on the GPU: the dual-return stream's range scans
    (mm) at precisions P = 1 .. 64 mm: bits per sample and per in-range
    sample, the largest reconstruction error (at most floor(P/2)), and
    encode/decode throughput."""
    import torch

    from paper_2209_08196_amd import jiffy
    x = torch.from_numpy(x_host.view(np.int32)).cuda()
    T, H, W = x_host.shape
    nz = x != 0
    n_nz = int(nz.sum())
    lay = jiffy.make_layout(H, W, [4], [1])
    buf = torch.empty(jiffy.encode_bound(lay, T), dtype=torch.uint8, device="cuda")
    dec = torch.empty_like(x)
    out = {"workload": f"dual-return-128x2048 range u32 (mm), {T} scans of {H}x{W}", "points": T * H * W,
           "in_range_fraction": round(n_nz / (T * H * W), 4), "sweep": []}
    prev = None
    for P in precisions:
        lay = jiffy.make_layout(H, W, [4], [P])
        enc = jiffy.Encoder([x], [P], out=buf)
        dcd = jiffy.Decoder(lay, T, [dec])
        s, _ = enc()
        dcd(s)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            s, _ = enc()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            dcd(s)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        err = int((dec.to(torch.int64) - x.to(torch.int64)).abs()[nz].max())  # ranges < 2^31: int32 storage
        bnz = 8.0 * s.numel() / n_nz
        row = {"P_mm": P, "bits_per_sample": round(8.0 * s.numel() / (T * H * W), 4),
               "bits_per_in_range_sample": round(bnz, 4),
               "bits_saved_vs_previous": round(prev - bnz, 4) if prev is not None else None,
               "max_abs_error_mm": err, "error_bound_mm": P // 2,
               "encode_points_per_s": round(T * H * W * reps / (t1 - t0), 1),
               "decode_points_per_s": round(T * H * W * reps / (t2 - t1), 1)}
        prev = bnz
        out["sweep"].append(row)
        log(f"quant P={P}: {row}")
    del x, buf, dec
    torch.cuda.empty_cache()
    return out


def _records(s):
    """(modes, record lengths, mask-frame lengths) of a stream with a length table."""
    A, = struct.unpack_from("<H", s, 6)
    T, = struct.unpack_from("<I", s, 16)
    p = 20 + 8 * A
    lens = np.array(struct.unpack_from(f"<{T * A}I", s, p), np.int64)
    p += 4 * T * A
    offs = p + np.concatenate([[0], np.cumsum(lens)[:-1]])
    b = np.frombuffer(s, np.uint8)
    modes = b[offs + 4].astype(np.int64)
    mlen = (b[offs + 8].astype(np.int64) | (b[offs + 9].astype(np.int64) << 8) | (b[offs + 10].astype(np.int64) << 16)
            | (b[offs + 11].astype(np.int64) << 24))
    return modes.reshape(T, A), lens.reshape(T, A), mlen.reshape(T, A)


def ablation_leg(cases):
    """Sec. IV-H / Table IV on the GPU: compression ratio (sample bytes over
    record bytes) of PFOR alone, Delta -> PFOR, Delta -> ZigZag -> PFOR (every
    pixel coded, no mask; jiffy_ablate), Mask -> Delta -> ZigZag -> PFOR (the
    I-only stream) and the codec (automatic I/P), per attribute and over all;
    and the mask frames of the codec's stream against the run-length mask
    codec on the same masks (the I-mask or the XOR mask, as each record
    chose)."""
    import torch

    from paper_2209_08196_amd import jiffy
    out = {}
    for name, host, precs, attr_names in cases:
        dev = [torch.from_numpy(p.view(_STORE[p.dtype.itemsize])).cuda() for p in host]
        T, H, W = host[0].shape
        raw = np.array([p.nbytes for p in host], np.float64)
        jiffy.ablate(dev, precs)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sz = jiffy.ablate(dev, precs).astype(np.int64)  # [T, A, 5]
        dt = time.perf_counter() - t0
        lay = jiffy.make_layout(H, W, [p.dtype.itemsize for p in host], precs)
        buf = torch.empty(jiffy.encode_bound(lay, T), dtype=torch.uint8, device="cuda")
        rec = {}
        for mode, key in ((jiffy.MODE_I_ONLY, "i_only"), (jiffy.MODE_AUTO, "jiffy")):
            s, _ = jiffy.encode(dev, precs, mode=mode, out=buf)
            rec[key] = _records(s.cpu().numpy().tobytes())
        levels = {"pfor": sz[:, :, 0].sum(0), "delta_pfor": sz[:, :, 1].sum(0),
                  "delta_zigzag_pfor": sz[:, :, 2].sum(0), "mask_delta_zigzag_pfor": rec["i_only"][1].sum(0),
                  "jiffy": rec["jiffy"][1].sum(0)}
        modes, _, mlen = rec["jiffy"]
        zstd_mask = ((mlen + 3) & ~3).sum(0)
        rl_mask = np.where(modes == 1, sz[:, :, 4], sz[:, :, 3]).sum(0)
        i_zstd = ((rec["i_only"][2] + 3) & ~3).sum(0)
        row = {"points": T * H * W * len(host), "scans": T, "shape": [H, W], "attributes": attr_names,
               "ablate_points_per_s": round(T * H * W * len(host) / dt, 1),
               "ratio_total": {k: round(float(raw.sum() / v.sum()), 3) for k, v in levels.items()},
               "ratio_per_attribute": {k: [round(float(r / b), 3) for r, b in zip(raw, v)] for k, v in levels.items()},
               "mask_bytes_codec_frame": int(zstd_mask.sum()), "mask_bytes_run_length": int(rl_mask.sum()),
               "mask_bytes_i_frame": int(i_zstd.sum()), "mask_bytes_i_run_length": int(sz[:, :, 3].sum()),
               "mask_run_length_over_frame": round(float(rl_mask.sum() / zstd_mask.sum()), 4),
               "p_records": int(modes.sum())}
        out[name] = row
        log(f"ablation {name}: {row}")
        del dev, buf
        torch.cuda.empty_cache()
    return out


def standardize_leg(clouds, H, W, reps=5):
    """Sec. III-A on the GPU: Cartesian clouds (float32 xyz plus three
    attributes per point) of the dual-return stream's range scans binned into
    range and attribute images, all scans in one call; throughput, the
    kernels' times (HIP events) and their algorithmic bytes (12 bytes of
    coordinates and the attributes per point read, the images and one 8-byte
    key per cell written and read back), and a comparison of sampled scans
    with the oracle."""
    import torch

    import oracle.standardize as ost
    from paper_2209_08196_amd import jiffy, synth
    S = len(clouds)
    n = max(len(x) for x, _ in clouds)
    xyz = np.full((S, n, 3), np.nan, np.float32)
    A = len(clouds[0][1])
    attrs = [np.zeros((S, n), clouds[0][1][a].dtype) for a in range(A)]
    for i, (x, at) in enumerate(clouds):
        xyz[i, :len(x)] = x
        for a in range(A):
            attrs[a][i, :len(x)] = at[a]
    e_lo, e_hi = synth.FOV_ELEV_RAD
    dx = torch.from_numpy(xyz).cuda()
    da = [torch.from_numpy(a.view(_STORE[a.dtype.itemsize])).cuda() for a in attrs]
    rng = torch.empty((S, H, W), dtype=torch.int32, device="cuda")
    outs = [torch.empty((S, H, W), dtype=d.dtype, device="cuda") for d in da]
    jiffy.standardize(dx, H, W, e_lo, e_hi, 0.001, 4, da, outs=(rng, outs))
    torch.cuda.synchronize()
    jiffy.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        jiffy.standardize(dx, H, W, e_lo, e_hi, 0.001, 4, da, outs=(rng, outs))
    dt = (time.perf_counter() - t0) / reps
    prof = jiffy.profile_read()
    jiffy.profile_enable(False)
    ab = sum(a.dtype.itemsize for a in attrs)
    cells = S * H * W
    alg = {"k_std_points": S * n * 12 + cells * 8, "k_std_gather": S * n * ab + cells * (8 + 4 + ab),
           "k_std_clear": cells * 8}
    kern = {k: round(v[0] / v[1], 4) for k, v in prof.items() if k in alg}
    got = rng.cpu().numpy().view(np.uint32)
    got_a = [o.cpu().numpy().view({1: np.uint8, 2: np.uint16, 4: np.uint32}[a.dtype.itemsize])
             for o, a in zip(outs, attrs)]
    checked, same = [0, S // 2, S - 1], True
    for s in checked:
        w, wa = ost.standardize(xyz[s], H, W, e_lo, e_hi, 0.001, 4, [a[s] for a in attrs])
        same &= bool(np.array_equal(got[s], w)) and all(np.array_equal(g[s], x) for g, x in zip(got_a, wa))
    out = {"workload": f"dual-return-128x2048 Cartesian clouds: {S} scans of up to {n} points (float32 xyz, "
                       f"{A} attributes), binned to {H}x{W}", "points": S * n, "ms_per_call": round(1e3 * dt, 3),
           "points_per_s": round(S * n / dt, 1), "kernels_ms": kern,
           "kernel_alg_gbps": {k: round(alg[k] / (kern[k] * 1e-3) / 1e9, 1) for k in kern},
           "oracle_scans_checked": checked, "identical": same}
    log(f"standardize: {out}")
    del dx, da, rng, outs
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# the oracle on the host (test infrastructure, timed as the CPU baseline)
# ---------------------------------------------------------------------------
def cpu_leg(host_period, ctx, n_single, n_all):
    """The oracle on whole 200-scan streams of the headline workload: one
    stream on one thread, then one stream per thread on all host cores.
    Their streams are compared byte for byte with the timed GPU encoder's."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    T, precs = ctx["T"], ctx["precs"]
    reps = T // SCENE_PERIOD

    def one(s):
        planes = [np.ascontiguousarray(np.tile(p, (reps, 1, 1))) for p in host_period[s]]
        t0 = time.perf_counter()
        ref, modes = oracle.encode(planes, precs)
        t1 = time.perf_counter()
        oracle.decode(ref)
        t2 = time.perf_counter()
        same = ref == ctx["streams"][s] and bool(np.array_equal(modes, ctx["modes"][s]))
        return t1 - t0, t2 - t1, same, sum(p.size for p in planes)

    log(f"cpu: oracle on {n_single} stream(s), one thread")
    t0 = time.perf_counter()
    single = [one(s) for s in range(n_single)]
    w1 = time.perf_counter() - t0
    pts1 = sum(r[3] for r in single)
    threads = min(n_all, pool_size())
    log(f"cpu: oracle on {n_all} streams, {threads} threads")
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:  # the oracle releases the GIL inside its C calls
        multi = list(ex.map(one, range(n_all)))
    wn = time.perf_counter() - t0
    ptsn = sum(r[3] for r in multi)
    identical = all(r[2] for r in single + multi)
    return {
        "value": round(ptsn / wn, 1), "unit": "points/s", "cores": threads, "kind": "oracle",
        "sample": f"{n_all} whole streams of the headline workload ({T} scans of 128x4096 each), encode + decode, "
                  f"one stream per thread on {threads} threads; {wn:.1f} s wall",
        "single_thread": {"value": round(pts1 / w1, 1), "cores": 1,
                          "sample": f"{n_single} whole stream(s), encode + decode, {w1:.1f} s",
                          "encode_s": round(sum(r[0] for r in single), 2),
                          "decode_s": round(sum(r[1] for r in single), 2)},
        "host_cpu": _cpu_model(), "host_cores": os.cpu_count(),
        "byte_identical_streams": n_all if identical else [i for i, r in enumerate(multi) if not r[2]],
    }, identical


# ---------------------------------------------------------------------------
# counter runs (rocprofv3) and their summary
# ---------------------------------------------------------------------------
def copy_run(nbytes):
    """A plain device copy of known size, three times: what FETCH_SIZE and
    WRITE_SIZE read for it calibrates those counters."""
    import torch
    torch.cuda.set_device(0)
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}), flush=True)


_DEC_TILE_NAMES = {"4": "k_dec_tiles_w32", "2": "k_dec_tiles_w16", "1": "k_dec_tiles_w8"}


def _kernel_key(full):
    """A profiler's kernel name as the library's timing hooks name it (the
    decoder tile kernel by sample width, other templates without arguments)."""
    name = full.split("(")[0].split("::")[-1]
    if "<" in name:
        base, args = name.split("<", 1)
        if base == "k_dec_tiles":
            return _DEC_TILE_NAMES.get(args.rstrip(">").split(",")[-1].strip(), base)
        name = base
    return name


def profile_summary(title, stats_csv, workload=None, sq_dirs=()):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run: per kernel
    its calls, mean duration and share of GPU time; with the workload's
    calibrated HBM counters (profiles/traffic.json, same kernel source) its
    bytes read and written per launch; with SQ counter folders the per-wave
    instruction mix, the share of wave time spent waiting and the VALU and
    LDS activity."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    traffic = {}
    if workload and os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("source_sha") == source_sha():
            traffic = tr.get("workloads", {}).get(workload, {}).get("kernels", {})
    out = [f"# {title}", "", "| kernel | calls | average us | % of GPU time | HBM read MB | HBM write MB |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        key = _kernel_key(r["Name"])
        t = traffic.get(key, {})
        name = r["Name"].split("(")[0]
        if len(name) > 60:
            name = name[:57] + "..."
        rd = f"{t['fetch_bytes'] / 1e6:.1f}" if t else ""
        wr = f"{t['write_bytes'] / 1e6:.1f}" if t else ""
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} | "
                   f"{rd} | {wr} |")
    if sq_dirs:
        c = {}
        for d in sq_dirs:
            import glob
            for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
                for row in csv.DictReader(open(f)):
                    k = _kernel_key(row["Kernel_Name"])
                    if not k.startswith("k_"):
                        continue
                    c.setdefault(k, {}).setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
        out += ["", "SQ counters per launch (means over dispatches; wave-level counts per wave):", "",
                "| kernel | waves | VALU instr/wave | LDS instr/wave | SALU instr/wave | VMEM rd/wr per wave | "
                "wave time waiting | LDS bank-conflict cycles / LDS active cycles |", "|---|---:|---:|---:|---:|---:|---:|---:|"]

        def m(k, n):
            v = c[k].get(n)
            return sum(v) / len(v) if v else float("nan")
        for k in sorted(c, key=lambda k: -m(k, "SQ_BUSY_CYCLES") if "SQ_BUSY_CYCLES" in c[k] else 0):
            w = m(k, "SQ_WAVES")
            out.append(f"| `{k}` | {w:.0f} | {m(k, 'SQ_INSTS_VALU') / w:.0f} | {m(k, 'SQ_INSTS_LDS') / w:.0f} | "
                       f"{m(k, 'SQ_INSTS_SALU') / w:.0f} | {m(k, 'SQ_INSTS_VMEM_RD') / w:.1f} / "
                       f"{m(k, 'SQ_INSTS_VMEM_WR') / w:.1f} | {m(k, 'SQ_WAIT_ANY') / m(k, 'SQ_WAVE_CYCLES'):.0%} | "
                       f"{m(k, 'SQ_LDS_BANK_CONFLICT') / max(m(k, 'SQ_ACTIVE_INST_LDS'), 1):.2f} |")
    print("\n".join(out))


def _counter_means(folder, counter):
    """Mean per dispatch of one counter, per kernel name, from a rocprofv3
    --pmc csv folder (values summed over the dispatch's rows), over the
    kernel's dispatches of its largest grid: the launch shape of the timed
    step (a leg's smaller launches, such as one scan per launch, are left
    out)."""
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter csv under {folder}")
    per, grid = {}, {}
    for row in csv.DictReader(open(files[0])):
        if row["Counter_Name"] != counter:
            continue
        name = _kernel_key(row["Kernel_Name"])
        key = (name, row["Dispatch_Id"])
        per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
        grid[key] = int(row["Grid_Size"])
    top = {}
    for (name, d), g in grid.items():
        top[name] = max(top.get(name, 0), g)
    out = {}
    for (name, d), v in per.items():
        if grid[(name, d)] != top[name]:
            continue
        t = out.setdefault(name, [0.0, 0])
        t[0] += v
        t[1] += 1
    return {k: v[0] / v[1] for k, v in out.items()}


def summarize_traffic(workload, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes):
    """HBM bytes per launch of every kernel of one workload: FETCH_SIZE and
    WRITE_SIZE (KiB) scaled by what they read for a copy of copy_bytes."""
    if not copy_bytes:
        raise SystemExit("--traffic needs --copy-bytes (the calibration copy's size)")
    f = _counter_means(fetch_dir, "FETCH_SIZE")
    w = _counter_means(write_dir, "WRITE_SIZE")
    cf = max(_counter_means(copy_fetch_dir, "FETCH_SIZE").values())
    cw = max(_counter_means(copy_write_dir, "WRITE_SIZE").values())
    kf, kw = copy_bytes / cf, copy_bytes / cw  # bytes per counter unit
    res = json.load(open(TRAFFIC_FILE)) if os.path.exists(TRAFFIC_FILE) else {}
    if res.get("source_sha") != source_sha():
        res = {"source_sha": source_sha(), "workloads": {}}
    res["workloads"][workload] = {
        "calibration": {"copy_bytes": copy_bytes, "fetch_bytes_per_unit": kf, "write_bytes_per_unit": kw},
        "kernels": {k: {"fetch_bytes": round(f[k] * kf), "write_bytes": round(w.get(k, 0.0) * kw)}
                    for k in sorted(f) if k.startswith("k_")}}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res["workloads"][workload]))


def trace_overlap(path):
    """From a rocprofv3 --kernel-trace csv: per HIP stream (queue) the
    library's kernels' busy time, and the time during which kernels of two
    or more streams ran at once."""
    import csv
    rows = list(csv.DictReader(open(path)))
    key = "Stream_Id" if rows and "Stream_Id" in rows[0] else "Queue_Id"
    iv = {}
    for r in rows:
        name = r["Kernel_Name"]
        if "jiffy" not in name:
            continue
        iv.setdefault(r[key], []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    events = []
    for q, lst in iv.items():
        for a, b in lst:
            events.append((a, 1, q))
            events.append((b, -1, q))
    events.sort()
    active = {}
    both = 0
    last = None
    busy = {q: 0 for q in iv}
    for t, d, q in events:
        if last is not None:
            live = [x for x, c in active.items() if c > 0]
            for x in live:
                busy[x] += t - last
            if len(live) >= 2:
                both += t - last
        active[q] = active.get(q, 0) + d
        last = t
    res = {"streams": {str(q): {"kernels": len(iv[q]), "busy_ms": round(busy[q] / 1e6, 3)} for q in iv},
           "overlap_ms": round(both / 1e6, 3), "key": key}
    print(json.dumps(res))
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--streams", type=int, default=None, help="headline streams (default: all 32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-stream batched leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the 256-stream serving leg")
    ap.add_argument("--only", choices=["headline", "batched", "serving", "heuristic", "quant", "ablation",
                                       "standardize"],
                    help="run one leg only")
    ap.add_argument("--no-heuristic", action="store_true", help="skip the trial-versus-brute-force leg")
    ap.add_argument("--no-ablation", action="store_true", help="skip the ablation leg")
    ap.add_argument("--no-standardize", action="store_true", help="skip the input standardization leg")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--serving-seconds", type=float, default=10.0)
    ap.add_argument("--profile-steps", type=int, default=1, help="steps timed per kernel with HIP events")
    ap.add_argument("--per-stream-steps", type=int, default=3,
                    help="headline steps also timed as one encode and one decode call per stream (0: skip)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes (counter calibration)")
    ap.add_argument("--traffic", nargs=5, metavar=("WORKLOAD", "FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="summarize four rocprofv3 --pmc output folders (FETCH_SIZE and WRITE_SIZE of a bench "
                         "run and of a --copy-bytes run) into " + os.path.relpath(TRAFFIC_FILE, ROOT))
    ap.add_argument("--profile-summary", nargs=2, metavar=("TITLE", "KERNEL_STATS_CSV"),
                    help="print a markdown summary of a rocprofv3 --stats run (with --traffic-workload and --sq)")
    ap.add_argument("--traffic-workload", help="workload key of the HBM counters in " + os.path.relpath(TRAFFIC_FILE, ROOT))
    ap.add_argument("--sq", nargs="*", default=(), help="rocprofv3 --pmc folders of SQ counters")
    ap.add_argument("--trace-overlap", metavar="KERNEL_TRACE_CSV",
                    help="summarize per-stream kernel time and cross-stream overlap of a rocprofv3 kernel trace")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(*args.profile_summary, workload=args.traffic_workload, sq_dirs=args.sq)
        return
    if args.trace_overlap:
        trace_overlap(args.trace_overlap)
        return
    if args.traffic:
        summarize_traffic(*args.traffic, copy_bytes=args.copy_bytes)
        return
    if args.copy_bytes:
        copy_run(args.copy_bytes)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (streams shard across GPUs "
              "without exchange, so the one-GPU figure is the per-GPU throughput).", file=sys.stderr)
        sys.exit(2)
    from paper_2209_08196_amd import synth

    legs = {args.only} if args.only else {"headline", "batched", "serving", "heuristic", "quant", "ablation",
                                          "standardize"}
    if args.no_heuristic:
        legs.discard("heuristic")
    if args.no_ablation:
        legs.discard("ablation")
    if args.no_standardize:
        legs.discard("standardize")
    if args.no_batched:
        legs.discard("batched")
    if args.no_serving:
        legs.discard("serving")
    # synthetic inputs first, in worker processes (the GPU is not touched yet)
    t0 = time.perf_counter()
    jobs = []
    n_head = synth.CONFIGS[HEAD_CID].streams if args.streams is None else args.streams
    if "headline" in legs:
        jobs += [(HEAD_CID, s, 0, SCENE_PERIOD) for s in range(n_head)]
    nb = args.warmup + args.batched_steps
    if "batched" in legs:
        jobs += [(3, s, 0, nb) for s in range(synth.CONFIGS[3].streams)]
    if "serving" in legs:
        jobs += [(4, s, 0, SERVING_CYCLE) for s in range(synth.CONFIGS[4].streams)]
    n_before_h = len(jobs)
    if "heuristic" in legs:  # the plain stream, the dual-return stream, two whole stress streams
        jobs += [(1, 0, 0, 10), (2, 0, 0, 100), (5, 0, 0, 200), (5, 1, 0, 200)]
    elif "quant" in legs or "ablation" in legs or "standardize" in legs:
        jobs += [(2, 0, 0, 100)]
    n_before_a = len(jobs)
    if "ablation" in legs:  # the dual-return stream seen by a sensor that never moves
        jobs += [(2, 0, 0, 100, True)]
    data = generate(jobs)
    abl_static = data[n_before_a] if "ablation" in legs else None
    data = data[:n_before_a]
    extra = data[n_before_h:]
    heur_host = extra if "heuristic" in legs else None
    dual_host = (extra[1] if "heuristic" in legs else extra[0]) \
        if ("quant" in legs or "ablation" in legs or "standardize" in legs) else None
    clouds = generate_clouds(dual_host) if "standardize" in legs else None
    quant_host = dual_host[0] if "quant" in legs else None
    data = data[:n_before_h]
    head_host = data[:n_head] if "headline" in legs else None
    o = n_head if "headline" in legs else 0
    batched_host = data[o:o + synth.CONFIGS[3].streams] if "batched" in legs else None
    o += synth.CONFIGS[3].streams if "batched" in legs else 0
    serving_host = data[o:] if "serving" in legs else None
    log(f"generated {len(jobs)} stream segments in {time.perf_counter() - t0:.1f}s on {gen_procs()} processes")

    import torch
    torch.cuda.set_device(0)
    result = {}
    if "headline" in legs:
        result, ctx = headline(args, head_host)
    if "batched" in legs:
        result["batched"] = batched_leg(batched_host, args.batched_steps, args.warmup)
        log(f"batched: {json.dumps(result['batched'])}")
    if "serving" in legs:
        result["serving"] = serving_leg(serving_host, args.serving_seconds)
    if "heuristic" in legs:
        g1, g2 = synth.stream(1, 0), synth.stream(2, 0)
        result["heuristic"] = heuristic_leg([
            ("plain-64x1024-range-1cm x10", heur_host[0], list(g1.precisions)),
            ("dual-return-128x2048-5attr-1mm x100", heur_host[1], list(g2.precisions)),
            ("stress-128x4096 stream 0 x200", heur_host[2], [1]),
            ("stress-128x4096 stream 1 x200", heur_host[3], [1])])
    if "quant" in legs:
        result["quant"] = quant_leg(quant_host)
    if "standardize" in legs:
        result["standardize"] = standardize_leg(clouds, *dual_host[0].shape[1:])
    if "ablation" in legs:
        g2 = synth.stream(2, 0)
        an = [a.name for a in g2.cfg.attrs]
        result["ablation"] = ablation_leg([
            ("dual-return-128x2048-5attr-1mm x100", dual_host, list(g2.precisions), an),
            ("dual-return-128x2048-5attr-1mm standing sensor x100", abl_static, list(g2.precisions), an)])
    if "headline" in legs and not args.no_cpu_baseline:
        cb, identical = cpu_leg(head_host, ctx, n_single=1, n_all=min(n_head, pool_size()))
        result["cpu_baseline"] = cb
        result["byte_identical"] = identical
        if not identical:
            log("GPU stream differs from the oracle")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
