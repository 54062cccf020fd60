#!/usr/bin/env python3
"""Encode+decode throughput of the Jiffy codec on one MI355X.

Workload: one sensor stream of 100 scans of 128x2048 with five attributes
(dual-return range u32, second-return range u32, signal u16, reflectivity u8,
near-IR u16), precision 1 mm, about 20% zero samples, seeded synthetic data
standing in for the paper's Ouster driving recordings (the sensor drives,
stops for 30 scans, drives again).  One step encodes all 100 scans
(jiffy_encode) and decodes the stream back (jiffy_decode); inputs and
outputs stay in device memory.  A point is one pixel of one attribute, as in
the paper's points/s (Sec. IV-F).

Prints one JSON line.  Besides the throughput it carries:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                mean launch time (HIP events on the launch stream) against
                the 8 TB/s HBM peak; `traffic` is the HBM bytes measured with
                rocprofv3 counters for the same kernel source (or null).
  cpu_baseline  the CPU oracle (single thread) on the same workload, and
                whether its stream is byte-identical to the GPU's.
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
CID = 2  # the dual-return 128x2048 five-attribute stream
N_SCANS = 100
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2209_08196_amd", "csrc", f)
                  for f in ("jiffy_encode.hip", "jiffy_decode.hip", "jiffy_device.h", "jiffy_internal.h")]


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def stream_stats(s: bytes, widths, npx):
    """Sizes of the stream's parts, read from its header and record headers."""
    A, = struct.unpack_from("<H", s, 6)
    T, = struct.unpack_from("<I", s, 16)
    p = 20 + 8 * A
    lens = struct.unpack_from(f"<{T * A}I", s, p)
    p += 4 * T * A
    st = dict(mask_bytes=0, frame_bytes=0, n_values=0, p_items=0, p_bytes=0, i_items=0,
              frame_bytes_w32=0, items_w32=0, x_bytes_w32=0, p_bytes_w32=0)
    for r, L in enumerate(lens):
        a = r % A
        mode = s[p + 4]
        flen, = struct.unpack_from("<I", s, p + 8)
        sec = (12 + flen + 3) & ~3
        N, = struct.unpack_from("<I", s, p + sec)
        nb = (N + 127) // 128
        hdr4 = (4 + 3 * nb + 3) & ~3
        b = np.frombuffer(s, np.uint8, nb, p + sec + 4).astype(np.int64)
        n = np.frombuffer(s, np.uint8, nb, p + sec + 4 + nb).astype(np.int64)
        B = np.frombuffer(s, np.uint8, nb, p + sec + 4 + 2 * nb).astype(np.int64)
        fb = int((16 * b + n + (n * (B - b) + 7) // 8).sum())
        st["frame_bytes"] += fb
        if widths[a] == 4:
            st["frame_bytes_w32"] += fb
            st["items_w32"] += 1
            st["x_bytes_w32"] += 4 * npx
        st["mask_bytes"] += flen
        st["n_values"] += N
        if mode == 1:
            st["p_items"] += 1
            st["p_bytes"] += widths[a] * npx
            if widths[a] == 4:
                st["p_bytes_w32"] += 4 * npx
        else:
            st["i_items"] += 1
        p += L
    st["stream_bytes"] = len(s)
    return st


def kernel_alg_bytes(name, st, x_bytes, n_items, nwords):
    """Bytes each kernel must move for the whole workload (one launch): its
    inputs read once and its outputs written once, intermediates it cannot
    avoid included (the valid-sample words, the packed frames)."""
    vb = 8 * nwords * n_items          # valid-sample words of every record
    vbp = 8 * nwords * st["p_items"]   # the previous scan's, for P-records
    F, M, S = st["frame_bytes"], st["mask_bytes"], st["stream_bytes"]
    Xp = st["p_bytes"]                 # samples of the P-records
    table = {
        "k_enc_tiles": x_bytes + Xp + vb + F,  # samples (+ previous scan) in, valid words and packed frames out
        "k_enc_mframe": vb + vbp + M,          # valid words in, mask frames out
        "k_enc_assemble": F + M + S,           # frames and masks in, stream out
        "k_dec_parse": M + vb,                 # mask frames in, valid words out
        "k_dec_mask": 2 * vb + vbp,            # mask chain over time
        "k_dec_tiles_w32": st["frame_bytes_w32"] + 8 * nwords * st["items_w32"] + st["x_bytes_w32"],
        "k_dec_tiles_w16": (F - st["frame_bytes_w32"]) + 8 * nwords * (n_items - st["items_w32"])
                           + (x_bytes - st["x_bytes_w32"]),
        "k_dec_temporal": 3 * Xp,              # P-scans: read both scans, write one
    }
    return table.get(name)


def batched_leg(steps, warmup):
    """64 sensor streams of four sizes (16x1024, 32x2048, 64x1024, 128x2048;
    range u32 at 1 cm and signal u16), one scan of every stream per step:
    the graph-replayed batch (jiffy_batch_run) against the plain batched
    call (jiffy_batch_encode_step) on twin streams, with byte-identical
    records required."""
    import torch

    from paper_2209_08196_amd import jiffy, synth
    cfg = synth.CONFIGS[3]
    T = warmup + steps
    gens = [synth.stream(3, s) for s in range(cfg.streams)]
    store = {1: np.uint8, 2: np.int16, 4: np.int32}
    scans = [[torch.from_numpy(p.view(store[p.dtype.itemsize])).cuda() for p in g.scans(0, T)] for g in gens]
    points = sum(g.H * g.W * len(g.widths) for g in gens)
    mk = lambda: [jiffy.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]  # noqa: E731
    sg, sp = mk(), mk()
    inputs = [[p[0] for p in sc] for sc in scans]
    outs_g = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sg]
    outs_p = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sp]
    batch = jiffy.Batch(sg, inputs, outs_g)
    identical = True
    tg = tp = 0.0
    for t in range(T):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lg, _ = batch.run([[p[t] for p in sc] for sc in scans])
        t1 = time.perf_counter()
        lp, _ = jiffy.batch_encode_step(sp, [[p[t] for p in sc] for sc in scans], outs_p)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if t >= warmup:
            tg += t1 - t0
            tp += t2 - t1
        if lg != lp or any(not torch.equal(outs_g[i][: lg[i]], outs_p[i][: lp[i]]) for i in range(len(gens))):
            identical = False
    batch.close()
    for s in sg + sp:
        s.close()
    return {"workload": f"{cfg.name}, {steps} steps", "streams": cfg.streams, "points_per_step": points,
            "graph_points_per_s": round(points * steps / tg, 1), "graph_ms_per_step": round(1e3 * tg / steps, 3),
            "plain_points_per_s": round(points * steps / tp, 1), "plain_ms_per_step": round(1e3 * tp / steps, 3),
            "byte_identical": identical}


def serving_leg(duration_s, budgets, scans_per_stream=2):
    """256 sensor streams (32x1024 .. 128x2048, range u32 and three u16
    attributes at 1 mm; 10 or 20 Hz each with random phase and jitter)
    served by continuous batching under device-memory budgets.  Each stream
    cycles through its first `scans_per_stream` synthetic scans.  Latency =
    records on the host minus arrival, in virtual time (each step advances
    the clock by its measured duration).  One served stream's records are
    compared with encoding its whole sequence alone (jiffy_encode)."""
    import torch

    from paper_2209_08196_amd import jiffy, serve, synth
    cfg = synth.CONFIGS[4]
    gens = [synth.stream(4, s) for s in range(cfg.streams)]
    store = {1: np.uint8, 2: np.int16, 4: np.int32}
    host = [g.scans(0, scans_per_stream) for g in gens]
    dev = [[torch.from_numpy(p.view(store[p.dtype.itemsize])).cuda() for p in h] for h in host]
    specs = {s: serve.StreamSpec(g.H, g.W, tuple(g.widths), tuple(g.precisions)) for s, g in enumerate(gens)}
    arrivals = synth.serving_arrivals(cfg.streams, duration_s)
    check = arrivals[0][1]  # the first stream to arrive is admitted under any budget that admits one
    ks = [k for _, s, k in arrivals if s == check]
    g = gens[check]
    # its alone-encoding: the whole sequence in one jiffy_encode call
    seq = [torch.stack([dev[check][a][k % scans_per_stream] for k in ks]).contiguous() for a in range(len(g.widths))]
    alone, _ = jiffy.encode(seq, g.precisions)
    want = split_records(alone.cpu().numpy().tobytes())
    A = len(g.widths)
    out = {"workload": f"{cfg.name}, {duration_s} s of arrivals", "streams": cfg.streams,
           "scans_offered": len(arrivals)}
    for budget in budgets:
        srv = serve.Server.gpu(specs, budget)
        st = srv.run(arrivals, lambda sid, k: [p[k % scans_per_stream] for p in dev[sid]], keep_results={check})
        res = st.summary()
        got = srv.results[check]
        res["alone_equal"] = len(got) == len(ks) and all(
            r == b"".join(want[k * A:(k + 1) * A]) for k, r in enumerate(got))
        srv.close()
        out[f"budget_{budget >> 20}MiB"] = res
        print(f"[bench] serving budget {budget >> 20} MiB: {res}", file=sys.stderr, flush=True)
    return out


def split_records(s: bytes):
    """The records of a stream with a record-length table (its header)."""
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


def _counter_means(folder, counter):
    """Mean per dispatch of one counter, per kernel name, from a rocprofv3
    --pmc csv folder (values summed over the dispatch's rows)."""
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter csv under {folder}")
    per = {}
    for row in csv.DictReader(open(files[0])):
        if row["Counter_Name"] != counter:
            continue
        name = row["Kernel_Name"].split("(")[0].split("::")[-1]
        key = (name, row["Dispatch_Id"])
        per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (name, _), v in per.items():
        t = out.setdefault(name, [0.0, 0])
        t[0] += v
        t[1] += 1
    return {k: v[0] / v[1] for k, v in out.items()}


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes):
    """HBM bytes per launch of every kernel: FETCH_SIZE and WRITE_SIZE (KiB)
    scaled by what they read for a copy of copy_bytes."""
    if not copy_bytes:
        raise SystemExit("--traffic needs --copy-bytes (the calibration copy's size)")
    f = _counter_means(fetch_dir, "FETCH_SIZE")
    w = _counter_means(write_dir, "WRITE_SIZE")
    cf = max(_counter_means(copy_fetch_dir, "FETCH_SIZE").values())
    cw = max(_counter_means(copy_write_dir, "WRITE_SIZE").values())
    kf, kw = copy_bytes / cf, copy_bytes / cw  # bytes per counter unit
    from paper_2209_08196_amd import synth
    res = {"source_sha": source_sha(), "workload": synth.CONFIGS[CID].name,
           "calibration": {"copy_bytes": copy_bytes, "fetch_bytes_per_unit": kf, "write_bytes_per_unit": kw},
           "kernels": {k: {"fetch_bytes": round(f[k] * kf), "write_bytes": round(w.get(k, 0.0) * kw)}
                       for k in sorted(f) if k.startswith("k_")}}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-stream batched leg")
    ap.add_argument("--only-batched", action="store_true", help="run only the 64-stream batched leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the 256-stream serving leg")
    ap.add_argument("--only-serving", action="store_true", help="run only the 256-stream serving leg")
    ap.add_argument("--profile-steps", type=int, default=3, help="steps timed per kernel with HIP events")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes (counter calibration)")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="summarize four rocprofv3 --pmc output folders (FETCH_SIZE and WRITE_SIZE of a bench "
                         "run and of a --copy-bytes run) into " + os.path.relpath(TRAFFIC_FILE, ROOT))
    args = ap.parse_args()
    if args.traffic:
        summarize_traffic(*args.traffic, copy_bytes=args.copy_bytes)
        return
    if args.copy_bytes:
        copy_run(args.copy_bytes)
        return
    if args.only_serving:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(serving_leg(1.0, [8 << 30, 64 << 20])), flush=True)
        return
    if args.only_batched:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(batched_leg(steps=args.steps, warmup=args.warmup)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (streams shard across GPUs "
              "without exchange, so the one-GPU figure is the per-GPU throughput).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2209_08196_amd import jiffy, synth

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    g = synth.stream(CID, 0)
    planes = g.scans(0, N_SCANS)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] generated {N_SCANS} scans of {g.H}x{g.W}, {len(planes)} attributes in {t_gen:.1f}s",
          file=sys.stderr, flush=True)
    store = {1: np.uint8, 2: np.int16, 4: np.int32}
    dev = [torch.from_numpy(p.view(store[p.dtype.itemsize])).cuda() for p in planes]
    precs = g.precisions
    widths = g.widths
    T, H, W = planes[0].shape
    npx = H * W
    A = len(planes)
    points = T * npx * A
    x_bytes = sum(p.nbytes for p in planes)
    lay = jiffy.make_layout(H, W, widths, precs)
    out = torch.empty(jiffy.encode_bound(lay, T), dtype=torch.uint8, device="cuda")
    dec = [torch.empty_like(d) for d in dev]
    stream = torch.cuda.current_stream()

    def step():
        s, modes = jiffy.encode(dev, precs, out=out)
        jiffy.decode(s, lay, T, outs=dec)
        return s, modes

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # correctness of this run: lossless round trip (P = 1 everywhere)
    s_dev, modes = step()
    for d, x in zip(dec, dev):
        if not torch.equal(d, x):
            raise SystemExit("decode(encode(x)) != x")
    s_gpu = s_dev.cpu().numpy().tobytes()
    st = stream_stats(s_gpu, widths, npx)
    print(f"[bench] stream {len(s_gpu)} bytes, ratio {x_bytes / len(s_gpu):.2f}, P-scans {st['p_items']}",
          file=sys.stderr, flush=True)

    # timed steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    enc = jiffy.Encoder(dev, precs, out=out, stream=stream)  # the same calls, arguments prepared once
    dcd = jiffy.Decoder(lay, T, dec, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ev_e0, ev_e1, ev_d1 in evs:
        ev_e0.record(stream)
        s, _ = enc()
        ev_e1.record(stream)
        dcd(s)
        ev_d1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in evs)
    dec_ms = sum(e1.elapsed_time(d1) for _, e1, d1 in evs)
    ms_per_step = 1e3 * wall / args.steps
    value = points / (wall / args.steps)
    print(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)

    if args.profile_steps <= 0:  # counter-collection runs: the kernels only
        print(json.dumps({"metric": METRIC, "ms_per_step": round(ms_per_step, 3)}), flush=True)
        return
    # per-kernel times with HIP events on the launch stream
    jiffy.profile_enable(True)
    for _ in range(args.profile_steps):
        step()
    torch.cuda.synchronize()
    prof = jiffy.profile_read()
    jiffy.profile_enable(False)
    n_items = T * A
    nwords = (npx + 63) // 64
    kernels = {k: dict(avg_ms=v[0] / v[1], launches=v[1]) for k, v in prof.items()}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    alg = kernel_alg_bytes(dom, st, x_bytes, n_items, nwords)
    avg_s = kernels[dom]["avg_ms"] / 1e3
    achieved = alg / avg_s / 1e9 if alg else None
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        ent = tr.get("kernels", {}).get(dom)
        if ent and tr.get("source_sha") == source_sha() and tr.get("workload") == g.cfg.name:
            traffic = ent["fetch_bytes"] + ent["write_bytes"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic, "kernel": dom, "alg_bytes_per_launch": alg,
                "avg_launch_ms": round(kernels[dom]["avg_ms"], 4)}
    path_alg = 2 * (x_bytes + st["p_bytes"]) + 2 * st["stream_bytes"]

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{g.cfg.name}, {T} scans, encode+decode", "scans": T, "height": H, "width": W,
                   "attributes": [a.name for a in g.cfg.attrs], "precision_mm": 1},
        "encode_points_per_s": round(points / (enc_ms / args.steps / 1e3), 1),
        "decode_points_per_s": round(points / (dec_ms / args.steps / 1e3), 1),
        "compression_ratio": round(x_bytes / st["stream_bytes"], 3),
        "p_scans": st["p_items"], "i_scans": st["i_items"],
        "path_alg_gbps": round(path_alg / (wall / args.steps) / 1e9, 1),
        "path_hbm_frac": round(path_alg / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["avg_ms"])},
    }

    if not args.no_batched:
        result["batched"] = batched_leg(steps=8, warmup=2)
        print(f"[bench] batched: {result['batched']}", file=sys.stderr, flush=True)
    if not args.no_serving:
        result["serving"] = serving_leg(1.0, [8 << 30, 64 << 20])

    if not args.no_cpu_baseline:
        import oracle  # the CPU-baseline leg: the oracle timed on the host

        planes_np = planes
        t0 = time.perf_counter()
        s_ref, m_ref = oracle.encode(planes_np, precs)
        t1 = time.perf_counter()
        oracle.decode(s_ref)
        t2 = time.perf_counter()
        identical = (s_ref == s_gpu) and bool(np.array_equal(m_ref, modes))
        result["byte_identical"] = identical
        result["cpu_baseline"] = {
            "value": round(points / (t2 - t0), 1), "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole workload ({T} scans x {A} attributes), encode + decode, one thread",
            "encode_s": round(t1 - t0, 2), "decode_s": round(t2 - t1, 2),
            "host_cpu": _cpu_model(), "host_cores": os.cpu_count(),
        }
        if not identical:
            print("[bench] GPU stream differs from the oracle", file=sys.stderr)
    print(json.dumps(result), flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
