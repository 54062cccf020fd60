"""GPU parity: the HIP library's streams are byte-identical to the oracle's,
with the same I/P decisions, and its decoder restores the oracle's output
exactly.  Every call goes through the C ABI (libjiffy.so)."""
import numpy as np
import pytest

import oracle
from conftest import hexbytes, load_golden
from formatcheck import split_stream
from gpu_util import banner, to_dev, to_host
from paper_2209_08196_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()  # raises if the library is missing
    return jiffy


def gpu_encode(J, planes, precs, mode=0, trial_rows=0):
    dev = [to_dev(p) for p in planes]
    out, modes = J.encode(dev, precs, mode=mode, trial_rows=trial_rows)
    return out.cpu().numpy().tobytes(), modes


def check_case(J, planes, precs, mode=0, trial_rows=0, name=""):
    banner("encode", name, [p.shape for p in planes], [p.dtype.name for p in planes], precs, "mode", mode)
    s_ref, m_ref = oracle.encode(planes, precs, mode=mode, trial_rows=trial_rows)
    s_gpu, m_gpu = gpu_encode(J, planes, precs, mode, trial_rows)
    assert np.array_equal(m_gpu, m_ref), (m_gpu.ravel()[:40], m_ref.ravel()[:40])
    if s_gpu != s_ref:
        _, rg = split_stream(s_gpu)
        _, rr = split_stream(s_ref)
        bad = [i for i, (a, b) in enumerate(zip(rg, rr)) if a != b]
        raise AssertionError(f"{name}: streams differ ({len(s_gpu)} vs {len(s_ref)} bytes); records {bad[:10]}")
    return s_ref


def test_golden_tiny_streams(J):
    g = load_golden("tiny_streams.txt")
    s0 = np.array([[[0, 5, 6, 0, 0, 0, 4, 4]]], np.uint8)
    s1 = np.array([[[0, 5, 7, 0, 0, 3, 4, 0]]], np.uint8)
    banner("golden tiny")
    s, m = gpu_encode(J, [s0], [1])
    assert s == hexbytes(g["one_scan"])
    s, m = gpu_encode(J, [np.concatenate([s0, s1])], [1])
    assert s == hexbytes(g["two_scans_auto"])
    assert m.tolist() == [[0], [1]]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_plain_64x1024_range_1cm(J, mode):
    g = synth.stream(1, 0)
    x = g.scans(0, 10)
    check_case(J, x, g.precisions, mode=mode, name=f"c1 mode{mode}")


def test_dual_return_128x2048_five_attributes_first_scans(J):
    g = synth.stream(2, 0)
    planes = g.scans(0, 4)
    for mode in (0, 1, 2):
        check_case(J, planes, g.precisions, mode=mode, name=f"c2x4 mode{mode}")


def _ragged_cases():
    rng = np.random.default_rng(21)
    cases = [
        (1, 1, 1, [1], 0.0, [1], 0), (2, 1, 1, [4], 0.5, [1], 2), (3, 1, 7, [2], 0.3, [3], 0),
        (2, 3, 5, [1, 2, 4], 0.2, [1, 2, 1000], 0), (3, 17, 129, [4], 0.1, [10], 0),
        (3, 200, 33, [2], 0.6, [1], 2), (2, 5, 4097, [4, 1], 0.05, [7, 1], 1), (2, 64, 64, [4], 1.0, [1], 0),
        (2, 64, 64, [4], 0.0, [1], 2), (3, 1, 300, [4], 0.0, [1], 0), (4, 33, 257, [2, 2], 0.45, [1, 5], 0),
    ]
    for T, H, W, widths, zf, precs, mode in cases:
        planes = []
        for w in widths:
            dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[w]
            planes.append(synth.random_scans(rng, T, H, W, dt, zf))
        yield (T, H, W, widths, zf, precs, mode), planes
    # smooth data so that P-scans and narrow frames occur
    for k in range(4):
        T, H, W = 3, int(rng.integers(1, 90)), int(rng.integers(1, 700))
        base = np.cumsum(rng.integers(-3, 4, size=(H, W)), axis=1) + 5000
        planes = []
        for t in range(T):
            v = base + rng.integers(-2, 3, size=(H, W)) * (t % 2)
            v[rng.random((H, W)) < 0.2] = 0
            planes.append(np.clip(v, 0, None))
        yield (T, H, W, "smooth", k), [np.stack(planes).astype(np.uint32)]


def test_ragged_and_degenerate_shapes(J):
    for desc, planes in _ragged_cases():
        precs = desc[5] if len(desc) > 5 and isinstance(desc[5], list) else [1] * len(planes)
        mode = desc[6] if len(desc) > 6 else 0
        check_case(J, planes, precs, mode=mode, name=str(desc))


def test_extreme_values_and_trial_rows(J):
    rng = np.random.default_rng(22)
    x = rng.integers(0, 2**32, size=(3, 9, 301), dtype=np.uint64).astype(np.uint32)
    x[:, :, ::3] = 0
    x[1, 2] = 0xFFFFFFFF
    for P in (1, 2, 3, 0xFFFFFFFF, 1000003):
        check_case(J, [x], [P], name=f"u32 extreme P={P}")
    y = rng.integers(0, 2**16, size=(4, 40, 100), dtype=np.uint64).astype(np.uint16)
    for k in (1, 3, 4, 39, 40, 1000):
        check_case(J, [y, y.copy()], [1, 3], trial_rows=k, name=f"trial_rows={k}")


def test_decode_round_trip_and_cross_decode(J):
    import torch
    g = synth.stream(2, 1)
    planes = g.scans(0, 5)
    s_ref, _ = oracle.encode(planes, g.precisions)
    ref = oracle.decode(s_ref)
    banner("decode c2x5")
    dev_stream = torch.from_numpy(np.frombuffer(s_ref, np.uint8).copy()).cuda()
    outs = J.decode(dev_stream)
    for a, (o, r) in enumerate(zip(outs, ref)):
        assert np.array_equal(to_host(o, r.dtype.itemsize), r), a
    # P > 1 and forced P-scans
    g1 = synth.stream(1, 3)
    x = g1.scans(0, 6)
    for mode in (0, 1, 2):
        banner("decode c1 mode", mode)
        s_ref, _ = oracle.encode(x, [10], mode=mode)
        ref = oracle.decode(s_ref)[0]
        s_gpu, _ = gpu_encode(J, x, [10], mode)
        assert s_gpu == s_ref
        outs = J.decode(torch.from_numpy(np.frombuffer(s_gpu, np.uint8).copy()).cuda())
        assert np.array_equal(to_host(outs[0], 4), ref)


def test_decode_ragged(J):
    import torch
    for desc, planes in _ragged_cases():
        precs = desc[5] if len(desc) > 5 and isinstance(desc[5], list) else [1] * len(planes)
        mode = desc[6] if len(desc) > 6 else 0
        banner("decode", desc)
        s_ref, _ = oracle.encode(planes, precs, mode=mode)
        ref = oracle.decode(s_ref)
        outs = J.decode(torch.from_numpy(np.frombuffer(s_ref, np.uint8).copy()).cuda())
        for o, r in zip(outs, ref):
            assert np.array_equal(to_host(o, r.dtype.itemsize), r), desc


def test_stream_api_matches_whole_sequence_encoding(J):
    import torch
    shapes = [(16, 1024), (32, 2048), (64, 1024), (7, 301)]
    gens = [synth.stream(3, s, size=shapes[s]) for s in range(len(shapes))]
    T = 4
    data = [g.scans(0, T) for g in gens]
    streams = [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]
    outs = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in streams]
    got = [[] for _ in gens]
    for t in range(T):
        banner("batch step", t)
        if t == 2:
            streams[1].reset()
        scans = [[to_dev(p[t]) for p in d] for d in data]
        lens, modes = J.batch_encode_step(streams, scans, outs)
        for i in range(len(gens)):
            got[i].append(outs[i][: lens[i]].cpu().numpy().tobytes())
    for i, g in enumerate(gens):
        if i == 1:
            s0, _ = oracle.encode([p[:2] for p in data[i]], g.precisions)
            s1, _ = oracle.encode([p[2:] for p in data[i]], g.precisions)
            recs = split_stream(s0)[1] + split_stream(s1)[1]
        else:
            s, _ = oracle.encode(data[i], g.precisions)
            recs = split_stream(s)[1]
        A = len(g.widths)
        for t in range(T):
            assert got[i][t] == b"".join(recs[t * A:(t + 1) * A]), (i, t)
    for s in streams:
        s.close()


def test_deterministic_repeat(J):
    g = synth.stream(2, 2)
    planes = g.scans(0, 3)
    a, _ = gpu_encode(J, planes, g.precisions)
    b, _ = gpu_encode(J, planes, g.precisions)
    assert a == b


def test_stress_128x4096_first_scans(J):
    g = synth.stream(5, 0)
    planes = g.scans(18, 22)  # crosses a scene cut at scan 20
    check_case(J, planes, g.precisions, name="c5 scans 18-21")


def test_incompressible_tiles(J):
    """Full-range random samples: frames near 32 bits wide, so a decode tile's
    packed bytes exceed what the decoder stages in LDS and it reads them
    from the record instead."""
    import torch
    rng = np.random.default_rng(31)
    x = rng.integers(1, 2**32, size=(3, 64, 1024), dtype=np.uint64).astype(np.uint32)
    x[1, :, 100:140] = 0
    y = rng.integers(0, 2**16, size=(3, 64, 1024), dtype=np.uint64).astype(np.uint16)
    for mode in (0, 2):
        s_ref = check_case(J, [x, y], [1, 1], mode=mode, name=f"random u32+u16 mode {mode}")
        ref = oracle.decode(s_ref)
        banner("decode random, mode", mode)
        outs = J.decode(torch.from_numpy(np.frombuffer(s_ref, np.uint8).copy()).cuda())
        for o, r in zip(outs, ref):
            assert np.array_equal(to_host(o, r.dtype.itemsize), r)


def test_large_masks_split_blocks(J):
    """Mask content over 128 KiB: RLE runs and Raw stretches split at the
    block limit, frames spanning many parse windows; encode and decode."""
    import torch
    rng = np.random.default_rng(41)
    H, W = 1024, 1280
    full = rng.integers(1, 256, size=(2, H, W), dtype=np.uint64).astype(np.uint8)  # no zeros: one long run
    sparse = full.copy()
    sparse[:, rng.random((H, W)) < 0.5] = 0  # random mask bytes: Raw blocks
    blocky = full.copy()
    blocky[1, 100:700] = 0  # a P-scan whose XOR mask has long runs
    for name, x in (("full", full), ("sparse", sparse), ("blocky", blocky)):
        s_ref = check_case(J, [x], [1], name=f"large mask {name}")
        ref = oracle.decode(s_ref)[0]
        banner("decode large mask", name)
        out = J.decode(torch.from_numpy(np.frombuffer(s_ref, np.uint8).copy()).cuda())[0]
        assert np.array_equal(to_host(out, 1), ref), name


@pytest.mark.parametrize("T", [33, 65, 600])
def test_long_mask_chains(J, T):
    """P-scan mask chains across many scans (the decoder's mask pass splits
    time into chunks of 32 scans and rounds of 512): forced P-scans, and a
    mix where static stretches (P) alternate with fresh noise (I)."""
    import torch
    rng = np.random.default_rng(T)
    base = synth.random_scans(rng, 1, 4, 40, np.uint16, 0.4, scale=500)
    x = np.repeat(base, T, axis=0)
    flips = rng.random(x.shape) < 0.05  # zeros appear and disappear: every XOR mask differs
    x = np.where(flips, np.where(x == 0, 7, 0), x).astype(np.uint16)
    noisy = rng.random(T) < 0.1
    x[noisy] = synth.random_scans(rng, int(noisy.sum()), 4, 40, np.uint16, 0.4, scale=500)
    for mode in (2, 0):
        banner("long mask chain", T, "mode", mode)
        s_ref, m = oracle.encode([x], [1], mode=mode)
        if mode == 2:
            assert m[1:].all()
        out = J.decode(torch.from_numpy(np.frombuffer(s_ref, np.uint8).copy()).cuda())[0]
        assert np.array_equal(to_host(out, 2), x), (T, mode)
