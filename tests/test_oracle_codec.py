"""Pins for the oracle's whole codec: hand-derived streams, lossless round
trip (Sec. III-C: decoding reverses every step), exhaustive tiny inputs, the
trial heuristic against brute force (Sec. III-E), the quantization trade-off
(Sec. IV-G) and corrupt-input handling.  CPU only."""
import numpy as np
import pytest

import oracle
from conftest import hexbytes, load_golden
from formatcheck import read_record, split_stream
from paper_2209_08196_amd import synth

DT = {8: np.uint8, 16: np.uint16, 32: np.uint32}


def quant_ref(x, P, bits):
    """Expected decode output: the de-quantized quantized scan."""
    x = x.astype(np.uint64)
    q = np.where(x == 0, 0, np.maximum(1, (x + P // 2) // P))
    return np.minimum(q * P, (1 << bits) - 1).astype(DT[bits])


def de_bruijn(k, n):
    """de Bruijn sequence B(k, n) (every length-n word over k symbols once,
    cyclically), by the standard Lyndon-word construction."""
    a = [0] * k * n
    seq = []

    def db(t, p):
        if t > n:
            if n % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, k):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    return seq


# ----------------------------------------------------- hand-derived streams
def test_golden_tiny_streams():
    g = load_golden("tiny_streams.txt")
    s0 = np.array([[[0, 5, 6, 0, 0, 0, 4, 4]]], np.uint8)
    s1 = np.array([[[0, 5, 7, 0, 0, 3, 4, 0]]], np.uint8)
    one, m1 = oracle.encode([s0])
    assert one == hexbytes(g["one_scan"])
    assert m1.tolist() == [[0]]
    two, m2 = oracle.encode([np.concatenate([s0, s1])])
    assert two == hexbytes(g["two_scans_auto"])
    assert m2.tolist() == [[0], [1]]
    assert np.array_equal(oracle.decode(two)[0], np.concatenate([s0, s1]))


# ------------------------------------------------------ exhaustive tiny -----
@pytest.mark.parametrize("bits", [8, 16, 32])
@pytest.mark.parametrize("mode", [oracle.MODE_AUTO, oracle.MODE_I_ONLY, oracle.MODE_P_ONLY])
def test_every_2x2_pair_round_trips(bits, mode):
    # all 256 2x2 scans with values {0..3}; consecutive scans of a de Bruijn
    # sequence B(256, 2) cover all 65,536 (previous, current) pairs
    seq = de_bruijn(256, 2)
    seq = seq + seq[:1]
    vals = np.array(seq, np.int64)
    scans = np.stack([(vals >> (2 * k)) & 3 for k in range(4)], axis=1).reshape(-1, 2, 2)
    scale = {8: 60, 16: 16000, 32: 1 << 30}[bits]
    for P in (1, 3):
        x = (scans * scale).astype(DT[bits])
        s, modes = oracle.encode([x], [P], mode=mode)
        y = oracle.decode(s)[0]
        assert np.array_equal(y, quant_ref(x, P, bits))
        assert modes[0, 0] == 0
        if mode == oracle.MODE_P_ONLY:
            assert modes[1:].all()
        if mode == oracle.MODE_I_ONLY:
            assert not modes.any()


def test_random_streams_round_trip_all_widths():
    rng = np.random.default_rng(11)
    for it in range(40):
        H, W = int(rng.integers(1, 20)), int(rng.integers(1, 70))
        T = int(rng.integers(1, 5))
        widths = list(rng.choice([1, 2, 4], size=int(rng.integers(1, 4))))
        planes, precs = [], []
        for w in widths:
            dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[w]
            top = int(rng.choice([3, 255, np.iinfo(dt).max]))
            planes.append(synth.random_scans(rng, T, H, W, dt, float(rng.random()), scale=min(top, np.iinfo(dt).max)))
            precs.append(int(rng.choice([1, 1, 2, 7, 1000])))
        mode = int(rng.integers(3))
        s, modes = oracle.encode(planes, precs, mode=mode, trial_rows=int(rng.integers(0, 6)))
        out = oracle.decode(s)
        for x, y, p in zip(planes, out, precs):
            assert np.array_equal(y, quant_ref(x, p, 8 * x.dtype.itemsize))
        lay = oracle.make_layout(H, W, widths, precs)
        assert len(s) <= oracle.encode_bound(lay, T)


def test_bound_holds_on_incompressible_input():
    rng = np.random.default_rng(12)
    for dt in (np.uint8, np.uint16, np.uint32):
        x = rng.integers(0, np.iinfo(dt).max, (3, 37, 53), dtype=np.uint64).astype(dt)
        x[:, :, ::2] = 0
        x[1, 5:9] = 0
        s, _ = oracle.encode([x], mode=oracle.MODE_P_ONLY)
        lay = oracle.make_layout(37, 53, [x.dtype.itemsize])
        assert len(s) <= oracle.encode_bound(lay, 3)
        assert np.array_equal(oracle.decode(s)[0], x)


# ------------------------------------------------- record structure --------
def test_records_follow_the_step_definitions():
    """Reads the stream with the independent test-side reader and checks each
    record against the paper's steps: mask polarity (1 = out of range), mask
    XOR for P-scans, zero removal, temporal difference, delta, ZigZag."""
    g = synth.stream(1, 0)
    x = g.scans(0, 4)[0]
    P = 10
    for mode in (oracle.MODE_I_ONLY, oracle.MODE_P_ONLY, oracle.MODE_AUTO):
        s, modes = oracle.encode([x], [P], mode=mode)
        hdr, recs = split_stream(s)
        assert (hdr["H"], hdr["W"], hdr["T"], hdr["A"]) == (64, 1024, 4, 1)
        assert hdr["attrs"] == [(4, P)]
        npx = 64 * 1024
        Qprev, mprev = None, None
        for t, r in enumerate(recs):
            rec = read_record(r, 32, npx, mprev)
            assert rec["mode"] == modes[t, 0]
            q = np.where(x[t] == 0, 0, np.maximum(1, (x[t].astype(np.int64) + 5) // 10)).ravel()
            mask = np.packbits((q == 0).astype(np.uint8), bitorder="little").tobytes()
            content = rec["mask_content"]
            if rec["mode"] == 1:
                content = bytes(a ^ b for a, b in zip(content, mprev))
            assert content == mask
            nz = np.nonzero(q)[0]
            vals = q[nz] - (Qprev[nz] if rec["mode"] == 1 else 0)
            vals = vals & 0xFFFFFFFF
            d = (vals - np.concatenate([[0], vals[:-1]])) & 0xFFFFFFFF
            sd = np.where(d >= 1 << 31, d.astype(np.int64) - (1 << 32), d.astype(np.int64))
            zz = np.where(sd >= 0, 2 * sd, -2 * sd - 1)
            assert np.array_equal(rec["z"], zz.astype(np.uint64))
            Qprev, mprev = q, mask


def test_trial_with_all_rows_equals_bruteforce():
    # Sec. III-E: with the trial covering every scanline the heuristic must
    # pick the mode whose full residual section is smaller
    checked = 0
    for cid, sid in ((1, 0), (3, 1), (3, 0)):
        g = synth.stream(cid, sid)
        x = g.scans(0, 5)[0]
        H = x.shape[1]
        P = g.precisions[0]
        _, m_auto = oracle.encode([x], [P], trial_rows=H)
        si, _ = oracle.encode([x], [P], mode=oracle.MODE_I_ONLY)
        sp, _ = oracle.encode([x], [P], mode=oracle.MODE_P_ONLY)
        ri, rp = split_stream(si)[1], split_stream(sp)[1]
        npx = x.shape[1] * x.shape[2]
        for t in range(1, 5):
            ci = read_record(ri[t], 32, npx)["section_bytes"]
            cp = read_record(rp[t], 32, npx, read_record(ri[t - 1], 32, npx)["mask"])["section_bytes"]
            assert m_auto[t, 0] == (1 if cp < ci else 0)
            checked += 1
    assert checked == 12


def test_static_scene_prefers_p():
    rng = np.random.default_rng(13)
    x = synth.random_scans(rng, 1, 16, 64, np.uint16, 0.2)
    seq = np.concatenate([x, x, x])
    s, modes = oracle.encode([seq])
    assert modes[:, 0].tolist() == [0, 1, 1]
    recs = split_stream(s)[1]
    rec = read_record(recs[1], 16, 16 * 64, read_record(recs[0], 16, 16 * 64)["mask"])
    assert not rec["z"].any()  # identical scans leave all-zero P residuals


def test_attributes_are_independent_records():
    g = synth.stream(2, 0)
    planes = [p[:, :32, :256] for p in g.scans(0, 3)]
    s, modes = oracle.encode(planes)
    _, recs = split_stream(s)
    for a, p in enumerate(planes):
        s1, m1 = oracle.encode([p])
        _, r1 = split_stream(s1)
        for t in range(3):
            r = bytearray(recs[t * len(planes) + a])
            r[5] = 0  # the attribute index byte
            assert bytes(r) == r1[t]
            assert m1[t, 0] == modes[t, a]


def test_previous_scan_argument_matches_the_sequence_tail():
    g = synth.stream(3, 2)
    planes = g.scans(0, 4)
    s_all, m_all = oracle.encode(planes, g.precisions)
    s_tail, m_tail = oracle.encode([p[2:] for p in planes], g.precisions, prev=[p[1] for p in planes])
    assert split_stream(s_all)[1][4:] == split_stream(s_tail)[1]
    assert np.array_equal(m_all[2:], m_tail)


def test_open_ended_stream_without_length_table():
    g = synth.stream(1, 0)
    x = g.scans(0, 3)[0]
    s, _ = oracle.encode([x], [10])
    hdr, recs = split_stream(s)
    head = bytearray(s[:20 + 8])
    head[16:20] = (0).to_bytes(4, "little")
    open_s = bytes(head) + b"".join(recs)
    lay, T = oracle.peek(open_s)
    assert T == 3
    assert np.array_equal(oracle.decode(open_s)[0], oracle.decode(s)[0])


# ----------------------------------------------- Sec. IV-G, Fig. 4 ---------
def test_doubling_precision_saves_about_one_bit_per_sample():
    g = synth.stream(1, 0)
    x = g.scans(0, 3)[0]
    nz = int((x != 0).sum())
    bits = []
    for P in (2, 4, 8, 16, 32, 64):
        s, _ = oracle.encode([x], [P], mode=oracle.MODE_I_ONLY)
        bits.append(8 * len(s) / nz)
        y = oracle.decode(s)[0].astype(np.int64)
        ok = x >= (P + 1) // 2
        assert np.abs(y[ok] - x[ok]).max() <= P // 2
    steps = -np.diff(bits)
    assert np.all(steps > 0.5) and np.all(steps < 1.5), bits


# --------------------------------------------------- robustness ------------
def test_corrupt_streams_are_rejected_or_decoded_never_crash():
    g = synth.stream(1, 0)
    x = g.scans(0, 3)[0][:, :16, :256]
    s, _ = oracle.encode([x], [10])
    rng = np.random.default_rng(14)
    for cut in (0, 3, 19, 27, 40, len(s) // 2, len(s) - 1):
        with pytest.raises(oracle.OracleError):
            oracle.decode(s[:cut])
    ok = bad = 0
    for _ in range(300):
        b = bytearray(s)
        i = int(rng.integers(len(b)))
        b[i] ^= 1 << int(rng.integers(8))
        try:
            oracle.decode(bytes(b))
            ok += 1
        except oracle.OracleError as e:
            assert e.code == oracle.E_CORRUPT
            bad += 1
    assert bad > 0


def test_count_must_match_the_mask():
    x = np.array([[[0, 5, 6, 0, 0, 0, 4, 4]]], np.uint8)
    s = bytearray(oracle.encode([x])[0])
    hdr_len = 20 + 8 + 4
    sec = hdr_len + 24  # record header 12 + frame 10 + pad 2
    assert s[sec] == 4
    s[sec] = 5
    with pytest.raises(oracle.OracleError) as e:
        oracle.decode(bytes(s))
    assert e.value.code == oracle.E_CORRUPT


def test_p_scan_first_is_corrupt():
    x = np.array([[[0, 5, 6, 0, 0, 0, 4, 4]]], np.uint8)
    s = bytearray(oracle.encode([x])[0])
    s[32 + 4] = 1
    with pytest.raises(oracle.OracleError):
        oracle.decode(bytes(s))


def test_invalid_layouts():
    x = np.zeros((1, 2, 2), np.uint8)
    with pytest.raises(oracle.OracleError):
        oracle.encode([x], [0])
    with pytest.raises(oracle.OracleError):
        oracle.encode([np.zeros((1, 0, 2), np.uint8)])
    lay = oracle.make_layout(2, 2, [1] * 8)
    assert oracle.encode_bound(lay, 1) > 0
    lay.n_attrs = 9
    assert oracle.encode_bound(lay, 1) == 0
