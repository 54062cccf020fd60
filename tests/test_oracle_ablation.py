"""Oracle pins of the ablated codecs (Sec. IV-H, Table IV) and of the
run-length mask codec.

Level 3 (delta, ZigZag, PFOR over every pixel) of a scan with no zeros is
the codec's I-record with its mask frame taken out, so it is checked
against the full encoder's records; levels 1-3 have closed forms on
constant scans and falling ramps (a wrong delta sign, a missing ZigZag or
a wrong width fails them); the run-length values are checked against a
plain loop, against hand-derived sections (``tests/golden/rl_masks.txt``)
and by decoding them back to the mask."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import ablation as ab
from formatcheck import split_stream, u32
from paper_2209_08196_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rl_masks.txt")


def _golden():
    kv = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    cases = []
    for name in sorted({k.split("_")[1] for k in kv}):
        b = kv[f"rl_{name}_bits"]
        bits = np.zeros(1000, bool) if b == "zeros1000" else np.array([c == "1" for c in b])
        vals = [int(t) for t in kv[f"rl_{name}_values"].split()]
        cases.append((name, bits, vals, bytes.fromhex(kv[f"rl_{name}"].replace(" ", ""))))
    return cases


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[0])
def test_run_length_golden(case):
    _, bits, vals, section = case
    assert list(ab.run_values(bits)) == vals
    assert oracle.pfor_encode(np.array(vals, np.uint32)) == section
    assert ab.rl_mask_bytes(bits) == ab.pad4(len(section))


def _runs_by_loop(bits):
    out, cur, n = [], False, 0
    for b in bits:
        if b == cur:
            n += 1
        else:
            out.append(n)
            cur, n = b, 1
    out.append(n)
    return [out[0]] + [r - 1 for r in out[1:]]


def test_run_values_match_a_loop_and_invert():
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 64, 129, 1000):
        for kind in ("iid", "clustered", "ones", "zeros"):
            if kind == "iid":
                bits = rng.random(n) < 0.3
            elif kind == "clustered":
                bits = np.repeat(rng.random(n // 8 + 1) < 0.5, 8)[:n]
            else:
                bits = np.full(n, kind == "ones")
            v = ab.run_values(bits)
            assert list(v) == _runs_by_loop(bits), (n, kind)
            assert np.array_equal(ab.runs_to_bits(v, n), bits)
            assert int(v.sum()) + len(v) - 1 == n


def test_vector_quantizer_equals_the_scalar_one():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 1 << 32, 2000, dtype=np.uint64)
    x[::7] = 0
    for P in (1, 2, 3, 10, 1000, (1 << 31) + 3):
        q = ab.quantize_plane(x, P)
        assert [int(a) for a in q] == [oracle.quantize(int(a), P) for a in x]


def test_vector_zigzag_equals_the_scalar_one():
    rng = np.random.default_rng(4)
    for bits in (8, 16, 32):
        d = rng.integers(0, 1 << bits, 3000, dtype=np.uint64)
        assert [int(a) for a in ab.zigzag(d, bits)] == [oracle.zigzag(int(a), bits) for a in d]


@pytest.mark.parametrize("dtype,P", [(np.uint32, 1), (np.uint16, 1), (np.uint8, 1), (np.uint32, 10)])
def test_level3_is_the_i_record_without_its_mask(dtype, P):
    """With no zero samples the mask removes nothing: the I-record's residual
    section codes the same vector as level 3."""
    rng = np.random.default_rng(8)
    g = synth.stream(2, 0)
    planes = [p[:3, :20, :300] for p in g.scans(0, 3)]
    x = planes[0].astype(np.uint64)
    x = np.where(x == 0, rng.integers(1, 40000, x.shape), x)
    top = np.iinfo(dtype).max
    x = np.minimum(x, top).astype(dtype)
    s, _ = oracle.encode([x], [P], mode=oracle.MODE_I_ONLY)
    _, recs = split_stream(s)
    for t, r in enumerate(recs):
        mlen = u32(r, 8)
        assert ab.levels(x[t], P, 8 * np.dtype(dtype).itemsize)[2] == len(r) - ab.pad4(mlen), t


def _hdr(nb):
    return 4 + ab.pad4(3 * nb)


def test_closed_forms_constant_scan():
    H, W = 4, 96  # 384 pixels, three full frames
    nb = 3
    for dtype, c in ((np.uint32, 1000), (np.uint32, 1), (np.uint16, 65000), (np.uint8, 200)):
        bits = 8 * np.dtype(dtype).itemsize
        B = c.bit_length()
        lv = ab.levels(np.full((H, W), c, dtype), 1, bits)
        assert lv[0] == 12 + ab.pad4(_hdr(nb) + nb * 16 * B)
        assert lv[1] == 12 + ab.pad4(_hdr(nb) + 1 + math.ceil(B / 8))  # c, then zeros
        zz = 2 * c if c < (1 << (bits - 1)) else 2 * ((1 << bits) - c) - 1
        assert lv[2] == 12 + ab.pad4(_hdr(nb) + 1 + math.ceil(zz.bit_length() / 8))


def test_closed_forms_falling_ramp():
    n = 512
    nb = n // 128
    for dtype in (np.uint32, np.uint16):
        bits = 8 * np.dtype(dtype).itemsize
        x = (n - np.arange(n)).astype(dtype).reshape(4, 128)
        lv = ab.levels(x, 1, bits)
        # deltas n, then -1 = 2^w - 1: every frame at full width
        assert lv[1] == 12 + ab.pad4(_hdr(nb) + nb * 16 * bits)
        # ZigZag: 2n, then ones: one exception in the first frame, width 1
        B0 = (2 * n).bit_length()
        assert lv[2] == 12 + ab.pad4(_hdr(nb) + 17 + math.ceil((B0 - 1) / 8) + (nb - 1) * 16)


def test_ablate_masks_and_first_scan():
    g = synth.stream(1, 0)
    x = g.scans(0, 3)[0][:, :16, :256]
    still = np.repeat(x[:1], 3, axis=0)
    for planes in ([x], [still]):
        r = ab.ablate(planes, [10])
        assert r.shape == (3, 1, 5)
        assert r[0, 0, 4] == r[0, 0, 3]
    n = 16 * 256
    # a standing sensor's mask repeats: the XOR mask is one run of n pixels
    r = ab.ablate([still], [10])
    assert (r[1:, 0, 4] == ab.pad4(8 + 1 + math.ceil(n.bit_length() / 8))).all()


def test_ablation_order_on_range_scans():
    """On range scans with zeros (c1 sizes) each added stage shrinks the
    records the way the ablation table reports: ZigZag repairs delta coding,
    the mask beats coding the zeros (its frame counted)."""
    g = synth.stream(1, 0)
    x = g.scans(0, 4)[0]
    r = ab.ablate([x], [10])[:, 0].astype(np.int64)
    s, _ = oracle.encode([x], [10], mode=oracle.MODE_I_ONLY)
    i_rec = np.array([len(t) for t in split_stream(s)[1]])
    assert (r[:, 2] < r[:, 1]).all()
    assert (i_rec < r[:, 2]).all()
