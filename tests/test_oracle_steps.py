"""Pins for the oracle's single steps against what the paper and the
mathematics fix (closed forms, exhaustive checks, brute force, hand-derived
fixtures).  CPU only."""
import itertools

import numpy as np
import pytest

import oracle
from conftest import hexbytes, load_golden
from formatcheck import read_section, read_zstd_frame


# ---------------------------------------------------------------- Eq. 1 ----
@pytest.mark.parametrize("bits", [8, 16])
def test_zigzag_is_the_standard_interleave_exhaustive(bits):
    # Standard ZigZag (the map Eq. 1 names): 0,-1,1,-2,2,... -> 0,1,2,3,4,...
    # so the codes, ordered by value, enumerate the signed integers by
    # increasing magnitude, negatives first.
    seen = np.zeros(1 << bits, bool)
    half = 1 << (bits - 1)
    for x in range(-half, half):
        d = x & ((1 << bits) - 1)
        z = oracle.zigzag(d, bits)
        expect = 2 * abs(x) - (1 if x < 0 else 0)
        assert z == expect
        assert z < (1 << bits)
        seen[z] = True
        assert oracle.unzigzag(z, bits) == d
    assert seen.all()  # a bijection onto [0, 2^w)


def test_zigzag_32_sampled_and_extremes():
    rng = np.random.default_rng(1)
    for d in list(rng.integers(0, 1 << 32, 20000, dtype=np.uint64)) + [0, 1, 0x7FFFFFFF, 0x80000000,
                                                                      0xFFFFFFFF]:
        d = int(d)
        z = oracle.zigzag(d, 32)
        x = d - (1 << 32) if d >> 31 else d
        assert z == (2 * x if x >= 0 else -2 * x - 1)
        assert oracle.unzigzag(z, 32) == d


def test_zigzag_textbook_values():
    # the textbook sequence of the standard ZigZag map
    pairs = [(0, 0), (-1, 1), (1, 2), (-2, 3), (2, 4), (2147483647, 4294967294), (-2147483648, 4294967295)]
    for x, z in pairs:
        assert oracle.zigzag(x & 0xFFFFFFFF, 32) == z


# --------------------------------------------------------- Sec. III-B ------
@pytest.mark.parametrize("P", [1, 2, 3, 10, 1000])
def test_quantize_error_bound_exhaustive(P):
    # Sec. III-B / Fig. 4: the round-trip error is at most half the precision;
    # P = 1 is the identity; zero (invalid) stays zero; valid stays valid.
    xs = np.arange(1, 1_000_001, dtype=np.uint64)
    q = (xs + P // 2) // P  # the same reading written out on arrays
    q = np.maximum(q, 1)
    step = max(1, len(xs) // 2000)
    for x in list(xs[::step]) + [1, P // 2, P // 2 + 1, P, P + 1, 999_999, 1_000_000]:
        x = int(x)
        if x == 0:
            continue
        qq = oracle.quantize(x, P)
        assert qq >= 1
        assert qq == q[x - 1]
        back = oracle.dequantize(qq, P, 32)
        if x >= (P + 1) // 2:
            assert abs(back - x) <= P // 2
    # exhaustively on the array form: the bound and monotonicity
    back = q * P
    ok = xs >= (P + 1) // 2
    assert np.all(np.abs(back[ok].astype(np.int64) - xs[ok].astype(np.int64)) <= P // 2)
    assert np.all(np.diff(q) >= 0)
    assert oracle.quantize(0, P) == 0
    if P == 1:
        assert np.all(q == xs)


def test_quantize_sampled_against_oracle_exhaustive_small():
    for P in (1, 2, 3, 7, 10):
        for x in range(0, 5000):
            q = oracle.quantize(x, P)
            if x == 0:
                assert q == 0
            else:
                assert q == max(1, (x + P // 2) // P)
                # nearest multiple of P (halves up) unless clamped to 1
                if x >= (P + 1) // 2:
                    cands = [k * P for k in range(max(0, x // P - 1), x // P + 3)]
                    best = min(cands, key=lambda c: (abs(c - x), -c))
                    assert q * P == best


def test_dequantize_saturates():
    assert oracle.dequantize(26, 10, 8) == 255
    assert oracle.dequantize(25, 10, 8) == 250
    assert oracle.dequantize(70000, 1, 16) == 65535
    assert oracle.dequantize(5, 3, 32) == 15


# --------------------------------------------------------- Sec. II PFOR ----
def _pack_block(z, b):
    """Independent byte-exact packer for one frame at a given b: LSB-first
    payload, exception positions, high parts.  Returns its length."""
    payload = 0
    for i, v in enumerate(z):
        payload |= (int(v) & ((1 << b) - 1)) << (i * b)
    B = max(int(v).bit_length() for v in z)
    exc = [i for i, v in enumerate(z) if int(v) >> b]
    high = 0
    for k, i in enumerate(exc):
        high |= (int(z[i]) >> b) << (k * (B - b))
    nhigh = (len(exc) * (B - b) + 7) // 8 if exc else 0
    return 16 * b + len(exc) + nhigh, payload.to_bytes(16 * b, "little"), bytes(exc), high.to_bytes(nhigh, "little")


def _frames(rng):
    yield np.zeros(128, np.uint32)
    yield np.full(128, 0xFFFFFFFF, np.uint32)
    yield np.arange(128, dtype=np.uint32)
    for _ in range(300):
        kind = rng.integers(4)
        if kind == 0:
            z = rng.geometric(0.05, 128).astype(np.uint32)
        elif kind == 1:
            z = rng.integers(0, 16, 128).astype(np.uint32)
            idx = rng.choice(128, rng.integers(1, 9), replace=False)
            z[idx] = rng.integers(1 << 10, 1 << 31, len(idx))
        elif kind == 2:
            z = rng.integers(0, 1 << int(rng.integers(1, 33)), 128, dtype=np.uint64).astype(np.uint32)
        else:
            z = np.zeros(128, np.uint32)
            z[rng.integers(128)] = rng.integers(1, 1 << 32, dtype=np.uint64)
        yield z


def test_pfor_choice_is_bruteforce_argmin_of_packed_bytes():
    rng = np.random.default_rng(2)
    for z in _frames(rng):
        b, n, B, cost = oracle.pfor_choose(z)
        assert B == max(int(v).bit_length() for v in z)
        sizes = {bb: _pack_block(z, bb)[0] for bb in range(0, B + 1)}
        best = min(sizes.values())
        assert cost == sizes[b] == best
        assert b == max(bb for bb, s in sizes.items() if s == best)  # ties -> larger b
        assert n == sum(1 for v in z if int(v) >> b)


def test_pfor_section_matches_independent_packer_and_reader():
    rng = np.random.default_rng(3)
    for n in [0, 1, 5, 127, 128, 129, 300, 1000]:
        z = rng.geometric(0.02, n).astype(np.uint32)
        if n > 3:
            z[rng.integers(n)] = 0xFFFFFFFF
        sec = oracle.pfor_encode(z)
        zz, frames, used = read_section(sec, 32, n)
        assert used == len(sec)
        assert np.array_equal(zz, z.astype(np.uint64))
        # byte-exact against the independent packer, frame by frame
        nb = (n + 127) // 128
        hdr = (4 + 3 * nb + 3) & ~3
        pay = pos = high = b""
        for j in range(nb):
            f = np.zeros(128, np.uint32)
            part = z[128 * j:128 * j + 128]
            f[:len(part)] = part
            _, p, e, h = _pack_block(f, frames[j][0])
            pay, pos, high = pay + p, pos + e, high + h
        assert sec[hdr:] == pay + pos + high
        assert sec[:4] == n.to_bytes(4, "little")
        # closed form of the size
        assert len(sec) == hdr + sum(oracle.pfor_choose(np.pad(z[128 * j:128 * j + 128],
                                                              (0, 128 - len(z[128 * j:128 * j + 128]))))[3]
                                     for j in range(nb))
        back, used2 = oracle.pfor_decode(sec, 32, n)
        assert np.array_equal(back, z) and used2 == len(sec)


def test_pfor_special_cases():
    # all zero -> b = 0, no payload, no exceptions
    assert oracle.pfor_choose(np.zeros(128, np.uint32))[:4] == (0, 0, 0, 0)
    # values below 2^b with one dominant width -> plain bit packing
    z = np.full(128, 5, np.uint32)
    b, n, B, cost = oracle.pfor_choose(z)
    assert (b, n, B, cost) == (3, 0, 3, 48)
    sec = oracle.pfor_encode(z)
    payload = sec[8:]
    assert payload == int("".join(["101"] * 128)[::-1], 2).to_bytes(48, "little")


def test_pfor_golden_frame():
    g = load_golden("frames_and_frames128.txt")
    z = np.ones(128, np.uint32)
    z[127] = 1000
    assert oracle.pfor_encode(z) == hexbytes(g["frame128"])


# ---------------------------------------------- Sec. III-C mask frame ------
def _runs(c):
    out, i = [], 0
    while i < len(c):
        j = i
        while j < len(c) and c[j] == c[i]:
            j += 1
        out.append((c[i], j - i))
        i = j
    return out


def _mask_contents(rng):
    yield b"\x00"
    yield b"\xff" * 8
    yield b"\x01\x02\x03"
    yield bytes(7) + b"\x01"
    yield bytes(8) + b"\x01"
    yield bytes(255)
    yield bytes(256)
    yield bytes(65791)
    yield bytes(65792)
    yield b"\xaa" * 131072
    yield b"\x00" * 131073 + b"\x01" * 5
    yield bytes(rng.integers(0, 256, 200000, dtype=np.uint8))
    for _ in range(60):
        n = int(rng.integers(1, 5000))
        parts = []
        while sum(map(len, parts)) < n:
            if rng.random() < 0.5:
                parts.append(bytes([int(rng.integers(256))]) * int(rng.integers(1, 40)))
            else:
                parts.append(bytes(rng.integers(0, 4, int(rng.integers(1, 30)), dtype=np.uint8)))
        yield b"".join(parts)[:n]


def test_frame_is_valid_rfc8878_and_follows_the_block_rule():
    rng = np.random.default_rng(4)
    for c in _mask_contents(rng):
        f = oracle.frame(c)
        content, info = read_zstd_frame(f)
        assert content == c
        assert info["single"] == 1 and info["checksum"] == 0
        n = len(c)
        fhd = info["fhd"]
        assert fhd == (0x20 if n <= 255 else 0x60 if n <= 65791 else 0xA0)
        # the block rule: long runs are RLE, everything else Raw, no two Raw
        # blocks adjacent unless split at 128 KiB
        expect = []
        raw = 0
        for byte, ln in _runs(c):
            if ln >= 8:
                if raw:
                    expect.append(("raw", raw))
                    raw = 0
                expect.append(("rle", ln))
            else:
                raw += ln
        if raw:
            expect.append(("raw", raw))
        split = []
        for kind, ln in expect:
            while ln > 131072:
                split.append((kind, 131072))
                ln -= 131072
            split.append((kind, ln))
        assert info["blocks"] == split
        assert oracle.unframe(f, n) == c
        # the size bound used for output buffers
        assert len(f) <= 16 + n + 4 * (n // 131072 + 1)


def test_frame_golden():
    g = load_golden("frames_and_frames128.txt")
    assert oracle.frame(hexbytes(g["frame_mixed_content"])) == hexbytes(g["frame_mixed"])
    assert oracle.frame(b"\xff" * 300) == hexbytes(g["frame_rle300"])


def test_unframe_rejects_malformed():
    good = oracle.frame(bytes(20) + b"\x05")
    bad = [
        good[:-1],                      # truncated
        good + b"\x00",                 # trailing byte
        b"\x00" + good[1:],             # magic
        good[:4] + bytes([good[4] | 0x04]) + good[5:],   # checksum flag
        good[:4] + bytes([good[4] | 0x08]) + good[5:],   # reserved bit
        good[:4] + bytes([good[4] & ~0x20 & 0xFF]) + good[5:],  # not single segment
    ]
    # a compressed block type
    hb = bytearray(good)
    hb[6] = (hb[6] & ~0x06) | 0x04
    bad.append(bytes(hb))
    for b in bad:
        with pytest.raises(oracle.OracleError):
            oracle.unframe(b, 21)
    with pytest.raises(oracle.OracleError):
        oracle.unframe(good, 22)  # content size mismatch


# ------------------------------------------------ Sec. III-E trial rows ----
def test_trial_rows_band_centres():
    assert oracle.trial_rows(128, 4) == [16, 48, 80, 112]
    assert oracle.trial_rows(16, 4) == [2, 6, 10, 14]
    assert oracle.trial_rows(1, 4) == [0]
    assert oracle.trial_rows(3, 4) == [0, 1, 2]
    for H in range(1, 40):
        for K in range(H, H + 3):
            assert oracle.trial_rows(H, K) == list(range(H))  # K >= H covers every row
        for K in range(1, 9):
            rows = oracle.trial_rows(H, K)
            assert rows == sorted(set(rows)) and all(0 <= r < H for r in rows)


# ------------------------------------------------ delta / prefix inverse ---
@pytest.mark.parametrize("bits", [8, 16, 32])
def test_delta_zigzag_then_prefix_sum_inverts(bits):
    rng = np.random.default_rng(5)
    m = (1 << bits) - 1
    s = [int(v) for v in rng.integers(0, 1 << bits, 500, dtype=np.uint64)]
    prev, z = 0, []
    for v in s:
        z.append(oracle.zigzag((v - prev) & m, bits))
        prev = v
    acc, back = 0, []
    for zz in z:
        acc = (acc + oracle.unzigzag(zz, bits)) & m
        back.append(acc)
    assert back == s


def test_all_pairs_tiny_exhaustive_zigzag_delta():
    for bits in (8,):
        m = (1 << bits) - 1
        for a, b in itertools.product(range(0, 256, 5), repeat=2):
            d = (b - a) & m
            assert (a + oracle.unzigzag(oracle.zigzag(d, bits), bits)) & m == b
