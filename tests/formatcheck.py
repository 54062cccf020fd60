"""Test-side readers of the Jiffy stream, written independently of both the
oracle and the GPU library: a minimal RFC 8878 frame reader (Raw/RLE blocks),
a residual-section reader and a stream splitter.  Used to check the oracle's
output against the format definitions, and to compare GPU and oracle
streams record by record."""
import struct

import numpy as np


def u32(b, o):
    return struct.unpack_from("<I", b, o)[0]


def read_zstd_frame(b):
    """RFC 8878 sec. 3.1.1, restricted to what a Raw/RLE frame can hold.
    Returns (content, info dict)."""
    assert b[:4] == bytes([0x28, 0xB5, 0x2F, 0xFD]), "magic"
    fhd = b[4]
    fcs_flag, single, unused, reserved, checksum, dict_flag = (
        fhd >> 6, (fhd >> 5) & 1, (fhd >> 4) & 1, (fhd >> 3) & 1, (fhd >> 2) & 1, fhd & 3)
    assert reserved == 0
    p = 5
    if not single:
        p += 1  # Window_Descriptor
    p += [0, 1, 2, 4][dict_flag]
    fcs_size = [1 if single else 0, 2, 4, 8][fcs_flag]
    fcs = int.from_bytes(b[p:p + fcs_size], "little") if fcs_size else None
    if fcs_size == 2:
        fcs += 256
    p += fcs_size
    out = bytearray()
    blocks = []
    while True:
        h = b[p] | (b[p + 1] << 8) | (b[p + 2] << 16)
        p += 3
        last, btype, size = h & 1, (h >> 1) & 3, h >> 3
        assert btype in (0, 1), "only Raw and RLE blocks are expected"
        assert size <= 128 * 1024
        if btype == 0:
            out += b[p:p + size]
            p += size
        else:
            out += bytes([b[p]]) * size
            p += 1
        blocks.append(("raw" if btype == 0 else "rle", size))
        if last:
            break
    if checksum:
        p += 4
    assert p == len(b), "frame must end after its last block"
    if fcs is not None:
        assert fcs == len(out)
    return bytes(out), dict(fhd=fhd, fcs=fcs, blocks=blocks, single=single, checksum=checksum)


def read_section(b, bits, n_expected=None):
    """Residual section -> (z values, per-frame (b, n, B), byte length)."""
    n = u32(b, 0)
    if n_expected is not None:
        assert n == n_expected
    nb = (n + 127) // 128
    bb = list(b[4:4 + nb])
    nn = list(b[4 + nb:4 + 2 * nb])
    BB = list(b[4 + 2 * nb:4 + 3 * nb])
    p = (4 + 3 * nb + 3) & ~3
    pay = sum(16 * x for x in bb)
    npos = sum(nn)
    high = sum((e * (B - x) + 7) // 8 for x, e, B in zip(bb, nn, BB))
    pay_b, pos_b, high_b = b[p:p + pay], b[p + pay:p + pay + npos], b[p + pay + npos:p + pay + npos + high]
    z = []
    po = pp = ph = 0
    for j in range(nb):
        x, e, B = bb[j], nn[j], BB[j]
        assert x <= B <= bits and e <= 128
        blk = int.from_bytes(pay_b[po:po + 16 * x], "little")
        vals = [(blk >> (i * x)) & ((1 << x) - 1) for i in range(128)]
        hw = B - x
        hb = int.from_bytes(high_b[ph:ph + (e * hw + 7) // 8], "little")
        for k in range(e):
            i = pos_b[pp + k]
            vals[i] |= ((hb >> (k * hw)) & ((1 << hw) - 1)) << x
        z += vals[:min(128, n - 128 * j)]
        po += 16 * x
        pp += e
        ph += (e * hw + 7) // 8
    return np.array(z, dtype=np.uint64), list(zip(bb, nn, BB)), p + pay + npos + high


def split_stream(s):
    """-> (header dict, list of record bytes)."""
    assert s[:4] == b"JFY1"
    ver, A = struct.unpack_from("<HH", s, 4)
    H, W, T = struct.unpack_from("<III", s, 8)
    attrs = []
    p = 20
    for _ in range(A):
        attrs.append((s[p], u32(s, p + 4)))
        p += 8
    recs = []
    if T:
        lens = [u32(s, p + 4 * i) for i in range(T * A)]
        p += 4 * T * A
        for L in lens:
            recs.append(s[p:p + L])
            p += L
    else:
        while p < len(s):
            L = u32(s, p)
            recs.append(s[p:p + L])
            p += L
    assert p == len(s)
    return dict(version=ver, A=A, H=H, W=W, T=T, attrs=attrs), recs


def read_record(r, bits, npx, prev_mask=None):
    """-> dict(mode, attr, mask_content, mask, z, frames, section_bytes).
    For a P-record the mask is the content XOR prev_mask (when given)."""
    L = u32(r, 0)
    assert L == len(r) and L % 4 == 0
    mode, attr = r[4], r[5]
    flen = u32(r, 8)
    content, finfo = read_zstd_frame(r[12:12 + flen])
    sec = (12 + flen + 3) & ~3
    mask = content
    if mode == 1:
        mask = bytes(a ^ b for a, b in zip(content, prev_mask)) if prev_mask is not None else None
    nz = None if mask is None else npx - sum(bin(x).count("1") for x in mask)  # bit 1 = zero sample
    z, frames, used = read_section(r[sec:], bits, nz)
    assert sec + ((used + 3) & ~3) == L
    return dict(mode=mode, attr=attr, mask_content=content, mask=mask, frame=finfo, z=z, frames=frames,
                section_bytes=used - ((4 + 3 * len(frames) + 3) & ~3))
