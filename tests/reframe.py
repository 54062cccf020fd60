"""Test-side re-framing of a Jiffy stream: every record's mask frame is
written again with other Raw/RLE block boundaries (all of them valid RFC 8878
blocks holding the same content), the record's length fields and the stream's
record-length table follow.  A decoder must give the same samples for the
re-framed stream as for the original; the block walk of the mask-frame parse
then meets blocks it never sees in the library's own frames: RLE blocks of
any length from 1, raw blocks of one byte or of thousands, blocks of no
content, blocks that run through several parse windows.

The new frame keeps the original frame header and stays within the frame
length the decoder accepts for the record's pixel count (16 + n + 4 (n / 2^17
+ 1) bytes for n content bytes, the longest frame any encoder here writes)."""
import struct

import numpy as np

from formatcheck import read_zstd_frame, split_stream, u32

ZBLOCK_MAX = 128 * 1024

POLICIES = ("mixed", "tiny", "one_raw", "long_rle")


def frame_bound(n):
    return 16 + n + 4 * (n // ZBLOCK_MAX + 1)


def _run_at(c, i):
    """Length of the run of equal bytes starting at i."""
    v = c[i]
    j = i + 1
    while j < len(c) and c[j] == v and j - i < ZBLOCK_MAX:
        j += 1
    return j - i


def _blocks(content, rng, policy, budget):
    """A list of (kind, start, size) covering content in order.  Runs of four
    or more equal bytes are RLE blocks, the stretches between them raw blocks
    (none longer than the format allows); other policies split them further,
    each split spent from a budget of extra frame bytes: an RLE run cut in two
    costs four, one more raw piece or a block without content three."""
    n = len(content)
    out = []
    if policy == "one_raw":  # the whole content as raw blocks of the largest size
        for i in range(0, n, ZBLOCK_MAX):
            out.append(("raw", i, min(ZBLOCK_MAX, n - i)))
        return out
    i = 0
    while i < n:
        run = _run_at(content, i)
        if run >= 4:
            if policy != "long_rle" and budget >= 4 and rng.random() < 0.3:
                cut = int(rng.integers(1, run))
                out += [("rle", i, cut), ("rle", i + cut, run - cut)]
                budget -= 4
            else:
                out.append(("rle", i, run))
            i += run
            continue
        j = i  # the raw stretch: up to the next run of four or more
        while j < n:
            r = _run_at(content, j)
            if r >= 4:
                break
            j += r
        while i < j:
            rem = j - i
            if policy == "long_rle" or budget < 3:
                s = min(rem, ZBLOCK_MAX)
            else:
                s = min(int(rng.integers(1, (4 if policy == "tiny" else 64) + 1)), rem, ZBLOCK_MAX)
                if s < rem:
                    budget -= 3
            out.append(("raw", i, s))
            i += s
            if policy == "tiny" and budget >= 3 and rng.random() < 0.05:
                out.append(("raw", i, 0))  # a block with no content
                budget -= 3
    return out


def _emit(content, blocks):
    b = bytearray()
    for k, (kind, start, size) in enumerate(blocks):
        last = 1 if k + 1 == len(blocks) else 0
        h = last | ((1 if kind == "rle" else 0) << 1) | (size << 3)
        b += bytes((h & 0xFF, (h >> 8) & 0xFF, (h >> 16) & 0xFF))
        b += content[start:start + 1] if kind == "rle" else content[start:start + size]
    return bytes(b)


def reframe_frame(frame, rng, policy):
    content, info = read_zstd_frame(frame)
    fcs_size = [1, 2, 4, 8][info["fhd"] >> 6]
    head = frame[:5 + fcs_size]
    n = len(content)
    compact = _emit(content, _blocks(content, rng, "long_rle", 0))
    budget = frame_bound(n) - len(head) - len(compact)
    body = _emit(content, _blocks(content, rng, policy, budget))
    assert len(head) + len(body) <= frame_bound(n)
    return head + body


def reframe_record(rec, rng, policy):
    L, mode, attr, resv, flen = struct.unpack_from("<IBBHI", rec, 0)
    assert L == len(rec) and resv == 0
    frame = reframe_frame(rec[12:12 + flen], rng, policy)
    rest = rec[(12 + flen + 3) & ~3:]
    sec = (12 + len(frame) + 3) & ~3
    out = struct.pack("<IBBHI", sec + len(rest), mode, attr, 0, len(frame)) + frame
    out += bytes(sec - len(out)) + rest
    return out


def reframe_stream(s, seed, policy):
    """The stream with every record's mask frame re-framed (seeded)."""
    rng = np.random.default_rng(seed)
    hdr, recs = split_stream(s)
    assert hdr["T"] > 0
    new = [reframe_record(r, rng, policy) for r in recs]
    p = 20 + 8 * hdr["A"]
    table = b"".join(struct.pack("<I", len(r)) for r in new)
    return s[:p] + table + b"".join(new)


def mask_blocks(s):
    """Per record of a stream: its mask frame's block list (kind, size)."""
    _, recs = split_stream(s)
    return [read_zstd_frame(r[12:12 + u32(r, 8)])[1]["blocks"] for r in recs]
