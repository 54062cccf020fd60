"""Malformed streams decoded on the GPU are reported as corrupt, and the
oracle rejects the same streams.  Each case changes one field that the
decoder reads from the stream, and each field is checked before the kernels
rely on it:

  stream    a length-table entry (shifted between two records, not a
            multiple of 4), the stream cut at every record boundary, bytes
            appended after the last record;
  record    its own length field, the mode (a P-scan first), the attribute
            byte, the mask-frame length (too long, one byte short);
  mask      the frame magic, the content size, the type and size of the
            first and second block headers, the last-block flag (cleared
            on the last block, set on the first), mask bits past the scan;
  section   the sample count (one more than the mask holds, more than the
            scan), a frame's widths (B above the sample width, b above B, an
            exception count above 128, exceptions with b = B), exception
            positions (past the frame's values, not increasing).

Every case runs through both decode entry points (the header read on the
host, and the layout given by the caller with the header checked on the
device); afterwards the intact stream still decodes to the oracle's
samples."""
import numpy as np
import pytest

import oracle
from formatcheck import split_stream, u32
from gpu_util import banner, to_host
from paper_2209_08196_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()
    return jiffy


def _stream():
    g = synth.stream(1, 0)
    x = g.scans(0, 3)[0][:, :16, :512]
    s, _ = oracle.encode([x], [10])
    return bytes(s), x.shape


def _ragged_stream():
    """3 x 7 pixels: the mask's last byte has bits past the scan."""
    rng = np.random.default_rng(5)
    x = synth.random_scans(rng, 2, 3, 7, np.uint16, 0.3, scale=300)
    s, _ = oracle.encode([x], [1])
    return bytes(s), x.shape


def _layout(s):
    hdr, recs = split_stream(s)
    A = hdr["A"]
    tab = 20 + 8 * A
    r0 = len(s) - sum(len(r) for r in recs)
    offs = [r0]
    for r in recs[:-1]:
        offs.append(offs[-1] + len(r))
    return tab, offs, [len(r) for r in recs]


def _record(s, ro):
    """Offsets of one record's fields inside the stream."""
    flen = u32(s, ro + 8)
    frame = ro + 12
    fhd = s[frame + 4]
    fcs_len = [1, 2, 4, 8][fhd >> 6]
    blk0 = frame + 5 + fcs_len
    sec = ro + ((12 + flen + 3) & ~3)
    N = u32(s, sec)
    nb = (N + 127) // 128
    widths = s[sec + 4:sec + 4 + nb]
    counts = s[sec + 4 + nb:sec + 4 + 2 * nb]
    pay0 = sec + ((4 + 3 * nb + 3) & ~3)
    pos0 = pay0 + 16 * sum(widths)
    return dict(flen=flen, frame=frame, fcs=frame + 5, fcs_len=fcs_len, blk0=blk0, sec=sec, N=N, nb=nb,
                widths=widths, counts=counts, pos0=pos0)


def _blocks(s, f):
    """(offset, last, type, size) of every block header of a record's mask frame."""
    out, p, end = [], f["blk0"], f["frame"] + f["flen"]
    while p < end:
        h = s[p] | (s[p + 1] << 8) | (s[p + 2] << 16)
        last, typ, size = h & 1, (h >> 1) & 3, h >> 3
        out.append((p, last, typ, size))
        p += 3 + (1 if typ == 1 else size)
        if last:
            break
    return out


def _put_header(b, p, last, typ, size):
    h = last | (typ << 1) | (size << 3)
    b[p:p + 3] = bytes([h & 0xFF, (h >> 8) & 0xFF, (h >> 16) & 0xFF])


def _put32(b, p, v):
    b[p:p + 4] = (v & 0xFFFFFFFF).to_bytes(4, "little")


def _cases(s):
    tab, offs, lens = _layout(s)
    out = []

    def case(name, fn):
        b = bytearray(s)
        fn(b)
        out.append((name, bytes(b)))

    # stream
    case("table entries shifted", lambda b: (_put32(b, tab, lens[0] + 4), _put32(b, tab + 4, lens[1] - 4)))
    case("table entry not a multiple of 4", lambda b: (_put32(b, tab, lens[0] + 2), _put32(b, tab + 4, lens[1] - 2)))
    for k in range(len(offs)):  # cut at every record boundary
        out.append((f"cut before record {k}", s[:offs[k]]))
    out.append(("bytes appended", s + b"\0\0\0\0"))
    # record 1 (a record after the first)
    r1 = offs[1]
    f1 = _record(s, r1)
    case("record length field", lambda b: _put32(b, r1, lens[1] + 4))
    case("P-scan first", lambda b: b.__setitem__(offs[0] + 4, 1))
    case("attribute byte", lambda b: b.__setitem__(r1 + 5, 1))
    case("mask frame too long", lambda b: _put32(b, r1 + 8, lens[1] - 11))
    case("mask frame one byte short", lambda b: _put32(b, r1 + 8, f1["flen"] - 1))
    # mask frame
    case("frame magic", lambda b: b.__setitem__(f1["frame"], b[f1["frame"]] ^ 0xFF))
    case("content size", lambda b: b.__setitem__(f1["fcs"], (b[f1["fcs"]] + 1) & 0xFF))
    blocks = _blocks(s, f1)
    assert len(blocks) >= 3, "the case needs a mask frame of several blocks"
    for i in (0, 1):
        p, last, typ, size = blocks[i]
        case(f"block {i} type 2", lambda b, p=p, last=last, size=size: _put_header(b, p, last, 2, size))
        case(f"block {i} type 3", lambda b, p=p, last=last, size=size: _put_header(b, p, last, 3, size))
        case(f"block {i} size + 1", lambda b, p=p, last=last, typ=typ, size=size: _put_header(b, p, last, typ, size + 1))
    p, _, typ, size = blocks[0]
    case("first block flagged last", lambda b: _put_header(b, p, 1, typ, size))
    p, _, typ, size = blocks[-1]
    case("last block not flagged", lambda b: _put_header(b, p, 0, typ, size))
    # section
    case("sample count + 1", lambda b: _put32(b, f1["sec"], f1["N"] + 1))
    case("sample count past the scan", lambda b: _put32(b, f1["sec"], 16 * 512 + 1))
    nb = f1["nb"]
    b0 = f1["sec"] + 4
    case("frame width B = 33", lambda b: b.__setitem__(b0 + 2 * nb, 33))
    j = next(k for k in range(nb) if f1["widths"][k] > 0)
    case("frame width b above B", lambda b: b.__setitem__(b0 + j, b[b0 + 2 * nb + j] + 1))
    case("exception count 129", lambda b: b.__setitem__(b0 + nb, 129))
    je = next(k for k in range(nb) if f1["counts"][k])
    case("exceptions with b = B", lambda b: b.__setitem__(b0 + je, b[b0 + 2 * nb + je]))
    pe = f1["pos0"] + sum(f1["counts"][:je])
    case("exception position past the values", lambda b: b.__setitem__(pe, 0xFF))
    jj = next((k for k in range(nb) if f1["counts"][k] >= 2), None)
    if jj is not None:
        pj = f1["pos0"] + sum(f1["counts"][:jj])
        case("exception positions not increasing", lambda b: b.__setitem__(pj + 1, b[pj]))
    return out


def _ragged_cases(s):
    """A mask bit past the scan: set the top bit of the last content byte."""
    tab, offs, lens = _layout(s)
    f = _record(s, offs[0])
    blocks = _blocks(s, f)
    p, last, typ, size = blocks[-1]
    b = bytearray(s)
    if typ == 0:
        b[p + 3 + size - 1] |= 0x80
    else:
        b[p + 3] |= 0x80
    return [("mask bit past the scan", bytes(b))]


def _check(J, s, shape, cases, width):
    import torch
    T, H, W = shape
    lay = J.make_layout(H, W, [width], [10 if width == 4 else 1])
    for name, b in cases:
        with pytest.raises(oracle.OracleError):
            oracle.decode(b)
        dev = torch.from_numpy(np.frombuffer(b, np.uint8).copy()).cuda()
        for known in (False, True):
            banner("corrupt stream", name, "layout given" if known else "header read")
            with pytest.raises(J.JiffyError) as e:
                J.decode(dev, lay, T) if known else J.decode(dev)
            assert e.value.code == J.E_CORRUPT, (name, e.value)
    ref = oracle.decode(s)[0]
    out = J.decode(torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda(), lay, T)[0]
    assert np.array_equal(to_host(out, width), ref)


def test_malformed_streams_are_corrupt(J):
    s, shape = _stream()
    _check(J, s, shape, _cases(s), 4)


def test_mask_bits_past_the_scan_are_corrupt(J):
    s, shape = _ragged_stream()
    _check(J, s, shape, _ragged_cases(s), 2)
