"""Malformed records decoded on the GPU are reported as corrupt.  Each case
changes one field that the decoder checks before it relies on it (the
record's mode, the mask frame's magic, a block type, the sample count, a
frame's widths, an exception position), so the kernels never act on the bad
value; the oracle rejects the same streams."""
import numpy as np
import pytest

import oracle
from formatcheck import split_stream, u32
from gpu_util import banner
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


def _record0(s):
    """Offsets of the first record's fields inside the stream."""
    hdr, recs = split_stream(s)
    r0 = len(s) - sum(len(r) for r in recs)  # the records follow the header and its length table
    flen = u32(s, r0 + 8)
    sec = r0 + ((12 + flen + 3) & ~3)
    N = u32(s, sec)
    nb = (N + 127) // 128
    widths = s[sec + 4:sec + 4 + nb]
    counts = s[sec + 4 + nb:sec + 4 + 2 * nb]
    pay0 = sec + ((4 + 3 * nb + 3) & ~3)
    pos0 = pay0 + 16 * sum(widths)
    return dict(r0=r0, frame=r0 + 12, sec=sec, N=N, nb=nb, widths=widths, counts=counts, pos0=pos0)


def _cases(s):
    f = _record0(s)
    out = []
    b = bytearray(s)
    b[f["r0"] + 4] = 1  # the first scan marked as a P-scan: nothing to predict from
    out.append(("P-scan first", b))
    b = bytearray(s)
    b[f["frame"]] ^= 0xFF  # mask frame magic
    out.append(("frame magic", b))
    b = bytearray(s)
    fhd = b[f["frame"] + 4]
    fcs = [1, 2, 4, 8][fhd >> 6]
    h0 = f["frame"] + 5 + fcs  # the first block header
    b[h0] = (b[h0] & ~0x06) | (2 << 1)  # block type 2 (compressed): not a Raw/RLE frame
    out.append(("block type", b))
    b = bytearray(s)
    b[f["sec"]:f["sec"] + 4] = (f["N"] + 1).to_bytes(4, "little")  # one sample more than the mask holds
    out.append(("sample count", b))
    b = bytearray(s)
    B0 = f["sec"] + 4 + 2 * f["nb"]
    b[B0] = 33  # a frame wider than the 32-bit samples
    out.append(("frame width", b))
    j = next(k for k in range(f["nb"]) if f["counts"][k])
    p = f["pos0"] + sum(f["counts"][:j])
    b = bytearray(s)
    b[p] = 0xFF  # an exception position past the frame's values
    out.append(("exception position", b))
    return out


def test_malformed_records_are_corrupt(J):
    import torch
    s, (T, H, W) = _stream()
    lay = J.make_layout(H, W, [4], [10])
    for name, b in _cases(s):
        with pytest.raises(oracle.OracleError):
            oracle.decode(bytes(b))
        dev = torch.from_numpy(np.frombuffer(bytes(b), np.uint8).copy()).cuda()
        for known in (False, True):
            banner("corrupt record", name, "layout given" if known else "header read")
            with pytest.raises(J.JiffyError) as e:
                J.decode(dev, lay, T) if known else J.decode(dev)
            assert e.value.code == J.E_CORRUPT, (name, e.value)
    # the intact stream still decodes to the oracle's samples afterwards
    ref = oracle.decode(s)[0]
    out = J.decode(torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda(), lay, T)[0]
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)
