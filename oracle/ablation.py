"""Ablated codecs and the run-length mask codec -- TEST INFRASTRUCTURE ONLY.

Only the test-suite and the benchmark's reference checks use this module.
Byte sizes of one scan of one attribute coded with stages of the codec left
out, the analogue of the ablation table (Sec. IV-H, Table IV):

  level 1  PFOR                         every pixel's quantized sample
  level 2  Delta -> PFOR                differences to the preceding pixel, modulo 2^w
  level 3  Delta -> ZigZag -> PFOR      the same, ZigZag-coded (Eq. 1)
  level 4  Mask -> Delta -> ZigZag -> PFOR   the I-record of the codec
  level 5  Mask -> Predict -> ...            the codec itself (trial I/P choice)

Levels 1-3 code every pixel (zeros included, no mask) into a record of the
codec's own layout: the 12-byte record head, no mask frame, the residual
section of the coded vector, padding to 4 bytes.  Levels 4 and 5 are the
records of the full encoder (``oracle.encode`` in I-only and automatic
mode) and are not recomputed here.

The run-length mask codec is the alternative to the mask frame: the zero
bitmask of Sec. III-C (XOR the previous scan's mask for a P-record, Sec.
III-D) read as alternating runs that start with a run of in-range pixels
(bit 0; that first run may be empty); the first run's length and every later
run's length minus one (those runs are never empty) are coded as one
residual section.  Its size is the section's bytes padded to 4.

Quantization (Sec. III-B) is applied first at every level.  The PFOR
section is the oracle's own coder (``oracle.pfor_encode``).
"""
import numpy as np

from . import pfor_encode

RECORD_HEAD = 12
N_LEVELS = 3          # levels computed here
N_SIZES = 5           # per record: levels 1-3, run-length mask of the I-mask and of the P-mask


def pad4(n):
    return (n + 3) & ~3


def quantize_plane(x, P):
    """Sec. III-B: nearest multiple of P, halves rounded up, a nonzero sample
    never becomes 0.  Returns uint64."""
    x = np.asarray(x).astype(np.uint64)
    if P == 1:
        return x
    q = (x + np.uint64(P // 2)) // np.uint64(P)
    return np.where(x == 0, np.uint64(0), np.maximum(q, np.uint64(1)))


def delta(v, bits):
    """Difference to the preceding value of the flattened vector (0 before
    the first), modulo 2^bits."""
    v = np.asarray(v, dtype=np.uint64)
    prev = np.concatenate([np.zeros(1, np.uint64), v[:-1]])
    return (v - prev) & np.uint64((1 << bits) - 1)


def zigzag(d, bits):
    """Eq. 1 read as the standard ZigZag map of a bits-wide two's-complement
    value: 2s for s >= 0, -2s - 1 for s < 0."""
    d = np.asarray(d, dtype=np.uint64)
    s = d.astype(np.int64)
    s = np.where(d >= np.uint64(1 << (bits - 1)), s - (1 << bits), s)
    return np.where(s >= 0, 2 * s, -2 * s - 1).astype(np.uint64)


def section_bytes(values):
    """Unpadded bytes of the residual section coding `values`."""
    z = np.asarray(values, dtype=np.uint64)
    assert z.size == 0 or int(z.max()) < (1 << 32)
    return len(pfor_encode(z.astype(np.uint32)))


def record_bytes(values):
    """A record with no mask frame: head, section, padding to 4."""
    return RECORD_HEAD + pad4(section_bytes(values))


def levels(scan, P, bits):
    """[level 1, level 2, level 3] record bytes of one scan ([H, W])."""
    v = quantize_plane(np.asarray(scan).ravel(), P)
    d = delta(v, bits)
    return [record_bytes(v), record_bytes(d), record_bytes(zigzag(d, bits))]


def mask_bits(scan):
    """Sec. III-C: one bit per pixel, 1 where the sample is zero (quantizing
    never makes a nonzero sample zero, so the raw samples decide)."""
    return (np.asarray(scan).ravel() == 0)


def run_values(bits):
    """The run-length codec's values of a flat bit vector."""
    b = np.asarray(bits, dtype=np.int8).ravel()
    n = b.size
    change = np.flatnonzero(np.diff(np.concatenate([np.zeros(1, np.int8), b])))  # where bit k != bit k-1
    ends = np.concatenate([np.zeros(1, np.int64), change, np.array([n], np.int64)])
    runs = np.diff(ends)
    runs[1:] -= 1
    return runs.astype(np.uint64)


def runs_to_bits(values, n):
    """Inverse of run_values."""
    out = np.zeros(n, bool)
    pos, bit = 0, False
    for i, u in enumerate(np.asarray(values, dtype=np.int64)):
        r = int(u) + (1 if i else 0)
        out[pos:pos + r] = bit
        pos += r
        bit = not bit
    assert pos == n
    return out


def rl_mask_bytes(bits):
    return pad4(section_bytes(run_values(bits)))


def ablate(planes, precisions=None):
    """planes: list of [T, H, W] arrays (one per attribute).  Returns uint64
    [T, A, 5]: levels 1-3 record bytes, run-length bytes of the scan's mask
    and of its mask XOR the previous scan's (the first scan: its own mask)."""
    A = len(planes)
    T = planes[0].shape[0]
    precisions = precisions or [1] * A
    out = np.zeros((T, A, N_SIZES), np.uint64)
    for a, p in enumerate(planes):
        bits = 8 * p.dtype.itemsize
        prev = None
        for t in range(T):
            out[t, a, :3] = levels(p[t], precisions[a], bits)
            m = mask_bits(p[t])
            out[t, a, 3] = rl_mask_bytes(m)
            out[t, a, 4] = rl_mask_bytes(m ^ prev) if prev is not None else out[t, a, 3]
            prev = m
    return out
