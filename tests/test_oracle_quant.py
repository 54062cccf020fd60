"""Oracle pins of quantization to a precision P (Sec. III-B) and of the
precision sweep (Sec. IV-G, Fig. 4).

The quantizer is checked by the properties that define it, over the whole
32-bit range and precisions up to 2^32 - 1: the result times P is a nearest
multiple of P to the sample (a tie goes up), zero stays zero, an in-range
sample stays in range.  The sweep checks what the paper reports for range
data: the reconstruction error is at most floor(P/2), and each doubling of
P saves about one bit per stored sample while the noise dominates."""
import numpy as np
import pytest

import oracle
from paper_2209_08196_amd import synth


def test_quantizer_is_the_nearest_multiple_over_the_32_bit_range():
    rng = np.random.default_rng(2209)
    xs = list(rng.integers(1, 1 << 32, 3000, dtype=np.uint64)) + [1, 2, (1 << 32) - 1, (1 << 32) - 2, 1 << 31]
    Ps = list(rng.integers(1, 1 << 32, 60, dtype=np.uint64)) + [1, 2, 3, 7, 1 << 16, (1 << 31) + 1,
                                                                (1 << 32) - 1, (1 << 32) - 2]
    for P in map(int, Ps):
        for x in map(int, xs[:: max(1, len(xs) // 400)]):
            q = oracle.quantize(x, P)
            d = q * P - x
            assert q >= 1
            assert 2 * abs(d) <= P or (q == 1 and x < P - P // 2), (x, P, q)  # nearest (or clamped to 1)
            if 2 * abs(d) == P:
                assert d > 0, (x, P)  # a tie rounds up
            if q > 1:
                assert abs((q - 1) * P - x) >= abs(d)
            assert abs((q + 1) * P - x) > abs(d) or 2 * abs(d) == P
        assert oracle.quantize(0, P) == 0


def test_sweep_error_bound_and_one_bit_per_doubling():
    g = synth.stream(2, 0)
    x = g.scans(0, 3)[0][:, :64, :1024]  # range in mm, three scans
    nz = x != 0
    bits = []
    for P in (1, 2, 4, 8, 16, 32, 64):
        s, _ = oracle.encode([x], [P])
        y = oracle.decode(s)[0].astype(np.int64)
        err = np.abs(y - x.astype(np.int64))
        assert err[nz].max() <= P // 2, P
        assert (y[~nz] == 0).all() and (y[nz] > 0).all()
        bits.append(8 * len(s) / nz.sum())
    saved = np.diff(bits) * -1
    assert (saved > 0).all()
    assert 0.85 <= saved[:4].mean() <= 1.1, saved  # P = 1 .. 16: about one bit per doubling
