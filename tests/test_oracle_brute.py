"""Oracle pins of the brute-force I/P choice (Sec. III-E: code the scan both
ways and keep the smaller).  Its records are read back with the test-side
stream reader and compared with the records of the forced I-only and
P-only streams: every record is the smaller of the two (equal sizes: the
I-record), the first scan is an I-scan, and the stream still decodes to the
input.  A choice of the larger record, ties going to P, or a comparison
that leaves out the mask fails one of these."""
import numpy as np
import pytest

import oracle
from formatcheck import split_stream
from paper_2209_08196_amd import synth


def _cases():
    rng = np.random.default_rng(11)
    g1 = synth.stream(1, 0)
    yield "c1", g1.scans(0, 6), list(g1.precisions)
    g2 = synth.stream(2, 0)
    yield "c2_crop", [p[:, :24, :512] for p in g2.scans(28, 34)], list(g2.precisions)  # includes standing still
    g5 = synth.stream(5, 0)
    yield "c5_crop", [p[:, :16, :1024] for p in g5.scans(16, 24)], [1]  # a scene cut inside
    # static scenes (P wins) and fresh noise (I wins) in one sequence
    base = synth.random_scans(rng, 1, 12, 200, np.uint16, 0.3, scale=900)
    still = np.repeat(base, 3, axis=0)
    still[1:, 5, :] ^= 1  # small changes: P records are tiny
    noisy = synth.random_scans(rng, 3, 12, 200, np.uint16, 0.3, scale=900)
    yield "mixed", [np.concatenate([still, noisy, still])], [1]


@pytest.mark.parametrize("name,planes,precs", list(_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_brute_keeps_the_smaller_record(name, planes, precs):
    A = len(planes)
    T = planes[0].shape[0]
    s_i, m_i = oracle.encode(planes, precs, mode=oracle.MODE_I_ONLY)
    s_p, m_p = oracle.encode(planes, precs, mode=oracle.MODE_P_ONLY)
    s_b, m_b = oracle.encode(planes, precs, mode=oracle.MODE_BRUTE)
    _, ri = split_stream(s_i)
    _, rp = split_stream(s_p)
    _, rb = split_stream(s_b)
    assert len(ri) == len(rp) == len(rb) == T * A
    chose_p = 0
    for r in range(T * A):
        t = r // A
        want_p = t > 0 and len(rp[r]) < len(ri[r])
        assert rb[r] == (rp[r] if want_p else ri[r]), (name, r)
        assert m_b[t, r % A] == (1 if want_p else 0), (name, r)
        assert rb[r][4] == (1 if want_p else 0)  # the record's own mode byte
        chose_p += want_p
    assert m_b[0].sum() == 0
    # the stream is the smallest of all choices, record by record
    s_a, _ = oracle.encode(planes, precs)
    assert len(s_b) <= min(len(s_i), len(s_p), len(s_a))
    out = oracle.decode(s_b)
    for a, p in enumerate(planes):
        if precs[a] == 1:
            assert np.array_equal(out[a], p)
    if name == "mixed":
        assert 0 < chose_p < T - 1  # both kinds occur


def test_brute_ties_go_to_the_i_scan():
    """Two identical all-zero scans: the P record (mask XOR previous = 0,
    no samples) and the I record (all-ones mask, no samples) code equally
    small frames; the I-record is kept."""
    z = np.zeros((2, 4, 64), np.uint32)
    s_i, _ = oracle.encode([z], [1], mode=oracle.MODE_I_ONLY)
    s_p, _ = oracle.encode([z], [1], mode=oracle.MODE_P_ONLY)
    s_b, m_b = oracle.encode([z], [1], mode=oracle.MODE_BRUTE)
    _, ri = split_stream(s_i)
    _, rp = split_stream(s_p)
    _, rb = split_stream(s_b)
    assert len(ri[1]) == len(rp[1])
    assert rb[1] == ri[1] and m_b[1, 0] == 0
