"""The re-framer used by the GPU re-framing tests, pinned on the CPU: a
re-framed stream holds other mask-frame blocks (checked with the format
reader) and the oracle decodes it to the same samples as the original."""
import numpy as np
import pytest

import oracle
from paper_2209_08196_amd import synth
from formatcheck import split_stream, u32
from reframe import POLICIES, frame_bound, mask_blocks, reframe_stream


def _case(kind):
    if kind == "c2":  # five attributes, the standing interval (P-records)
        g = synth.stream(2, 0)
        return g.scans(28, 31), list(g.precisions)
    g = synth.stream(5, 0)  # 128x4096 at 60% zeros: eight parse windows per mask frame
    return g.scans(0, 2), list(g.precisions)


@pytest.mark.parametrize("kind", ["c2", "c5"])
@pytest.mark.parametrize("policy", POLICIES)
def test_reframed_stream_decodes_the_same(kind, policy):
    planes, precs = _case(kind)
    s, _ = oracle.encode(planes, precs)
    r = reframe_stream(s, seed=7, policy=policy)
    old, new = mask_blocks(s), mask_blocks(r)
    assert len(old) == len(new)
    assert any(a != b for a, b in zip(old, new)), "the block boundaries must change"
    ref = oracle.decode(s)
    got = oracle.decode(r)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    for blocks, rec in zip(new, split_stream(r)[1]):
        assert u32(rec, 8) <= frame_bound(sum(size for _, size in blocks))  # what the decoder accepts
    if policy == "one_raw":
        assert all(all(k == "raw" for k, _ in b) for b in new)
    if policy == "tiny":
        assert any(size == 0 for b in new for k, size in b if k == "raw"), "blocks without content"
        assert any(k == "rle" and size < 4 for b in new for k, size in b) or any(
            k == "raw" and 0 < size <= 4 for b in new for k, size in b)
