"""GPU: streams whose mask frames carry other valid block boundaries than the
encoders write (RLE blocks from one byte, raw blocks of 1 to 4 bytes or of a
whole window and more, blocks without content, runs cut in two) decode to the
oracle's samples, one stream per call and several per call."""
import numpy as np
import pytest

import oracle
from gpu_util import banner, to_host
from paper_2209_08196_amd import synth
from reframe import POLICIES, reframe_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()
    return jiffy


def _case(kind, sid=0):
    if kind == "c2":  # five attributes, the standing interval (P-records)
        g = synth.stream(2, sid)
        return g.scans(28, 31), list(g.precisions)
    g = synth.stream(5, sid)  # 128x4096 at 60% zeros: eight parse windows per mask frame
    return g.scans(0, 2), list(g.precisions)


def _dev(b):
    import torch
    return torch.from_numpy(np.frombuffer(b, np.uint8).copy()).cuda()


@pytest.mark.parametrize("kind", ["c2", "c5"])
@pytest.mark.parametrize("policy", POLICIES)
def test_reframed_decode(J, kind, policy):
    planes, precs = _case(kind)
    s, _ = oracle.encode(planes, precs)
    r = reframe_stream(s, seed=11, policy=policy)
    ref = oracle.decode(s)
    banner("decode reframed", kind, policy, len(s), len(r))
    got = J.decode(_dev(r))
    for a, want in enumerate(ref):
        assert np.array_equal(to_host(got[a], want.dtype.itemsize), want), (kind, policy, a)


def test_reframed_decode_many(J):
    import torch
    streams = [_case("c5", sid) for sid in range(3)]
    precs = streams[0][1]
    raw = [oracle.encode(p, precs)[0] for p, _ in streams]
    ins = [_dev(reframe_stream(s, seed=20 + k, policy=POLICIES[k % len(POLICIES)])) for k, s in enumerate(raw)]
    T, H, W = streams[0][0][0].shape
    lay = J.make_layout(H, W, [4], precs)
    outs = [[torch.empty((T, H, W), dtype=torch.int32, device="cuda")] for _ in ins]
    banner("decode_many reframed", len(ins))
    dec = J.DecoderMany(lay, T, ins, outs)
    got = dec([int(x.numel()) for x in ins])
    for k, s in enumerate(raw):
        want = oracle.decode(s)[0]
        assert np.array_equal(to_host(got[k][0], 4), want), k
