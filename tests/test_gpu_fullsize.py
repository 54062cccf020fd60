"""Parity at the measured workloads' full sizes, in the launch configuration
the benchmark times (a prepared Encoder and Decoder over every scan of the
stream at once): the dual-return 128x2048 stream (100 scans, five
attributes) and one whole 200-scan 128x4096 stream of the stress set (60%
zeros, a scene cut every 20 scans).  The GPU stream is compared with the
oracle's byte for byte and its I/P decisions one by one; the decoded planes
with the oracle's decode of the same stream and, as every precision here is
1 (lossless), with the input itself."""
import numpy as np
import pytest

import oracle
from formatcheck import split_stream
from gpu_util import banner, to_dev, to_host
from paper_2209_08196_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()  # raises if the library is missing
    return jiffy


def _full_stream(J, cid, n_scans, name):
    import torch
    g = synth.stream(cid, 0)
    planes = g.scans(0, n_scans)
    precs = list(g.precisions)
    T, H, W = planes[0].shape
    banner("full size encode", name, (T, H, W), [p.dtype.name for p in planes])
    dev = [to_dev(p) for p in planes]
    s, m = J.Encoder(dev, precs)()
    s_gpu = s.cpu().numpy().tobytes()
    m_gpu = m.copy()
    s_ref, m_ref = oracle.encode(planes, precs)
    assert np.array_equal(m_gpu, m_ref), name
    if s_gpu != s_ref:
        _, rg = split_stream(s_gpu)
        _, rr = split_stream(s_ref)
        bad = [i for i, (a, b) in enumerate(zip(rg, rr)) if a != b]
        raise AssertionError(f"{name}: streams differ ({len(s_gpu)} vs {len(s_ref)} bytes); records {bad[:10]}")
    banner("full size decode", name)
    lay = J.make_layout(H, W, [p.dtype.itemsize for p in planes], precs)
    outs = [torch.full_like(d, 0x55) for d in dev]  # stale contents: every sample must be written
    J.Decoder(lay, T, outs)(s)
    ref = oracle.decode(s_ref)
    for a, (o, r, p) in enumerate(zip(outs, ref, planes)):
        h = to_host(o, r.dtype.itemsize)
        assert np.array_equal(h, r), (name, a)
        assert precs[a] == 1 and np.array_equal(h, p), (name, a)


def test_dual_return_128x2048_full_stream(J):
    _full_stream(J, 2, 100, "dual-return 128x2048 x100, 5 attributes")


def test_stress_128x4096_full_stream(J):
    _full_stream(J, 5, 200, "stress 128x4096 x200")
