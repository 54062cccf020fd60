"""GPU: jiffy_encode_noalloc (the encoder over the library's fixed device
scratch, for callers that cannot allocate) writes exactly the stream and the
I/P decisions jiffy_encode writes, through the C ABI, on two calls in a row
with the second on a smaller input (the scratch keeps the first call's
contents), and both equal the oracle's.  A capacity shortfall reports the
same length as jiffy_encode; a call too large for the scratch is refused
before anything runs."""
import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev
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


def _both(J, planes, precs, mode=0):
    import torch
    dev = [to_dev(p) for p in planes]
    T, H, W = planes[0].shape
    lay = J.make_layout(H, W, [p.dtype.itemsize for p in planes], precs)
    bound = J.encode_bound(lay, T)
    out_a = torch.empty(bound, dtype=torch.uint8, device="cuda")
    out_b = torch.full((bound,), 0xA5, dtype=torch.uint8, device="cuda")
    s_a, m_a = J.encode(dev, precs, mode=mode, out=out_a)
    s_b, m_b = J.encode(dev, precs, mode=mode, out=out_b, noalloc=True)
    got = s_b.cpu().numpy().tobytes()
    assert got == s_a.cpu().numpy().tobytes()
    assert np.array_equal(m_a, m_b)
    ref, m_ref = oracle.encode(planes, precs, mode=mode)
    assert got == ref and np.array_equal(m_b, m_ref)
    return dev, len(got)


def test_noalloc_equals_encode_on_two_calls(J):
    g = synth.stream(1, 0)
    x = g.scans(0, 10)
    banner("noalloc call 1: 64x1024 x10 range, P=10")
    _both(J, x, list(g.precisions))
    g2 = synth.stream(2, 0)
    y = [p[:, :16, :300] for p in g2.scans(0, 3)]  # smaller, five attributes, a ragged row width
    banner("noalloc call 2: 16x300 x3, 5 attributes")
    _both(J, y, list(g2.precisions))
    banner("noalloc call 3: the first input again, P-only")
    _both(J, x, list(g.precisions), mode=2)


def test_noalloc_capacity_and_scratch_limits(J):
    import torch
    g = synth.stream(1, 0)
    x = g.scans(0, 4)
    dev = [to_dev(p) for p in x]
    banner("noalloc capacity shortfall")
    full, _ = J.encode(dev, g.precisions)
    small = torch.empty(100, dtype=torch.uint8, device="cuda")
    with pytest.raises(J.JiffyError) as e:
        J.encode(dev, g.precisions, out=small, noalloc=True)
    assert e.value.code == J.E_CAPACITY
    banner("noalloc scratch limit (refused on the host)")
    big = torch.zeros((32, 128, 4096), dtype=torch.int32, device="cuda")  # about 168 MB of workspace
    out = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(J.JiffyError) as e:
        J.encode([big], [1], out=out, noalloc=True)
    assert e.value.code == J.E_SCRATCH
    assert full.numel() > 100
