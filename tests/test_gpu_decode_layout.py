"""jiffy_decode_layout: decoding with the layout and scan count known to the
caller (nothing read back before the kernels; the header is checked and the
records are indexed on the device) restores the oracle's output exactly.  A
stream that does not match the given layout, or whose length table does not
add up, is reported as corrupt, and then no record is parsed at all: every
case below leaves the records themselves intact, so the kernels only ever
see well-formed records or none."""
import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev, to_host
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


def _dev(b):
    import torch
    return torch.from_numpy(np.frombuffer(bytes(b), np.uint8).copy()).cuda()


def _layout(J, planes, precs):
    T, H, W = planes[0].shape
    return J.make_layout(H, W, [p.dtype.itemsize for p in planes], precs), T


def _cases():
    g = synth.stream(2, 0)
    yield "dual-return 128x2048 x3", g.scans(0, 3), list(g.precisions), 0
    g = synth.stream(1, 2)
    yield "plain 64x1024 P=10 x4 forced P", g.scans(0, 4), list(g.precisions), 2
    rng = np.random.default_rng(61)
    yield "ragged 3x17x129 u16+u8", [synth.random_scans(rng, 3, 17, 129, np.uint16, 0.3),
                                     synth.random_scans(rng, 3, 17, 129, np.uint8, 0.1)], [3, 1], 0
    yield "one pixel", [synth.random_scans(rng, 2, 1, 1, np.uint32, 0.5)], [1], 0


def test_decode_layout_matches_oracle(J):
    for name, planes, precs, mode in _cases():
        banner("decode_layout", name)
        s_ref, _ = oracle.encode(planes, precs, mode=mode)
        ref = oracle.decode(s_ref)
        lay, T = _layout(J, planes, precs)
        outs = J.decode(_dev(s_ref), lay, T)
        for a, (o, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(to_host(o, r.dtype.itemsize), r), (name, a)


def test_decode_layout_of_device_encoded_stream(J):
    """The stream jiffy_encode left on the device, decoded in place."""
    g = synth.stream(2, 3)
    x = g.scans(0, 4)
    banner("encode + decode_layout in place, dual-return x4")
    s, _ = J.encode([to_dev(p) for p in x], g.precisions)
    lay, T = _layout(J, x, list(g.precisions))
    outs = J.decode(s, lay, T)
    for a, (o, p) in enumerate(zip(outs, x)):
        assert np.array_equal(to_host(o, p.dtype.itemsize), p), a  # P = 1: lossless


def _corrupt(J, fn):
    with pytest.raises(J.JiffyError) as e:
        fn()
    assert e.value.code == J.E_CORRUPT, e.value


def test_decode_layout_rejects_mismatched_layouts_and_tables(J):
    g = synth.stream(1, 0)
    x = g.scans(0, 3)
    precs = list(g.precisions)
    s_ref, _ = oracle.encode(x, precs)
    lay, T = _layout(J, x, precs)
    A, H, W = 1, x[0].shape[1], x[0].shape[2]
    p = 20 + 8 * A
    banner("decode_layout mismatches")
    _corrupt(J, lambda: J.decode(_dev(s_ref), lay, T - 1))
    _corrupt(J, lambda: J.decode(_dev(s_ref), lay, T + 1))
    _corrupt(J, lambda: J.decode(_dev(s_ref), J.make_layout(H, W, [4], [precs[0] + 1]), T))
    _corrupt(J, lambda: J.decode(_dev(s_ref), J.make_layout(W, H, [4], precs), T))
    _corrupt(J, lambda: J.decode(_dev(s_ref), J.make_layout(H, W, [2], precs), T))
    # a record length changed by 4: the table no longer adds up to the stream
    b = bytearray(s_ref)
    n0 = int.from_bytes(b[p:p + 4], "little")
    b[p:p + 4] = (n0 + 4).to_bytes(4, "little")
    _corrupt(J, lambda: J.decode(_dev(b), lay, T))
    _corrupt(J, lambda: J.decode(_dev(b)))  # the host-read header path indexes on the device too
    # lengths that still add up but are not multiples of 4
    b = bytearray(s_ref)
    n1 = int.from_bytes(b[p + 4:p + 8], "little")
    b[p:p + 4] = (n0 + 1).to_bytes(4, "little")
    b[p + 4:p + 8] = (n1 - 1).to_bytes(4, "little")
    _corrupt(J, lambda: J.decode(_dev(b), lay, T))
    _corrupt(J, lambda: J.decode(_dev(b)))
    # a header without a length table is not accepted here
    b = bytearray(s_ref[:p]) + bytearray(s_ref[p + 4 * T * A:])
    b[16:20] = (0).to_bytes(4, "little")
    _corrupt(J, lambda: J.decode(_dev(b), lay, T))
    # the open-ended stream itself decodes through jiffy_decode
    ref = oracle.decode(s_ref)[0]
    assert np.array_equal(to_host(J.decode(_dev(b))[0], 4), ref)
    # and the valid stream still decodes after all of the above
    assert np.array_equal(to_host(J.decode(_dev(s_ref), lay, T)[0], 4), ref)


def test_repeated_calls_on_the_same_buffers_see_new_contents(J):
    """A call with the same arguments as the previous one reuses its plan;
    the inputs' contents are still read afresh, and a workspace that grew in
    between (a larger decode) is not reused stale."""
    import torch
    g = synth.stream(1, 4)
    x, y = g.scans(0, 4), g.scans(4, 8)
    precs = list(g.precisions)
    lay, T = _layout(J, x, precs)
    dev = [to_dev(p) for p in x]
    out = torch.empty(J.encode_bound(lay, T), dtype=torch.uint8, device="cuda")
    outs = [torch.empty_like(d) for d in dev]
    big = synth.stream(2, 5).scans(0, 6)
    s_big, _ = oracle.encode(big, synth.stream(2, 5).precisions)
    for rnd, data in enumerate((x, y, x, y)):
        banner("repeat round", rnd)
        for d, p in zip(dev, data):
            d.copy_(to_dev(p))
        s_ref, m_ref = oracle.encode(data, precs)
        s, m = J.encode(dev, precs, out=out)
        assert s.cpu().numpy().tobytes() == s_ref, rnd
        assert np.array_equal(m, m_ref), rnd
        ref = oracle.decode(s_ref)[0]
        for _ in range(2):  # the second decode reuses the first one's plan
            outs[0].zero_()
            J.decode(s, lay, T, outs=outs)
            assert np.array_equal(to_host(outs[0], 4), ref), rnd
        if rnd == 1:  # a larger decode in between grows the workspace
            J.decode(_dev(s_big))


def test_prepared_encoder_and_decoder(J):
    """Encoder / Decoder (arguments prepared once) give the oracle's stream
    and samples, and see new input contents on every call."""
    import torch
    g = synth.stream(2, 7)
    x, y = g.scans(0, 3), g.scans(3, 6)
    precs = list(g.precisions)
    lay, T = _layout(J, x, precs)
    dev = [to_dev(p) for p in x]
    enc = J.Encoder(dev, precs)
    outs = [torch.empty_like(d) for d in dev]
    dcd = J.Decoder(lay, T, outs)
    for rnd, data in enumerate((x, y, x)):
        banner("prepared round", rnd)
        for d, p in zip(dev, data):
            d.copy_(to_dev(p))
        s_ref, m_ref = oracle.encode(data, precs)
        s, m = enc()
        assert s.cpu().numpy().tobytes() == s_ref, rnd
        assert np.array_equal(m, m_ref), rnd
        for o in outs:
            o.zero_()
        dcd(s)
        for a, (o, p) in enumerate(zip(outs, data)):
            assert np.array_equal(to_host(o, p.dtype.itemsize), p), (rnd, a)  # P = 1: lossless


def test_alternating_plans_and_reuse_after_an_error(J):
    """Two prepared encoders with different arguments in turn, decodes in
    between: each call's plan either is still in the workspace or is uploaded
    again, and every stream equals the oracle's.  A plan reused right after
    a call that ran out of output space starts with a clear error word."""
    import torch
    gA, gB = synth.stream(1, 5), synth.stream(2, 6)
    xA, xB = gA.scans(0, 3), gB.scans(0, 2)
    pA, pB = list(gA.precisions), list(gB.precisions)
    encA = J.Encoder([to_dev(p) for p in xA], pA)
    encB = J.Encoder([to_dev(p) for p in xB], pB)
    refA, refB = oracle.encode(xA, pA)[0], oracle.encode(xB, pB)[0]
    for rnd, (enc, ref) in enumerate([(encA, refA), (encA, refA), (encB, refB), (encA, refA), (encB, refB),
                                      (encB, refB)]):
        banner("alternating plans, call", rnd)
        s, _ = enc()
        assert s.cpu().numpy().tobytes() == ref, rnd
        if rnd % 2:
            J.decode(s)  # the decoder's workspace is its own
    # an output buffer too small for incompressible samples, then compressible ones in the same planes
    rng = np.random.default_rng(71)
    hard = rng.integers(1, 2**32, size=(2, 16, 256), dtype=np.uint64).astype(np.uint32)
    easy = np.full((2, 16, 256), 1234, np.uint32)
    dev = to_dev(hard)
    ref_easy = oracle.encode([easy], [1])[0]
    out = torch.empty(len(ref_easy) + 64, dtype=torch.uint8, device="cuda")
    enc = J.Encoder([dev], [1], out=out)
    banner("capacity error, then the same plan with compressible samples")
    with pytest.raises(J.JiffyError) as e:
        enc()
    assert e.value.code == J.E_CAPACITY
    dev.copy_(to_dev(easy))
    s, _ = enc()
    assert s.cpu().numpy().tobytes() == ref_easy
