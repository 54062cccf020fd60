"""GPU: several scan sequences encoded and decoded in one launch sequence
(jiffy_encode_many / jiffy_decode_many).  Each stream's output equals the
oracle's encoding of that stream alone, with its modes, and the decode
restores the oracle's samples, including P-records (mask chains and the
temporal pass over many columns), more columns than one stream may have
attributes, a short output (capacity error), a corrupt stream among good
ones, and calls interleaved with single-stream calls (plan reuse)."""
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


def _streams(kind, n):
    rng = np.random.default_rng(n)
    if kind == "c1":
        return [synth.stream(1, s).scans(0, 4) for s in range(n)], [10]
    if kind == "c2_crop":  # five attributes, the standing interval (P-records)
        out = []
        for s in range(n):
            g = synth.stream(2, 0, base_seed=s)
            out.append([p[:, :24, :512] for p in g.scans(28, 33)])
        return out, list(synth.stream(2, 0).precisions)
    if kind == "ragged":  # two attributes of odd widths, random modes
        return [[synth.random_scans(rng, 6, 5, 37, np.uint16, 0.3, scale=400),
                 synth.random_scans(rng, 6, 5, 37, np.uint8, 0.2, scale=60)] for _ in range(n)], [3, 1]
    raise ValueError(kind)


def _check_many(J, streams, precs, mode=0, tag=""):
    import torch
    dev = [[to_dev(p) for p in planes] for planes in streams]
    banner("encode_many", tag, len(streams), [p.shape for p in streams[0]], "mode", mode)
    enc = J.EncoderMany(dev, precs, mode=mode)
    outs, modes = enc()
    for s, planes in enumerate(streams):
        ref, mref = oracle.encode(planes, precs, mode=mode)
        assert outs[s].cpu().numpy().tobytes() == ref, (tag, s)
        assert np.array_equal(modes[s], mref), (tag, s)
    banner("decode_many", tag)
    T, H, W = streams[0][0].shape
    lay = J.make_layout(H, W, [p.dtype.itemsize for p in streams[0]], precs)
    dec_out = [[torch.empty_like(d) for d in planes] for planes in dev]
    dec = J.DecoderMany(lay, T, enc.outs, dec_out)
    got = dec(enc.lengths)
    for s, planes in enumerate(streams):
        ref = oracle.decode(outs[s].cpu().numpy().tobytes())
        for a, r in enumerate(ref):
            assert np.array_equal(to_host(got[s][a], r.dtype.itemsize), r), (tag, s, a)
    return enc, dec, dev, dec_out


@pytest.mark.parametrize("kind,n,mode", [("c1", 3, 0), ("c2_crop", 2, 0), ("c2_crop", 2, 2), ("ragged", 6, 0),
                                         ("ragged", 1, 1)])
def test_many_equals_oracle(J, kind, n, mode):
    streams, precs = _streams(kind, n)
    _check_many(J, streams, precs, mode, f"{kind} x{n}")


def test_many_repeated_and_interleaved(J):
    import torch
    streams, precs = _streams("c2_crop", 3)
    enc, dec, dev, dec_out = _check_many(J, streams, precs, 0, "first")
    # a single-stream encode and decode in between, then the prepared calls again
    s1, _ = J.encode(dev[1], precs)
    assert s1.cpu().numpy().tobytes() == oracle.encode(streams[1], precs)[0]
    single = J.decode(s1)
    for a, p in enumerate(streams[1]):
        assert np.array_equal(to_host(single[a], p.dtype.itemsize), oracle.decode(oracle.encode(streams[1], precs)[0])[a])
    for rep in range(2):
        banner("encode_many again", rep)
        for d in dec_out:
            for t in d:
                t.zero_()
        outs, _ = enc()
        for s, planes in enumerate(streams):
            assert outs[s].cpu().numpy().tobytes() == oracle.encode(planes, precs)[0], (rep, s)
        got = dec(enc.lengths)
        for s, planes in enumerate(streams):
            ref = oracle.decode(outs[s].cpu().numpy().tobytes())
            for a, r in enumerate(ref):
                assert np.array_equal(to_host(got[s][a], r.dtype.itemsize), r), (rep, s, a)
    torch.cuda.synchronize()


def test_many_capacity_and_corrupt(J):
    import torch
    streams, precs = _streams("c1", 3)
    dev = [[to_dev(p) for p in planes] for planes in streams]
    T, H, W = streams[0][0].shape
    lay = J.make_layout(H, W, [4], precs)
    bound = J.encode_bound(lay, T)
    outs = [torch.empty(bound, dtype=torch.uint8, device="cuda") for _ in range(3)]
    outs[1] = torch.empty(64, dtype=torch.uint8, device="cuda")  # too small
    banner("encode_many capacity")
    enc = J.EncoderMany(dev, precs, outs=outs)
    with pytest.raises(J.JiffyError) as e:
        enc()
    assert e.value.code == J.E_CAPACITY
    assert enc.lengths[1] == len(oracle.encode(streams[1], precs)[0])  # the bytes needed
    # a corrupt stream among good ones
    good = [oracle.encode(p, precs)[0] for p in streams]
    bad = bytearray(good[2])
    bad[len(bad) - 40] ^= 0xFF
    ins = [torch.from_numpy(np.frombuffer(b, np.uint8).copy()).cuda() for b in (good[0], good[1], bytes(bad))]
    dec_out = [[torch.empty_like(d) for d in planes] for planes in dev]
    dec = J.DecoderMany(lay, T, ins, dec_out)
    banner("decode_many corrupt")
    try:
        dec()
        flipped_ok = True
    except J.JiffyError as err:
        assert err.code == J.E_CORRUPT
        flipped_ok = False
    try:
        oracle.decode(bytes(bad))
        oracle_ok = True
    except oracle.OracleError:
        oracle_ok = False
    assert flipped_ok == oracle_ok
    # the good streams alone decode; a wrong length (the table no longer adds up) is corrupt
    dec2 = J.DecoderMany(lay, T, ins[:2], dec_out[:2])
    banner("decode_many bad length")
    with pytest.raises(J.JiffyError) as e:
        dec2([len(good[0]), len(good[1]) - 4])
    assert e.value.code == J.E_CORRUPT
    banner("decode_many good pair")
    got = dec2([len(good[0]), len(good[1])])
    for s in range(2):
        assert np.array_equal(to_host(got[s][0], 4), oracle.decode(good[s])[0])
