"""Parity at the measured workloads' full sizes, in the launch configurations
the benchmark times (a prepared Encoder and Decoder over every scan of the
stream at once): the dual-return 128x2048 stream (100 scans, five
attributes) and one whole 200-scan 128x4096 stream of the stress set (60%
zeros, a scene cut every 20 scans).  The GPU stream is compared with the
oracle's byte for byte and its I/P decisions one by one; the decoded planes
with the oracle's decode of the same stream and, as every precision here is
1 (lossless), with the input itself.  The batched workload's 64 streams go
through the graph-replayed batch and the plain batched step."""
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


def test_batched_64_streams_full_batch(J):
    """All 64 streams of the batched workload (four sizes, range at 1 cm and
    signal), three steps of one scan each, through the graph-replayed batch
    and the plain batched step as the benchmark runs them; each stream's
    records equal the oracle's encoding of its sequence."""
    import torch
    T = 3
    gens = [synth.stream(3, s) for s in range(synth.CONFIGS[3].streams)]
    data = [g.scans(0, T) for g in gens]
    mk = lambda: [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]  # noqa: E731
    sg, sp = mk(), mk()
    dev = [[to_dev(p) for p in d] for d in data]
    outs_g = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sg]
    outs_p = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sp]
    batch = J.Batch(sg, [[p[0] for p in d] for d in dev], outs_g)
    got_g = [[] for _ in gens]
    got_p = [[] for _ in gens]
    for t in range(T):
        banner("batched 64 streams, step", t)
        lg, _ = batch.run([[p[t] for p in d] for d in dev])
        lp, _ = J.batch_encode_step(sp, [[p[t] for p in d] for d in dev], outs_p)
        assert lg == lp, t
        for i in range(len(gens)):
            got_g[i].append(outs_g[i][: lg[i]].cpu().numpy().tobytes())
            got_p[i].append(outs_p[i][: lp[i]].cpu().numpy().tobytes())
    batch.close()
    for s in sg + sp:
        s.close()
    for i, g in enumerate(gens):
        recs = split_stream(oracle.encode(data[i], list(g.precisions))[0])[1]
        A = len(g.widths)
        for t in range(T):
            want = b"".join(recs[t * A:(t + 1) * A])
            assert got_g[i][t] == want, ("graph", i, t)
            assert got_p[i][t] == want, ("plain", i, t)
