"""GPU: a batch of streams replayed from one HIP graph per step gives the
same records as the plain batched step and as the oracle on each stream's
whole sequence (Sec. III-D: P-scans predict from the resident previous scan).
Every call goes through the C ABI (libjiffy.so)."""
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
    jiffy.lib()
    return jiffy


SHAPES = [(16, 1024), (32, 2048), (64, 1024), (7, 301), (128, 2048), (1, 5)]


def _oracle_records(data, precs, reset_at=None):
    """Records of one stream's sequence, restarted (I-scan) at reset_at."""
    if reset_at is None:
        return split_stream(oracle.encode(data, precs)[0])[1]
    a = split_stream(oracle.encode([p[:reset_at] for p in data], precs)[0])[1]
    b = split_stream(oracle.encode([p[reset_at:] for p in data], precs)[0])[1]
    return a + b


def test_graph_batch_matches_plain_step_and_oracle(J):
    import torch
    T = 5
    gens = [synth.stream(3, s, size=SHAPES[s]) for s in range(len(SHAPES))]
    data = [g.scans(0, T) for g in gens]
    mk = lambda: [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]  # noqa: E731
    sa, sb = mk(), mk()
    inputs = [[torch.zeros((g.H, g.W), dtype=to_dev(p[0]).dtype, device="cuda") for p in dd]
              for g, dd in zip(gens, data)]
    outs_a = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sa]
    outs_b = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sb]
    batch = J.Batch(sa, inputs, outs_a)
    got_a = [[] for _ in gens]
    got_b = [[] for _ in gens]
    for t in range(T):
        banner("graph batch step", t)
        if t == 3:
            sa[1].reset()
            sb[1].reset()
        for i, d in enumerate(data):  # eager work between replays: fill the inputs
            for a, p in enumerate(d):
                inputs[i][a].copy_(to_dev(p[t]))
        la, ma = batch.run()
        torch.cuda.synchronize()
        lb, mb = J.batch_encode_step(sb, [[to_dev(p[t]) for p in d] for d in data], outs_b)
        assert la == lb, (t, la, lb)
        assert np.array_equal(ma, mb)
        for i in range(len(gens)):
            got_a[i].append(outs_a[i][: la[i]].cpu().numpy().tobytes())
            got_b[i].append(outs_b[i][: lb[i]].cpu().numpy().tobytes())
    for i, g in enumerate(gens):
        recs = _oracle_records(data[i], g.precisions, reset_at=3 if i == 1 else None)
        A = len(g.widths)
        for t in range(T):
            want = b"".join(recs[t * A:(t + 1) * A])
            assert got_a[i][t] == want, ("graph", i, t)
            assert got_b[i][t] == want, ("plain", i, t)
    batch.close()
    for s in sa + sb:
        s.close()


def test_graph_batch_capacity_error_leaves_state(J):
    """An output that does not fit: JIFFY_E_CAPACITY with the bytes needed,
    and no stream advances (the next run repeats the same scan as an I-scan)."""
    import torch
    g = synth.stream(3, 0, size=(16, 1024))
    x = g.scans(0, 2)
    s = J.Stream(g.H, g.W, g.widths, g.precisions)
    inp = [torch.zeros((g.H, g.W), dtype=to_dev(p[0]).dtype, device="cuda") for p in x]
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    b = J.Batch([s], [inp], [small])
    for a, p in enumerate(x):
        inp[a].copy_(to_dev(p[0]))
    with pytest.raises(J.JiffyError) as e:
        b.run()
    assert e.value.code == -2
    b.close()
    big = torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda")
    b = J.Batch([s], [inp], [big])
    lens, modes = b.run()
    want = split_stream(oracle.encode([p[:1] for p in x], g.precisions)[0])[1]
    assert big[: lens[0]].cpu().numpy().tobytes() == b"".join(want)
    assert modes.ravel().tolist() == [0] * len(g.widths)
    b.close()
    s.close()


def test_graph_batch_with_inputs_named_per_run(J):
    """run() naming each step's input tensors (no copies) gives the oracle's
    records; replays interleave with eager work and synchronizations."""
    import torch
    T = 4
    gens = [synth.stream(3, s, size=SHAPES[s]) for s in (0, 3, 5)]
    data = [g.scans(0, T) for g in gens]
    dev = [[to_dev(p) for p in d] for d in data]
    streams = [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]
    outs = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in streams]
    batch = J.Batch(streams, [[p[0] for p in d] for d in dev], outs)
    got = [[] for _ in gens]
    for t in range(T):
        banner("graph batch, named inputs, step", t)
        junk = torch.arange(1 << 20, device="cuda").sum()  # eager work between replays
        lens, _ = batch.run([[p[t] for p in d] for d in dev])
        torch.cuda.synchronize()
        assert int(junk) == (1 << 20) * ((1 << 20) - 1) // 2
        for i in range(len(gens)):
            got[i].append(outs[i][: lens[i]].cpu().numpy().tobytes())
    for i, g in enumerate(gens):
        recs = _oracle_records(data[i], g.precisions)
        A = len(g.widths)
        for t in range(T):
            assert got[i][t] == b"".join(recs[t * A:(t + 1) * A]), (i, t)
    batch.close()
    for s in streams:
        s.close()


def test_open_ended_stream_of_step_records_decodes(J):
    """Records from batched steps, behind a header with no length table
    (T = 0: records until the end), decode on the GPU to the oracle's
    output for the same scans."""
    import torch
    g = synth.stream(3, 1, size=(32, 2048))
    T = 5
    x = g.scans(0, T)
    s = J.Stream(g.H, g.W, g.widths, g.precisions)
    out = torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda")
    recs = []
    for t in range(T):
        lens, _ = J.batch_encode_step([s], [[to_dev(p[t]) for p in x]], [out])
        recs.append(out[: lens[0]].cpu().numpy().tobytes())
    s.close()
    full, _ = oracle.encode(x, g.precisions)
    A = len(g.widths)
    head = bytearray(full[:20 + 8 * A])
    head[16:20] = (0).to_bytes(4, "little")
    open_s = bytes(head) + b"".join(recs)
    banner("decode open-ended stream", len(open_s))
    outs = J.decode(torch.from_numpy(np.frombuffer(open_s, np.uint8).copy()).cuda())
    ref = oracle.decode(full)
    for o, r in zip(outs, ref):
        assert np.array_equal(to_host(o, r.dtype.itemsize), r)
