"""GPU: the fused persistent encoder (one launch whose workgroups take work
items from a queue in dependency order) writes exactly the streams and
records of the kernel chain and of the oracle: whole sequences
(jiffy_encode), batch steps (direct and graph-replayed, the 64-stream
batched set), asynchronous step contexts, at one workgroup per compute unit
and at full occupancy; and every candidate of the autotuner is
byte-identical."""
import numpy as np
import pytest

import oracle
from formatcheck import split_stream
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
    yield jiffy
    jiffy.set_tuning(0, 0)


def _wgs(J):
    _, m = J.get_tuning()
    assert m >= 1
    return sorted({1, m})


@pytest.mark.parametrize("case", ["c1", "c2_crop", "random_full", "ragged_tiny", "p_only"])
def test_fused_sequences_equal_oracle(J, case):
    rng = np.random.default_rng(7)
    mode = 0
    if case == "c1":
        g = synth.stream(1, 0)
        x, precs = g.scans(0, 6), list(g.precisions)
    elif case == "c2_crop":
        g = synth.stream(2, 0)
        x, precs = [p[:, :40, :1000] for p in g.scans(0, 4)], list(g.precisions)
    elif case == "random_full":
        x = [synth.random_scans(rng, 3, 33, 517, np.uint32, 0.1)]
        precs = [1]
    elif case == "ragged_tiny":
        x = [synth.random_scans(rng, 5, 3, 7, dt, 0.4, scale=300) for dt in (np.uint32, np.uint16, np.uint8)]
        precs = [3, 1, 2]
    else:
        g = synth.stream(1, 0)
        x, precs, mode = g.scans(0, 5), list(g.precisions), 2
    ref, mref = oracle.encode(x, precs, mode=mode)
    dev = [to_dev(p) for p in x]
    for w in _wgs(J):
        banner("fused sequence", case, "wgs/CU", w)
        J.set_tuning(1, w)
        try:
            s, m = J.encode(dev, precs, mode=mode)
        finally:
            J.set_tuning(0, 0)
        got = s.cpu().numpy().tobytes()
        assert np.array_equal(m, mref), (case, w)
        if got != ref:
            _, rg = split_stream(got)
            _, rr = split_stream(ref)
            bad = [i for i, (a, b) in enumerate(zip(rg, rr)) if a != b]
            raise AssertionError(f"{case} at {w} workgroups/CU: records {bad[:10]} differ")


def test_fused_batched_set_graph_and_direct(J):
    """All 64 streams of the batched set (four sizes), three steps, through
    the fused launch in a graph-replayed batch and in the direct batched
    call; each stream's records equal the oracle's encoding of its scans."""
    import torch
    T = 3
    gens = [synth.stream(3, s) for s in range(synth.CONFIGS[3].streams)]
    data = [g.scans(0, T) for g in gens]
    dev = [[to_dev(p) for p in d] for d in data]
    want = []
    for g, d in zip(gens, data):
        recs = split_stream(oracle.encode(d, g.precisions)[0])[1]
        A = len(g.widths)
        want.append([b"".join(recs[t * A:(t + 1) * A]) for t in range(T)])
    for w in _wgs(J):
        banner("fused batched set", "wgs/CU", w)
        J.set_tuning(1, w)
        mk = lambda: [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]  # noqa: E731
        sg, sd = mk(), mk()
        og = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sg]
        od = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sd]
        batch = J.Batch(sg, [[p[0] for p in d] for d in dev], og)
        try:
            for t in range(T):
                at = [[p[t] for p in d] for d in dev]
                lg, _ = batch.run(at)
                ld, _ = J.batch_encode_step(sd, at, od)
                for i in range(len(gens)):
                    assert og[i][:lg[i]].cpu().numpy().tobytes() == want[i][t], (w, t, i, "graph")
                    assert od[i][:ld[i]].cpu().numpy().tobytes() == want[i][t], (w, t, i, "direct")
        finally:
            J.set_tuning(0, 0)
            batch.close()
            for s in sg + sd:
                s.close()


def test_fused_step_context(J):
    import torch
    gens = [synth.stream(4, s) for s in range(5)]
    data = [g.scans(0, 2) for g in gens]
    dev = [[to_dev(p) for p in d] for d in data]
    banner("fused step context")
    J.set_tuning(1, 0)
    streams = [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]
    step = J.Step(64, 8 << 20)
    out = torch.empty(40 << 20, dtype=torch.uint8, device="cuda")
    try:
        for t in range(2):
            step.submit(streams, [[p[t] for p in d] for d in dev], out)
            lens, _ = step.finish()
            buf = out[:sum(lens)].cpu().numpy().tobytes()
            p = 0
            for i, (g, d) in enumerate(zip(gens, data)):
                recs = split_stream(oracle.encode(d, g.precisions)[0])[1]
                A = len(g.widths)
                assert buf[p:p + lens[i]] == b"".join(recs[t * A:(t + 1) * A]), (t, i)
                p += lens[i]
    finally:
        J.set_tuning(0, 0)
        step.close()
        for s in streams:
            s.close()


def test_autotuner_candidates_are_byte_identical(J, tmp_path):
    from paper_2209_08196_amd import autotune
    gens = [synth.stream(3, s) for s in range(16)]
    data = [g.scans(0, 3) for g in gens]
    dev = [[to_dev(p) for p in d] for d in data]
    scans = [[[p[t] for p in d] for d in dev] for t in range(3)]
    mk = lambda: [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]  # noqa: E731
    banner("autotune 16 streams")
    try:
        rep = autotune.tune(mk, scans, cache=str(tmp_path / "tune.json"))
        assert not rep["cached"]
        assert len(rep["candidates"]) >= 2
        assert all(c["byte_identical"] for c in rep["candidates"]), rep
        assert J.get_tuning()[0] == rep["best"]
        rep2 = autotune.tune(mk, scans, cache=str(tmp_path / "tune.json"))
        assert rep2["cached"] and rep2["best"] == rep["best"]
    finally:
        J.set_tuning(0, 0)
