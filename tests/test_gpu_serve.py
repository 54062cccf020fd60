"""GPU: the serving loop (continuous batching with admission by a
device-memory budget) gives every admitted stream exactly the records of
encoding its scan sequence alone (the oracle), through the C ABI."""
import numpy as np
import pytest

import oracle
from formatcheck import split_stream
from gpu_util import banner, to_dev
from paper_2209_08196_amd import serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()
    return jiffy


def test_served_streams_equal_their_alone_encoding(J):
    sizes = [(8, 256), (16, 128), (4, 1024), (16, 512), (2, 64)]
    n = 10
    gens = [synth.stream(4, s, size=sizes[s % len(sizes)]) for s in range(n)]
    arrivals = synth.serving_arrivals(n, 0.35, base_seed=1)
    T = [1 + max([k for _, s, k in arrivals if s == sid], default=-1) for sid in range(n)]
    data = [g.scans(0, max(t, 1)) for g, t in zip(gens, T)]
    dev = [[to_dev(p) for p in d] for d in data]
    specs = {s: serve.StreamSpec(g.H, g.W, tuple(g.widths), tuple(g.precisions)) for s, g in enumerate(gens)}
    costs = {s: serve.state_bytes(g.H, g.W, g.widths) + serve.record_bound(g.H, g.W, g.widths)
             for s, g in enumerate(gens)}
    ws = int(1.25 * max(serve.workspace_bytes(g.H, g.W, g.widths) for g in gens))
    first = sorted({s: min(t for t, ss, _ in arrivals if ss == s) for s in range(n)}.items(), key=lambda x: x[1])
    budget = ws + sum(costs[s] for s, _ in first[:6]) + 1  # the first six streams to arrive fit
    banner("serve", n, "streams", len(arrivals), "scans, budget", budget)
    srv = serve.Server.gpu(specs, budget)
    st = srv.run(arrivals, lambda sid, k: [p[k] for p in dev[sid]], keep_results=True)
    try:
        assert st.streams_admitted == 6 and st.streams_rejected == n - 6
        assert srv.admitted == {s for s, _ in first[:6]}
        assert st.scans_done + st.scans_dropped == len(arrivals)
        for sid in srv.admitted:
            g = gens[sid]
            recs = split_stream(oracle.encode(data[sid], g.precisions)[0])[1]
            A = len(g.widths)
            assert len(srv.results[sid]) == T[sid]
            for k, got in enumerate(srv.results[sid]):
                assert got == b"".join(recs[k * A:(k + 1) * A]), (sid, k)
        s = st.summary()
        assert 0 <= s["p50_ms"] <= s["p99_ms"]
        assert np.isfinite(s["points_per_s_busy"])
    finally:
        srv.close()
