"""GPU: the serving loop (real-time continuous batching over two
asynchronous step contexts, stream states in a budgeted pool) gives every
admitted stream exactly the records of encoding each of its sessions' scan
sequence alone (the oracle), through the C ABI, at the serving
configuration's sizes (32x1024, 64x1024, 64x2048, 128x2048; range u32 and
three 16-bit attributes at 1 mm)."""
import collections

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


def _check_against_oracle(srv, gens, data):
    """Every kept record equals the oracle's record of the same scan when
    the stream's session is encoded alone (a session starts with an I-scan)."""
    checked = 0
    for sid, res in srv.results.items():
        g = gens[sid]
        A = len(g.widths)
        by_sess = collections.OrderedDict()
        for sess, k, rec in res:
            by_sess.setdefault(sess, []).append((k, rec))
        for sess, items in by_sess.items():
            ks = [k for k, _ in items]
            assert ks == sorted(ks) and len(set(ks)) == len(ks), (sid, sess, ks)
            planes = [np.ascontiguousarray(p[ks]) for p in data[sid]]
            recs = split_stream(oracle.encode(planes, g.precisions)[0])[1]
            for i, (k, got) in enumerate(items):
                assert got == b"".join(recs[i * A:(i + 1) * A]), (sid, sess, k)
                checked += 1
    return checked


def _serving_data(n, duration, session_s=None, seed=0):
    gens = [synth.stream(4, s) for s in range(n)]
    arrivals = synth.serving_arrivals(n, duration, base_seed=seed, session_s=session_s)
    T = [1 + max([k for _, s, k in arrivals if s == sid], default=0) for sid in range(n)]
    data = [g.scans(0, t) for g, t in zip(gens, T)]
    specs = {s: serve.StreamSpec(g.H, g.W, tuple(g.widths), tuple(g.precisions)) for s, g in enumerate(gens)}
    return gens, arrivals, data, specs


def test_served_streams_equal_their_alone_encoding(J):
    n = 32
    gens, arrivals, data, specs = _serving_data(n, 0.3)
    assert {(g.H, g.W) for g in gens} == set(synth.CONFIGS[4].sizes)
    dev = [[to_dev(p) for p in d] for d in data]
    banner("serve", n, "streams at the serving sizes,", len(arrivals), "scans, 8 GiB")
    srv = serve.Server.gpu(specs, 8 << 30)
    try:
        st = srv.run(arrivals, lambda sid, k: [p[k] for p in dev[sid]], keep_results=True)
        assert st.scans_dropped == 0 and st.scans_done == len(arrivals)
        assert st.admissions == n
        assert _check_against_oracle(srv, gens, data) == len(arrivals)
        s = st.summary()
        assert 0 < s["p50_ms"] <= s["p99_ms"]
    finally:
        srv.close()


def test_served_streams_under_a_tight_budget_with_sessions(J):
    """Streams connect for 0.1-0.2 s each within 0.6 s; the budget holds
    a few states, so scans are dropped, idle streams are closed and their
    memory is reused by later ones; every served session still equals its
    alone-encoding."""
    n = 24
    gens, arrivals, data, specs = _serving_data(n, 0.6, session_s=(0.1, 0.2), seed=3)
    dev = [[to_dev(p) for p in d] for d in data]
    probe = serve.Server.gpu({0: specs[0]}, 8 << 30)
    one_step = probe.fixed // probe.slots
    probe.close()
    budget = 2 * one_step + 4 * max(J.stream_state_bytes(s.height, s.width, s.widths) for s in specs.values())
    banner("serve with sessions", n, "streams,", len(arrivals), "scans, budget", budget)
    srv = serve.Server.gpu(specs, budget, idle_s=0.05)
    try:
        st = srv.run(arrivals, lambda sid, k: [p[k] for p in dev[sid]], keep_results=True)
        assert st.scans_done + st.scans_dropped == len(arrivals)
        assert st.scans_done > 0 and st.evictions > 0 and st.admissions > 4
        assert st.pool_peak_bytes <= srv.pool.capacity
        assert _check_against_oracle(srv, gens, data) == st.scans_done
    finally:
        srv.close()


def test_two_step_contexts_in_flight(J):
    """Two jiffy_step contexts submitted on two HIP streams before either is
    finished: both finish with the records of the plain batched call."""
    import torch
    gens = [synth.stream(4, s) for s in range(6)]
    data = [g.scans(0, 2) for g in gens]
    dev = [[to_dev(p) for p in d] for d in data]
    banner("two step contexts")
    mk = lambda: [J.Stream(g.H, g.W, g.widths, g.precisions) for g in gens]  # noqa: E731
    sa, sb = mk(), mk()
    steps = [J.Step(64, 8 << 20), J.Step(64, 8 << 20)]
    outs = [torch.empty(40 << 20, dtype=torch.uint8, device="cuda") for _ in range(2)]
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    ref = [torch.empty(s.record_bound(), dtype=torch.uint8, device="cuda") for s in sb]
    try:
        for k in range(2):
            torch.cuda.synchronize()
            steps[0].submit(sa[:3], [[p[k] for p in d] for d in dev[:3]], outs[0], stream=hs[0])
            steps[1].submit(sa[3:], [[p[k] for p in d] for d in dev[3:]], outs[1], stream=hs[1])
            with pytest.raises(J.JiffyError):  # a stream in an unfinished step is refused
                J.batch_encode_step([sa[0]], [[p[k] for p in dev[0]]], [ref[0]])
            la, _ = steps[0].finish()
            lb, _ = steps[1].finish()
            lr, _ = J.batch_encode_step(sb, [[p[k] for p in d] for d in dev], ref)
            got = []
            for lens, out in ((la, outs[0]), (lb, outs[1])):
                p = 0
                for n in lens:
                    got.append(out[p:p + n].cpu().numpy().tobytes())
                    p += n
            want = [ref[i][:lr[i]].cpu().numpy().tobytes() for i in range(6)]
            assert got == want, k
    finally:
        for s in steps:
            s.close()
        for s in sa + sb:
            s.close()
