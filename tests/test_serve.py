"""Host logic of the serving loop (no GPU): admission by the device-memory
budget, one scan per stream per step in arrival order, workspace-limited
steps, virtual-time latencies.  The encoder is a stand-in that records what
it was given."""
from paper_2209_08196_amd import serve
from paper_2209_08196_amd.serve import Server, StreamSpec


def _specs(n, shape=(16, 64), widths=(4, 2)):
    return {s: StreamSpec(shape[0], shape[1], widths, (1,) * len(widths)) for s in range(n)}


def _fake_encoder(log):
    def step(sids, scans):
        log.append(list(zip(sids, scans)))
        return [f"{sid}:{k}".encode() for sid, k in zip(sids, scans)]
    return step


def test_admission_by_budget_rejects_late_streams():
    specs = _specs(6)
    one = serve.state_bytes(16, 64, (4, 2)) + serve.record_bound(16, 64, (4, 2))
    ws = int(1.25 * serve.workspace_bytes(16, 64, (4, 2)))
    budget = 3 * one + ws  # room for three streams and one step's workspace
    arrivals = sorted([(0.001 * s + 0.01 * k, s, k) for s in range(6) for k in range(4)])
    log = []
    srv = Server(specs, budget, _fake_encoder(log))
    st = srv.run(arrivals, lambda sid, k: k, keep_results=True)
    assert srv.admitted == {0, 1, 2} and srv.rejected == {3, 4, 5}
    assert st.scans_done == 12 and st.scans_dropped == 12
    for sid in range(3):  # every admitted scan, in order, exactly once
        assert srv.results[sid] == [f"{sid}:{k}".encode() for k in range(4)]
    assert st.resident_bytes == 3 * one <= budget - ws


def test_one_scan_per_stream_per_step_in_arrival_order():
    specs = _specs(3)
    arrivals = [(0.0, 0, 0), (0.0, 0, 1), (0.0, 1, 0), (0.0, 2, 0), (0.0, 0, 2)]
    log = []
    srv = Server(specs, 1 << 40, _fake_encoder(log))
    st = srv.run(arrivals, lambda sid, k: k)
    for step in log:
        sids = [s for s, _ in step]
        assert len(sids) == len(set(sids))
    seq0 = [k for step in log for s, k in step if s == 0]
    assert seq0 == [0, 1, 2]
    assert st.steps == 3 and st.batch_sizes == [3, 1, 1]
    assert all(x >= 0 for x in st.latencies_s)


def test_workspace_limits_the_step():
    specs = _specs(8)
    one = serve.state_bytes(16, 64, (4, 2)) + serve.record_bound(16, 64, (4, 2))
    w = serve.workspace_bytes(16, 64, (4, 2))
    budget = 8 * one + int(1.25 * 3 * w) + 1  # all streams, three scans' workspace per step
    arrivals = [(0.0, s, 0) for s in range(8)]
    log = []
    srv = Server(specs, budget, _fake_encoder(log))
    st = srv.run(arrivals, lambda sid, k: k)
    assert len(srv.admitted) == 8
    assert st.batch_sizes == [3, 3, 2]


def test_max_batch_and_virtual_clock():
    specs = _specs(5)
    arrivals = [(1.0 + 0.5 * k, s, k) for k in range(3) for s in range(5)]
    arrivals.sort()
    srv = Server(specs, 1 << 40, _fake_encoder([]), max_batch=2)
    st = srv.run(arrivals, lambda sid, k: k)
    assert max(st.batch_sizes) == 2
    assert st.scans_done == 15
    assert st.sim_end_s >= 2.0  # the clock followed the arrivals
    s = st.summary()
    assert s["p99_ms"] >= s["p50_ms"] >= 0


def test_accounting_matches_the_stream_state():
    # two halves of samples (+16 bytes each) and of valid words, per attribute
    assert serve.state_bytes(2, 64, (4,)) == 2 * (128 * 4 + 16) + 2 * 8 * 2


def test_dropped_only_arrivals_do_not_make_empty_steps():
    specs = _specs(2)
    one = serve.state_bytes(16, 64, (4, 2)) + serve.record_bound(16, 64, (4, 2))
    budget = one + int(1.25 * serve.workspace_bytes(16, 64, (4, 2)))
    arrivals = [(0.0, 0, 0), (0.5, 1, 0), (1.0, 1, 1), (1.5, 0, 1)]
    srv = Server(specs, budget, _fake_encoder([]))
    st = srv.run(arrivals, lambda sid, k: k)
    assert st.scans_done == 2 and st.scans_dropped == 2
    assert 0 not in st.batch_sizes
