"""GPU: the ablated codecs' record sizes and the run-length mask codec's
sizes (jiffy_ablate) equal the oracle's, value for value: synthetic range
and attribute scans, ragged and tiny shapes, full-range noise, all-zero and
zero-free scans, a standing sensor (empty XOR masks), more records than the
run-length kernel has workgroups, and whole 128x4096 scans."""
import numpy as np
import pytest

from gpu_util import banner, to_dev
from oracle import ablation as ab
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


def _case(name):
    rng = np.random.default_rng(17)
    if name == "c1":
        g = synth.stream(1, 0)
        return g.scans(0, 4), list(g.precisions)
    if name == "c2_crop":
        g = synth.stream(2, 0)
        return [p[:, :24, :512] for p in g.scans(28, 32)], list(g.precisions)
    if name == "ragged_tiny":
        return [synth.random_scans(rng, 5, 3, 7, dt, 0.4, scale=300) for dt in (np.uint32, np.uint16, np.uint8)], \
            [3, 1, 2]
    if name == "random_full":
        return [synth.random_scans(rng, 3, 33, 517, np.uint32, 0.1)], [1]
    if name == "zeros_and_full":
        z = np.zeros((3, 16, 200), np.uint16)
        z[1] = rng.integers(1, 65535, (16, 200))
        return [z], [1]
    if name == "standing":
        g = synth.stream(1, 0)
        x = g.scans(0, 1)[0]
        return [np.repeat(x, 3, axis=0)], [10]
    if name == "many_records":  # 300 scans x 2 attributes: the run-length kernel loops over records
        return [synth.random_scans(rng, 300, 5, 13, np.uint16, 0.5, scale=50),
                synth.random_scans(rng, 300, 5, 13, np.uint8, 0.2, scale=9)], [1, 1]
    if name == "c5_full":
        g = synth.stream(5, 0)
        return g.scans(18, 21), [1]  # a scene cut at scan 20
    raise ValueError(name)


CASES = ["c1", "c2_crop", "ragged_tiny", "random_full", "zeros_and_full", "standing", "many_records", "c5_full"]


@pytest.mark.parametrize("name", CASES)
def test_ablation_sizes_equal_oracle(J, name):
    planes, precs = _case(name)
    banner("ablate", name, planes[0].shape)
    want = ab.ablate(planes, precs)
    got = J.ablate([to_dev(p) for p in planes], precs)
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)[:8]
        raise AssertionError(f"{name}: first mismatches (t, a, k) {bad.tolist()}: "
                             f"got {[int(got[tuple(b)]) for b in bad]} want {[int(want[tuple(b)]) for b in bad]}")


def test_ablation_repeated_and_argument_checks(J):
    import torch
    planes, precs = _case("c1")
    dev = [to_dev(p) for p in planes]
    a = J.ablate(dev, precs)
    b = J.ablate(dev, precs)
    assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        J.ablate([dev[0].cpu()], precs)
    with pytest.raises(ValueError):
        J.ablate([dev[0][:, :, :-1]], precs)  # not contiguous
    assert torch.cuda.is_available()
