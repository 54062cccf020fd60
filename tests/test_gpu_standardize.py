"""GPU: input standardization (jiffy_standardize) equals the oracle's range
and attribute images cell for cell: synthetic Cartesian scans of the
plain, dual-return and 128x4096 streams (jittered, shuffled, with invalid
points, farther duplicates and ties), several scans per call padded with
NaN points, uniform random clouds with many points per cell, 8/16/32-bit
range images, and empty calls.  Cells that a point within a few units in
the last place of a bin edge could reach are left out of the comparison
(atan2 is not correctly rounded); none occur in these inputs."""
import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host
from oracle import standardize as st
from paper_2209_08196_amd import synth

pytestmark = pytest.mark.gpu
E_LO, E_HI = synth.FOV_ELEV_RAD


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08196_amd import jiffy
    jiffy.lib()
    return jiffy


def _pad(arrs, n, fill):
    out = np.full((len(arrs), n) + arrs[0].shape[1:], fill, arrs[0].dtype)
    for i, a in enumerate(arrs):
        out[i, :len(a)] = a
    return out


def _check(J, scans, H, W, unit, rb, name):
    """scans: list of (xyz [N, 3] float32, attrs list of [N])."""
    import torch
    n = max(len(x) for x, _ in scans)
    A = len(scans[0][1])
    xyz = _pad([x for x, _ in scans], n, np.nan)
    attrs = [_pad([at[a] for _, at in scans], n, 0) for a in range(A)]
    banner("standardize", name, xyz.shape, rb)
    rng_d, att_d = J.standardize(torch.from_numpy(xyz).cuda(), H, W, E_LO, E_HI, unit, rb,
                                 [to_dev(a) for a in attrs])
    got = to_host(rng_d, rb)
    got_a = [to_host(o, attrs[a].dtype.itemsize) for a, o in enumerate(att_d)]
    for s, (x, at) in enumerate(scans):
        want, want_a = st.standardize(xyz[s], H, W, E_LO, E_HI, unit, rb, [a[s] for a in attrs])
        amb, alt = st.ambiguous(xyz[s], H, W, E_LO, E_HI, unit, rb)
        keep = np.ones((H, W), bool)
        row, col, _, _ = st.bins(xyz[s], H, W, E_LO, E_HI, unit, rb)
        for i in np.flatnonzero(amb):
            keep[row[i], col[i]] = False
        for r, c in alt:
            if 0 <= r < H:
                keep[r, c % W] = False
        assert keep.mean() > 0.999, (name, s)
        assert np.array_equal(got[s][keep], want[keep]), (name, s, int((got[s] != want).sum()))
        for a in range(A):
            assert np.array_equal(got_a[a][s][keep], want_a[a][keep]), (name, s, a)


@pytest.mark.parametrize("cid", [1, 2, 5])
def test_stream_scans_equal_oracle(J, cid):
    g = synth.stream(cid, 0)
    sc = g.scans(4, 7)
    H, W = sc[0].shape[1:]
    rng = np.random.default_rng(40 + cid)
    scans = []
    for t in range(3):
        imgs = [p[t] for p in sc[1:]] or [(sc[0][t] % 251).astype(np.uint8)]
        xyz, attrs, _ = synth.cartesian_scan(rng, sc[0][t], imgs)
        scans.append((xyz, attrs))
    _check(J, scans, H, W, 0.001, 4, f"c{cid}")


@pytest.mark.parametrize("rb,unit", [(1, 0.1), (2, 0.001), (2, 0.01), (4, 0.0005)])
def test_random_clouds(J, rb, unit):
    rng = np.random.default_rng(rb * 7 + int(unit * 1e4))
    H, W = 32, 256
    scans = []
    for n in (20000, 5000, 1):
        r = rng.uniform(0, 90, n)
        e = rng.uniform(E_LO - 0.1, E_HI + 0.1, n)  # some outside the band
        a = rng.uniform(-np.pi, np.pi, n)
        xyz = np.stack([r * np.cos(e) * np.cos(a), r * np.cos(e) * np.sin(a), r * np.sin(e)], 1).astype(np.float32)
        xyz[rng.random(n) < 0.01] = np.nan
        attrs = [rng.integers(0, 1 << 16, n).astype(np.uint16), rng.integers(0, 1 << 32, n, dtype=np.uint64)
                 .astype(np.uint32)]
        scans.append((xyz, attrs))
    _check(J, scans, H, W, unit, rb, f"random rb{rb} unit{unit}")


def test_empty_calls(J):
    import torch
    xyz = torch.full((2, 10, 3), float("nan"), dtype=torch.float32, device="cuda")
    r, _ = J.standardize(xyz, 4, 8, E_LO, E_HI)
    assert not r.any()
    r, _ = J.standardize(torch.empty((3, 0, 3), dtype=torch.float32, device="cuda"), 4, 8, E_LO, E_HI)
    assert r.shape == (3, 4, 8) and not r.any()
    with pytest.raises(ValueError):
        J.standardize(xyz.double(), 4, 8, E_LO, E_HI)
    with pytest.raises(J.JiffyError):
        J.standardize(xyz, 4, 8, E_HI, E_LO)  # an empty band
