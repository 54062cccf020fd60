"""Oracle pins of input standardization (Sec. III-A).

A range image turned into Cartesian points (jittered inside their bins, in
random order, with invalid points and farther duplicates) comes back
exactly, attributes included; points on the axes land in the columns a
quarter turn apart; the nearest point wins a cell and ties go to the earlier
point (checked against a plain loop over the points); invalid and
out-of-range points leave zeros."""
import numpy as np
import pytest

from oracle import standardize as st
from paper_2209_08196_amd import synth

E_LO, E_HI = synth.FOV_ELEV_RAD


@pytest.mark.parametrize("cid,t", [(1, 0), (2, 3), (5, 7)])
def test_range_image_round_trip(cid, t):
    g = synth.stream(cid, 0)
    sc = g.scans(t, t + 1)
    img = sc[0][0]
    H, W = img.shape
    rng = np.random.default_rng(cid)
    attr_imgs = [p[0] for p in sc[1:]] or [(img % 251).astype(np.uint8)]
    xyz, attrs, _ = synth.cartesian_scan(rng, img, attr_imgs, tie_frac=0.0)
    out, ao = st.standardize(xyz, H, W, E_LO, E_HI, 0.001, 4, attrs)
    assert np.array_equal(out, img)
    for a, im in zip(ao, attr_imgs):
        assert np.array_equal(a, np.where(img > 0, im, 0))
    assert not st.ambiguous(xyz, H, W, E_LO, E_HI, 0.001)[0].any()


def test_axes_and_band_centre():
    H, W = 64, 1024
    pts = np.array([[1.5, 0, 0], [0, 1.5, 0], [-1.5, 0, 0], [0, -1.5, 0]], np.float32)
    row, col, q, valid = st.bins(pts, H, W, E_LO, E_HI, 0.001, 4)
    assert valid.all()
    assert list(col) == [0, W // 4, W // 2, 3 * W // 4]
    assert list(row) == [H // 2] * 4  # elevation 0 is the middle of a symmetric band
    assert list(q) == [1500] * 4
    # the top edge of the band is row 0, the bottom edge is outside
    top = np.array([[np.cos(E_HI), 0, np.sin(E_HI)]], np.float32)
    assert st.bins(top, H, W, E_LO, E_HI, 0.001, 4)[0][0] in (0,)


def test_invalid_points_leave_zeros():
    H, W = 16, 64
    pts = np.array([[np.nan, 1, 1], [0, 0, 0], [np.inf, 0, 0], [5, 0, 5],  # NaN, origin, inf, above the band
                    [70.0, 0, 0],                                         # beyond 16 bits of millimetres
                    [0.0004, 0, 0]], np.float32)                          # rounds to q = 0
    img16, _ = st.standardize(pts, H, W, E_LO, E_HI, 0.001, 2)
    assert not img16.any()
    img32, _ = st.standardize(pts, H, W, E_LO, E_HI, 0.001, 4)
    assert img32.sum() == 70000  # only the far point, in 32 bits
    two = np.array([[0.3, 0, 0], [0.26, 0, 0]], np.float32)
    img8, _ = st.standardize(two, H, W, E_LO, E_HI, 0.001, 1)
    assert not img8.any()  # 300 and 260 mm do not fit in 8 bits
    img8, _ = st.standardize(two, H, W, E_LO, E_HI, 0.01, 1)
    assert img8.max() == 26 and img8.sum() == 26  # centimetres: the nearer point


def test_nearest_wins_and_ties_go_to_the_earlier_point():
    rng = np.random.default_rng(9)
    H, W = 8, 32
    n = 4000  # many points per cell
    r = rng.integers(1, 40, n) * 0.25  # few distinct ranges: many ties
    e = rng.uniform(E_LO + 1e-3, E_HI - 1e-3, n)
    a = rng.uniform(0, 2 * np.pi, n)
    xyz = np.stack([r * np.cos(e) * np.cos(a), r * np.cos(e) * np.sin(a), r * np.sin(e)], 1).astype(np.float32)
    attr = np.arange(n, dtype=np.uint32)  # the point's own index
    img, (who,) = st.standardize(xyz, H, W, E_LO, E_HI, 0.001, 4, [attr])
    img_l, win_l = st.standardize_loop(xyz, H, W, E_LO, E_HI, 0.001, 4)
    assert np.array_equal(img, img_l)
    filled = win_l >= 0
    assert np.array_equal(who[filled], win_l[filled].astype(np.uint32))
    assert filled.mean() > 0.9


def test_many_scans_are_independent():
    g = synth.stream(1, 0)
    sc = g.scans(0, 2)[0]
    rng = np.random.default_rng(2)
    outs = []
    for t in range(2):
        xyz, _, _ = synth.cartesian_scan(rng, sc[t])
        outs.append(st.standardize(xyz, 64, 1024, E_LO, E_HI, 0.001)[0])
    assert np.array_equal(np.stack(outs), sc)
