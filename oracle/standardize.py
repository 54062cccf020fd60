"""Input standardization (Sec. III-A) -- TEST INFRASTRUCTURE ONLY.

Only the test-suite and the benchmark's reference checks use this module.
Cartesian points become the canonical range image: spherical coordinates,
a bin by elevation (row) and azimuth (column), the range quantized to an
unsigned integer of the image's width, zero where no valid point landed.
The paper states the steps, not their conventions; this project reads them
as follows (all arithmetic in IEEE double, each operation rounded once, in
the order written):

  x, y, z        the point's float32 coordinates (metres), widened exactly
  r              sqrt(x*x + y*y + z*z)
  e              atan2(z, sqrt(x*x + y*y))           elevation
  a              atan2(y, x), plus 2 pi when negative  azimuth in [0, 2 pi)
  row            floor(((e_hi - e) * H) / (e_hi - e_lo)); valid when 0 <= row < H
  col            floor((a * W) / (2 pi)), W becoming 0 (a rounded up to 2 pi)
  q              floor(r / unit + 0.5); valid when 1 <= q <= 2^(8 w) - 1

A point with a non-finite coordinate, outside the elevation band or with q
out of range is dropped (Sec. III-A: invalid and out-of-range measurements
are zero).  Several points in one cell: the one with the smallest q wins,
ties going to the earlier point.  The winner's attributes (integers of
their own widths, one per point) are carried into attribute images of the
same grid; empty cells hold zeros.

atan2 is not correctly rounded, so another implementation may put a point
lying within a few units in the last place of a bin edge into the
neighbouring bin; ``ambiguous`` lists such points for the tests.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def _prep(xyz):
    p = np.asarray(xyz, dtype=np.float32).reshape(-1, 3).astype(np.float64)
    return p[:, 0], p[:, 1], p[:, 2]


def spherical(xyz):
    """(r, elevation, azimuth in [0, 2 pi)) of every point, in double."""
    x, y, z = _prep(xyz)
    with np.errstate(invalid="ignore"):
        h = np.sqrt(x * x + y * y)
        r = np.sqrt(x * x + y * y + z * z)
        e = np.arctan2(z, h)
        a = np.arctan2(y, x)
        a = np.where(a < 0, a + TWO_PI, a)
    return r, e, a


def bins(xyz, H, W, e_lo, e_hi, unit, range_bytes):
    """(row, col, q, valid) per point."""
    r, e, a = spherical(xyz)
    with np.errstate(invalid="ignore"):
        fr = np.floor(((e_hi - e) * H) / (e_hi - e_lo))
        fc = np.floor((a * W) / TWO_PI)
        fq = np.floor(r / unit + 0.5)
    fc = np.where(fc == W, 0.0, fc)
    top = float((1 << (8 * range_bytes)) - 1)
    finite = np.isfinite(fr) & np.isfinite(fc) & np.isfinite(fq)
    valid = finite & (fr >= 0) & (fr < H) & (fc >= 0) & (fc < W) & (fq >= 1) & (fq <= top)
    row = np.where(valid, fr, 0).astype(np.int64)
    col = np.where(valid, fc, 0).astype(np.int64)
    q = np.where(valid, fq, 0).astype(np.uint64)
    return row, col, q, valid


def standardize(xyz, H, W, e_lo, e_hi, unit, range_bytes=4, attrs=()):
    """xyz: [N, 3] float32; attrs: per attribute an [N] integer array.
    Returns (range image [H, W], list of attribute images)."""
    row, col, q, valid = bins(xyz, H, W, e_lo, e_hi, unit, range_bytes)
    rdt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[range_bytes]
    img = np.zeros((H, W), rdt)
    winner = np.full((H, W), -1, np.int64)
    best = np.zeros((H, W), np.uint64)
    idx = np.flatnonzero(valid)
    # earliest point first among equal q: a stable sort on q, then the first per cell
    order = idx[np.argsort(q[idx], kind="stable")]
    cells = row[order] * W + col[order]
    _, first = np.unique(cells, return_index=True)
    w = order[first]
    cw = row[w] * W + col[w]
    winner.ravel()[cw] = w
    best.ravel()[cw] = q[w]
    img.ravel()[cw] = q[w].astype(rdt)
    outs = []
    for at in attrs:
        at = np.asarray(at)
        o = np.zeros((H, W), at.dtype)
        o.ravel()[cw] = at[w]
        outs.append(o)
    return img, outs


def standardize_loop(xyz, H, W, e_lo, e_hi, unit, range_bytes=4):
    """The same by a plain loop over points (small inputs)."""
    row, col, q, valid = bins(xyz, H, W, e_lo, e_hi, unit, range_bytes)
    rdt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[range_bytes]
    img = np.zeros((H, W), rdt)
    win = np.full((H, W), -1, np.int64)
    for i in range(len(q)):
        if not valid[i]:
            continue
        rr, cc = row[i], col[i]
        if win[rr, cc] < 0 or q[i] < img[rr, cc]:
            img[rr, cc] = q[i]
            win[rr, cc] = i
    return img, win


def ambiguous(xyz, H, W, e_lo, e_hi, unit, range_bytes=4, ulps=8):
    """Valid points whose row or column could change under an atan2 a few
    units in the last place away.  Returns (mask, alternative cells)."""
    r, e, a = spherical(xyz)
    valid = bins(xyz, H, W, e_lo, e_hi, unit, range_bytes)[3]
    amb = np.zeros(r.shape, bool)
    alt = []
    with np.errstate(invalid="ignore"):
        for de, da in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            e2 = e + de * ulps * np.spacing(np.abs(e) + 1e-300)
            a2 = a + da * ulps * np.spacing(np.abs(a) + 1e-300)
            fr = np.floor(((e_hi - e2) * H) / (e_hi - e_lo))
            fr0 = np.floor(((e_hi - e) * H) / (e_hi - e_lo))
            fc = np.floor((a2 * W) / TWO_PI) % W
            fc0 = np.floor((a * W) / TWO_PI) % W
            d = valid & ((fr != fr0) | (fc != fc0))
            amb |= d
            for i in np.flatnonzero(d):
                alt.append((int(fr[i]), int(fc[i])))
    return amb, alt
