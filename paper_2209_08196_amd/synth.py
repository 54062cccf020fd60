"""Seeded synthetic LiDAR scan sequences.

Stand-ins for the paper's Ouster / Newer College / NTU VIRAL recordings
(Sec. IV-B, Tables I-II), which are not available here.  The generator only
produces raw sensor samples (ranges in millimetres, 8/16-bit attributes, zero
as the no-return sentinel of Sec. III-A); it contains none of the codec's
arithmetic, so both the GPU library and the CPU oracle take its output as
plain input.

Scene model: H beams over a +-22.5 degree vertical field of view, W columns
over 360 degrees of azimuth, sensor 1.8 m above a ground plane, 4-8 vertical
walls enclosing the sensor at 8-60 m and 10-30 boxes at 5-60 m.  A scan is
the scene's panorama seen at the sensor's yaw (whole-column rotation) with
a first-order correction for a small translation, Gaussian range noise of
about 20 mm (10 mm fixed per sensor pixel, 17 mm fresh every scan) and zero blobs from a smooth random field fixed in world
azimuth, thresholded so that the zero fraction hits the configuration's
target.  Attributes follow the surface and range:
  signal ~ Poisson(k * albedo / max(r_m, 1)^2), reflectivity = per-surface
  base + Poisson noise, near-IR ~ Poisson(smooth ambient field),
  second return = first return + U(0.5, 20) m on about 10% of pixels.
"""
from __future__ import annotations

import dataclasses

import numpy as np

MAX_RANGE_MM = 120_000  # OS1-like maximum range (Table I)
MIN_RANGE_MM = 300
SENSOR_HEIGHT_M = 1.8
NOISE_STATIC_MM = 10.0   # fixed per sensor pixel (calibration bias)
NOISE_TEMPORAL_MM = 17.0  # fresh every scan; about 20 mm in total

_DTYPES = {"u8": np.uint8, "u16": np.uint16, "u32": np.uint32}


@dataclasses.dataclass(frozen=True)
class Attr:
    name: str
    dtype: str  # "u8" | "u16" | "u32"
    precision: int


@dataclasses.dataclass(frozen=True)
class Config:
    cid: int
    name: str
    streams: int
    scans: int
    sizes: tuple  # candidate (H, W) shapes
    attrs: tuple  # Attr tuple
    zero_frac: float
    yaw_deg: tuple  # per-scan yaw step range (lo, hi) in degrees
    yaw_per_stream: bool  # draw one yaw step per stream (else per scan)
    cut_every: int  # new scene every n scans (0 = never)
    size_rule: str  # "first" | "mod" | "uniform"
    stops: tuple = ()  # (first, end) scan ranges with the sensor standing still


RANGE_P10 = Attr("range", "u32", 10)
RANGE_P1 = Attr("range", "u32", 1)

CONFIGS = {
    1: Config(1, "plain-64x1024-range-1cm", 1, 10, ((64, 1024),), (RANGE_P10,), 0.15, (0.5, 0.5), True, 0,
              "first"),
    2: Config(2, "dual-return-128x2048-5attr-1mm", 1, 100, ((128, 2048),),
              (RANGE_P1, Attr("range2", "u32", 1), Attr("signal", "u16", 1), Attr("reflectivity", "u8", 1),
               Attr("nearir", "u16", 1)), 0.20, (0.5, 0.5), True, 0, "first", ((30, 60),)),
    3: Config(3, "batched-64-streams-mixed-range-signal", 64, 50,
              ((16, 1024), (32, 2048), (64, 1024), (128, 2048)), (RANGE_P10, Attr("signal", "u16", 1)), 0.20,
              (0.0, 2.0), True, 0, "mod"),
    4: Config(4, "serving-256-streams-range-3x16bit", 256, 0, ((32, 1024), (64, 1024), (64, 2048), (128, 2048)),
              (RANGE_P1, Attr("signal", "u16", 1), Attr("nearir", "u16", 1), Attr("reflectivity16", "u16", 1)),
              0.20, (0.0, 2.0), True, 0, "uniform"),
    5: Config(5, "stress-128x4096-drone-range-1mm", 32, 200, ((128, 4096),), (RANGE_P1,), 0.60, (5.0, 15.0),
              False, 20, "first"),
}


def _smooth_field(rng, h, w, cell_h=8, cell_w=32):
    """Smooth random field on an (h, w) grid, periodic in w (azimuth)."""
    ch = max(2, h // cell_h + 2)
    cw = max(4, w // cell_w)
    coarse = rng.standard_normal((ch, cw))
    ys = np.linspace(0, ch - 1, h)
    y0 = np.floor(ys).astype(int)
    y1 = np.minimum(y0 + 1, ch - 1)
    fy = (ys - y0)[:, None]
    xs = np.arange(w) * cw / w
    x0 = np.floor(xs).astype(int) % cw
    x1 = (x0 + 1) % cw
    fx = (xs - np.floor(xs))[None, :]
    rows = coarse[y0] * (1 - fy) + coarse[y1] * fy
    return rows[:, x0] * (1 - fx) + rows[:, x1] * fx


class _Scene:
    """Static world geometry rendered as a panorama at the start position."""

    def __init__(self, rng, H, W, zero_frac):
        el = np.deg2rad(np.linspace(22.5, -22.5, H))[:, None]
        az = (2 * np.pi * np.arange(W) / W)[None, :]
        dx = np.cos(el) * np.cos(az)
        dy = np.cos(el) * np.sin(az)
        dz = np.sin(el) * np.ones_like(az)
        self.dirs = (dx.astype(np.float32), dy.astype(np.float32), dz.astype(np.float32))
        best = np.full((H, W), np.inf, np.float32)
        sid = np.zeros((H, W), np.int16)
        # ground plane z = 0 (surface id 1)
        with np.errstate(divide="ignore", invalid="ignore"):
            tg = np.where(dz < 0, SENSOR_HEIGHT_M / -dz, np.inf).astype(np.float32)
        hit = tg < best
        best[hit], sid[hit] = tg[hit], 1
        # enclosing vertical walls n . p = c (surface ids 2..)
        nw = int(rng.integers(4, 9))
        base = rng.uniform(0, 2 * np.pi)
        for k in range(nw):
            alpha = base + 2 * np.pi * k / nw + rng.uniform(-0.2, 0.2)
            c = rng.uniform(8.0, 60.0)
            nd = np.cos(alpha) * dx + np.sin(alpha) * dy
            with np.errstate(divide="ignore", invalid="ignore"):
                tw = np.where(nd > 1e-6, c / nd, np.inf).astype(np.float32)
            hit = tw < best
            best[hit], sid[hit] = tw[hit], 2 + k
        # axis-aligned boxes standing on the ground (surface ids 16..)
        nbx = int(rng.integers(10, 31))
        oz = SENSOR_HEIGHT_M
        for k in range(nbx):
            d = rng.uniform(5.0, 60.0)
            phi = rng.uniform(0, 2 * np.pi)
            cx, cy = d * np.cos(phi), d * np.sin(phi)
            hx, hy, hz = rng.uniform(0.5, 3.0), rng.uniform(0.5, 3.0), rng.uniform(0.5, 4.0)
            lo = np.array([cx - hx, cy - hy, 0.0])
            hi = np.array([cx + hx, cy + hy, hz])
            tmin = np.full((H, W), -np.inf, np.float32)
            tmax = np.full((H, W), np.inf, np.float32)
            for o, dv, l, h in ((0.0, dx, lo[0], hi[0]), (0.0, dy, lo[1], hi[1]), (oz, dz, lo[2], hi[2])):
                with np.errstate(divide="ignore", invalid="ignore"):
                    inv = 1.0 / dv
                    t1 = (l - o) * inv
                    t2 = (h - o) * inv
                t1, t2 = np.minimum(t1, t2), np.maximum(t1, t2)
                # rays parallel to a slab: inside -> unbounded, outside -> miss
                par = np.abs(dv) < 1e-9
                inside = (o >= l) & (o <= h)
                t1 = np.where(par, -np.inf if inside else np.inf, t1)
                t2 = np.where(par, np.inf if inside else -np.inf, t2)
                tmin = np.maximum(tmin, t1)
                tmax = np.minimum(tmax, t2)
            tb = np.where((tmax >= tmin) & (tmin > 0), tmin, np.inf).astype(np.float32)
            hit = tb < best
            best[hit], sid[hit] = tb[hit], 16 + k
        rng_mm = best * 1000.0
        valid = np.isfinite(rng_mm) & (rng_mm <= MAX_RANGE_MM) & (rng_mm >= MIN_RANGE_MM)
        self.range_mm = np.where(valid, rng_mm, 0.0).astype(np.float32)
        self.surface = np.where(valid, sid, 0)
        # zero blobs fixed in world azimuth
        field = _smooth_field(rng, H, W)
        f0 = 1.0 - valid.mean()
        extra = max(0.0, zero_frac - f0)
        if extra > 0 and valid.any():
            thr = np.quantile(field[valid], 1.0 - extra / valid.mean())
            self.blob = field > thr
        else:
            self.blob = np.zeros((H, W), bool)
        nsurf = 16 + 31
        self.albedo = rng.uniform(0.1, 1.0, nsurf)
        self.refl_base = rng.uniform(10, 200, nsurf)
        self.ambient = 50.0 + 1450.0 / (1.0 + np.exp(-1.5 * _smooth_field(rng, H, W, 16, 64)))
        # about 10% of all pixels carry a second return
        p2 = 0.10 / max(1.0 - zero_frac, 0.1)
        self.second_p = np.clip(p2 * (1.0 + 0.8 * _smooth_field(rng, H, W)), 0.0, 1.0)


class StreamGen:
    """One sensor stream of a configuration.  scans(t0, t1) returns a list of
    [t1-t0, H, W] arrays, one per attribute, in the configuration's order."""

    def __init__(self, cfg: Config, stream_id: int = 0, base_seed: int = 0, size=None, standing=False):
        if standing:  # the same scene seen by a sensor that never moves (a fixed monitoring sensor)
            cfg = dataclasses.replace(cfg, stops=((0, 1 << 30),))
        self.cfg = cfg
        self.stream_id = stream_id
        ss = np.random.SeedSequence([cfg.cid, stream_id, base_seed])
        self._seed = ss
        rng = np.random.default_rng(ss.spawn(1)[0])
        if size is not None:
            self.H, self.W = size
        elif cfg.size_rule == "mod":
            self.H, self.W = cfg.sizes[stream_id % len(cfg.sizes)]
        elif cfg.size_rule == "uniform":
            self.H, self.W = cfg.sizes[int(rng.integers(len(cfg.sizes)))]
        else:
            self.H, self.W = cfg.sizes[0]
        lo, hi = cfg.yaw_deg
        self._stream_yaw = float(rng.uniform(lo, hi))
        self._rng_seq = ss
        self._static_noise = np.random.default_rng(ss.spawn(2)[1]).normal(0.0, NOISE_STATIC_MM, (self.H, self.W))
        self._scene_cache = {}
        self._pose_cache = None

    @property
    def widths(self):
        return [np.dtype(_DTYPES[a.dtype]).itemsize for a in self.cfg.attrs]

    @property
    def precisions(self):
        return [a.precision for a in self.cfg.attrs]

    @property
    def dtypes(self):
        return [_DTYPES[a.dtype] for a in self.cfg.attrs]

    def _scene(self, idx):
        if idx not in self._scene_cache:
            self._scene_cache.clear()
            rng = np.random.default_rng(np.random.SeedSequence([self.cfg.cid, self.stream_id, 7919, idx]))
            self._scene_cache[idx] = _Scene(rng, self.H, self.W, self.cfg.zero_frac)
        return self._scene_cache[idx]

    def _poses(self, n):
        """Yaw (degrees) and x-translation (m) for scans 0..n-1."""
        if self._pose_cache is None or len(self._pose_cache[0]) < n:
            rng = np.random.default_rng(np.random.SeedSequence([self.cfg.cid, self.stream_id, 104729]))
            m = max(n, 64)
            lo, hi = self.cfg.yaw_deg
            steps = np.full(m, self._stream_yaw) if self.cfg.yaw_per_stream else rng.uniform(lo, hi, m)
            steps[0] = 0.0
            moving = np.ones(m)
            for a, b in self.cfg.stops:  # stop-and-go: no motion inside a stop
                moving[a:b] = 0.0
            cut = self.cfg.cut_every
            yaw = np.zeros(m)
            tx = np.zeros(m)
            for t in range(1, m):
                if cut and t % cut == 0:
                    continue
                yaw[t] = yaw[t - 1] + steps[t] * moving[t]
                tx[t] = tx[t - 1] + 0.05 * moving[t]
            self._pose_cache = (yaw, tx)
        return self._pose_cache

    def scan(self, t: int):
        cfg = self.cfg
        yaw, tx = self._poses(t + 1)
        scene = self._scene(t // cfg.cut_every if cfg.cut_every else 0)
        rng = np.random.default_rng(np.random.SeedSequence([cfg.cid, self.stream_id, 31337, t]))
        shift = int(round(yaw[t] / 360.0 * self.W)) % self.W
        roll = lambda a: np.roll(a, -shift, axis=1)  # noqa: E731
        dx = roll(scene.dirs[0])
        r = roll(scene.range_mm).astype(np.float64)
        valid = (r > 0) & ~roll(scene.blob)
        r = r - tx[t] * 1000.0 * dx + self._static_noise + rng.normal(0.0, NOISE_TEMPORAL_MM, r.shape)
        r = np.clip(np.rint(r), 1, MAX_RANGE_MM + 1000)
        rng_u32 = np.where(valid, r, 0).astype(np.uint32)
        sid = roll(scene.surface)
        out = []
        for a in cfg.attrs:
            if a.name == "range":
                v = rng_u32
            elif a.name == "range2":
                has2 = valid & (rng.random(r.shape) < roll(scene.second_p))
                r2 = r + rng.uniform(500.0, 20000.0, r.shape)
                v = np.where(has2, np.rint(r2), 0).astype(np.uint32)
            elif a.name == "signal":
                lam = 4.0e5 * scene.albedo[sid] / np.maximum(r / 1000.0, 1.0) ** 2
                v = np.where(valid, np.minimum(rng.poisson(np.minimum(lam, 1e6)), 65535), 0).astype(np.uint16)
            elif a.name in ("reflectivity", "reflectivity16"):
                base = scene.refl_base[sid]
                val = np.minimum(np.rint(base + rng.poisson(8.0, r.shape)), 255)
                v = np.where(valid, val, 0).astype(np.uint8 if a.dtype == "u8" else np.uint16)
            elif a.name == "nearir":
                v = np.where(valid, np.minimum(rng.poisson(roll(scene.ambient)), 65535), 0).astype(np.uint16)
            else:
                raise ValueError(a.name)
            out.append(v)
        return out

    def scans(self, t0: int, t1: int):
        per = [self.scan(t) for t in range(t0, t1)]
        return [np.stack([p[a] for p in per]) for a in range(len(self.cfg.attrs))]


def stream(cid: int, stream_id: int = 0, base_seed: int = 0, size=None, standing=False) -> StreamGen:
    return StreamGen(CONFIGS[cid], stream_id, base_seed, size, standing)


def random_scans(rng, T, H, W, dtype, zero_frac=0.2, scale=None):
    """Unstructured random scans for edge-case tests: uniform values with a
    given fraction of zeros.  Returns [T, H, W]."""
    dt = np.dtype(dtype)
    top = scale if scale is not None else np.iinfo(dt).max
    v = rng.integers(1, int(top) + 1, size=(T, H, W), dtype=np.uint64)
    z = rng.random((T, H, W)) < zero_frac
    return np.where(z, 0, v).astype(dt)


FOV_ELEV_RAD = (-np.pi / 8, np.pi / 8)  # the +-22.5 degree vertical field of view


def cartesian_scan(rng, range_mm, attr_imgs=(), e_lo=FOV_ELEV_RAD[0], e_hi=FOV_ELEV_RAD[1], jitter=0.3,
                   invalid_frac=0.02, dup_frac=0.02, tie_frac=0.005):
    """The raw output of a sensor that reports Cartesian points (Sec. III-A):
    every nonzero pixel of a range image (mm) becomes a float32 point in
    metres at its row's elevation and its column's azimuth (row 0 at the top
    of the band, column 0 at azimuth 0, counter-clockwise), each moved by a
    uniform fraction of a bin up to +-jitter, at a range of the pixel's
    millimetres plus 0.25 mm (float32 rounding stays far below that).  Mixed
    in, in random order: invalid points (NaN, the origin, above the band),
    farther duplicates of some pixels, and duplicates at the same
    millimetre (ties).  Each point carries its pixel's attribute values;
    duplicates carry other values.
    Returns (xyz [N, 3] float32, attribute arrays [N], pixel index [N], -1 for invalid points)."""
    H, W = range_mm.shape
    rows, cols = np.nonzero(range_mm)
    pix = rows * W + cols
    n = pix.size
    nd, nt = int(dup_frac * n), int(tie_frac * n)
    di = rng.choice(n, nd + nt, replace=nd + nt > n)
    pix_all = np.concatenate([pix, pix[di]])
    rows_all, cols_all = pix_all // W, pix_all % W
    mm = range_mm.ravel()[pix_all].astype(np.float64)
    mm[n:n + nd] += rng.uniform(1.0, 5000.0, nd).round()
    m = pix_all.size
    r = (mm + 0.25) / 1000.0
    e = e_hi - (rows_all + 0.5 + rng.uniform(-jitter, jitter, m)) * (e_hi - e_lo) / H
    a = (cols_all + 0.5 + rng.uniform(-jitter, jitter, m)) * 2.0 * np.pi / W
    xyz = np.stack([r * np.cos(e) * np.cos(a), r * np.cos(e) * np.sin(a), r * np.sin(e)], 1)
    attrs = []
    for img in attr_imgs:
        v = img.ravel()[pix_all].copy()
        top = np.iinfo(img.dtype).max
        v[n:] = rng.integers(0, top, m - n, endpoint=True).astype(img.dtype)
        attrs.append(v)
    ni = int(invalid_frac * n)
    bad = np.zeros((ni, 3))
    kind = rng.integers(0, 3, ni)
    bad[kind == 0] = np.nan
    up = kind == 2  # above the band, 30 m away
    ang = e_hi + 0.05
    bad[up] = [30.0 * np.cos(ang), 0.0, 30.0 * np.sin(ang)]
    xyz = np.concatenate([xyz, bad])
    attrs = [np.concatenate([v, rng.integers(0, np.iinfo(v.dtype).max, ni, endpoint=True).astype(v.dtype)])
             for v in attrs]
    src = np.concatenate([pix_all, np.full(ni, -1)])
    order = rng.permutation(xyz.shape[0])
    return xyz[order].astype(np.float32), [v[order] for v in attrs], src[order]


def serving_arrivals(n_streams: int, duration_s: float, base_seed: int = 0, session_s=None):
    """Arrival times (s) of scans for the serving configuration: each stream
    runs at 10 or 20 Hz (fair coin) with a random phase and Poisson(2) ms
    jitter.  With session_s = (lo, hi) each stream is connected only for a
    window of U(lo, hi) seconds starting at a uniform time (sensors that come
    and go).  Returns a list of (time, stream_id, scan_index), time-sorted;
    scan indices count each stream's scans from 0."""
    rng = np.random.default_rng(np.random.SeedSequence([4, 999, base_seed]))
    events = []
    for s in range(n_streams):
        period = 0.1 if rng.random() < 0.5 else 0.05
        phase = rng.uniform(0, period)
        lo, hi = 0.0, duration_s
        if session_s is not None:
            length = min(rng.uniform(*session_s), duration_s)
            lo = rng.uniform(0, duration_s - length)
            hi = lo + length
        k = j = 0
        while True:
            t = phase + j * period + rng.poisson(2.0) * 1e-3
            j += 1
            if t >= hi or t >= duration_s:
                break
            if t < lo:
                continue
            events.append((t, s, k))
            k += 1
    events.sort()
    return events


def config_pixels(cid: int) -> int:
    cfg = CONFIGS[cid]
    if cfg.size_rule == "mod":
        return sum(cfg.sizes[s % len(cfg.sizes)][0] * cfg.sizes[s % len(cfg.sizes)][1] for s in range(cfg.streams))
    h, w = cfg.sizes[0]
    return cfg.streams * h * w


__all__ = ["CONFIGS", "Config", "Attr", "StreamGen", "stream", "random_scans", "serving_arrivals", "cartesian_scan",
           "config_pixels"]
