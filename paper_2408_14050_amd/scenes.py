"""Seeded synthetic disparity scenes for the occlusion detector.

This module only *generates inputs*: a fused centre-view fp32 disparity map
D (H x W, row-major), the peripheral-camera baselines (angle in degrees,
measured from +x towards +y with y pointing down, and the baseline ratio r),
the scan length L of every view and the detector thresholds.  It contains
none of the detector's arithmetic, so the CPU oracle and the GPU library can
both be fed from it without sharing any of the method.

The scene statistics stand in for the paper's evaluation data (SceneFlow,
the synthetic hyperspectral database and the CAMSI recording of Sec. 4),
which are not available: a smooth background plane plus fronto-parallel and
slanted objects painted back to front (painter's algorithm, ascending
disparity, so nearer surfaces overwrite farther ones), optional thin
structures and i.i.d. Gaussian noise.

Workloads (frame sizes are W x H):

* ``c0``  256x192, one view at 0 deg, r = 1, 4 axis-aligned rectangles,
  no noise, L = 32.
* ``c1``  1280x960, 3x3 array: 8 views at k*45 deg, r = 1 (axis) or sqrt(2)
  (diagonal), 20 objects (rectangles, rotated ellipses, slanted planes) with
  disparity in [0, 48], noise sigma 0.1, L_v = ceil(max(D) * r_v) + 2.
* ``c2``  3840x2160, 4x4 array with the reference camera at grid (1, 1):
  15 views at atan2(dy, dx), r = hypot(dx, dy); 40 layered occluders and
  100 thin structures with disparity up to 128, noise 0.1,
  L_v = min(400, ceil(max(D) * r_v) + 2).
* ``c3``  64 frames, sizes drawn from {640x480, 1280x960, 1920x1080,
  2048x1536}, c1 statistics with object sizes scaled by W / 1280.
* ``c4``  c1 statistics at 1920x1080 (evaluation frames of the learned
  tile proposal) and 256x256 training crops cut from 1280x960 frames.
* ``paper``  c1 statistics at 1600x1200 with 8 views: the shape of the
  paper's runtime experiment (Table 3), used as a context line only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "make_scene", "make_batch", "make_c1_like", "training_crops",
    "config_scan_len", "CONFIG_NAMES", "PARAMS_C0", "DEFAULT_PARAMS",
]

# Detector thresholds used by every workload (edge threshold gamma, disparity
# threshold beta, distance threshold zeta, number of neighbours N).
DEFAULT_PARAMS = dict(edge_thr=1.0, disp_thr=0.5, dist_thr=1.0, neighbours=1)
PARAMS_C0 = dict(DEFAULT_PARAMS)

CONFIG_NAMES = ("c0", "c1", "c2", "c3", "c4", "paper")

SQRT2_F32 = np.float32(math.sqrt(2.0))


@dataclass
class Scene:
    """One frame and its views."""
    name: str
    seed: int
    D: np.ndarray                 # float32 [H, W], C-contiguous
    angles: np.ndarray            # float64 [V], degrees
    ratios: np.ndarray            # float32 [V]
    scan_len: np.ndarray          # int32 [V]
    params: dict = field(default_factory=lambda: dict(DEFAULT_PARAMS))

    @property
    def H(self) -> int:
        return int(self.D.shape[0])

    @property
    def W(self) -> int:
        return int(self.D.shape[1])

    @property
    def n_views(self) -> int:
        return int(self.angles.shape[0])

    @property
    def pixel_views(self) -> int:
        return self.H * self.W * self.n_views


# ---------------------------------------------------------------------------
# scan length recipe of the workloads (a parameter choice, not the method):
# L_v = ceil(max(D) * r_v) + 2, product in fp32, optionally capped.
# ---------------------------------------------------------------------------
def config_scan_len(D: np.ndarray, ratios: np.ndarray, cap: int | None = None) -> np.ndarray:
    dmax = np.float32(D.max())
    out = []
    for r in np.asarray(ratios, dtype=np.float32):
        prod = np.float32(dmax * np.float32(r))
        L = int(math.ceil(float(prod))) + 2
        if cap is not None:
            L = min(cap, L)
        out.append(max(L, 1))
    return np.asarray(out, dtype=np.int32)


# ---------------------------------------------------------------------------
# painting primitives
# ---------------------------------------------------------------------------
def _background(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """Random linear gradient rising from exactly 1 to 4 across the frame."""
    theta = rng.uniform(0.0, 2.0 * math.pi)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    proj = x * math.cos(theta) + y * math.sin(theta)
    lo, hi = proj.min(), proj.max()
    if hi > lo:
        bg = 1.0 + 3.0 * (proj - lo) / (hi - lo)
    else:
        bg = np.ones_like(proj)
    return bg


def _paint_rect(D, cx, cy, w, h, value):
    H, W = D.shape
    x0 = int(round(cx - w / 2.0))
    y0 = int(round(cy - h / 2.0))
    xa, xb = max(0, x0), min(W, x0 + w)
    ya, yb = max(0, y0), min(H, y0 + h)
    if xa < xb and ya < yb:
        D[ya:yb, xa:xb] = value


def _paint_slanted(D, cx, cy, w, h, d0, gx, gy, dmax):
    H, W = D.shape
    x0 = int(round(cx - w / 2.0))
    y0 = int(round(cy - h / 2.0))
    xa, xb = max(0, x0), min(W, x0 + w)
    ya, yb = max(0, y0), min(H, y0 + h)
    if xa < xb and ya < yb:
        yy, xx = np.mgrid[ya:yb, xa:xb].astype(np.float64)
        D[ya:yb, xa:xb] = np.clip(d0 + gx * (xx - x0) + gy * (yy - y0), 0.0, dmax)


def _paint_ellipse(D, cx, cy, a, b, phi, value):
    H, W = D.shape
    R = max(a, b) + 1
    xa, xb = max(0, int(math.floor(cx - R))), min(W, int(math.ceil(cx + R)) + 1)
    ya, yb = max(0, int(math.floor(cy - R))), min(H, int(math.ceil(cy + R)) + 1)
    if xa >= xb or ya >= yb:
        return
    yy, xx = np.mgrid[ya:yb, xa:xb].astype(np.float64)
    dx, dy = xx - cx, yy - cy
    cp, sp = math.cos(phi), math.sin(phi)
    u = (dx * cp + dy * sp) / a
    v = (-dx * sp + dy * cp) / b
    inside = (u * u + v * v) <= 1.0
    sub = D[ya:yb, xa:xb]
    sub[inside] = value


def _paint_segment(D, x0, y0, x1, y1, width, value):
    H, W = D.shape
    pad = width / 2.0 + 1
    xa, xb = max(0, int(math.floor(min(x0, x1) - pad))), min(W, int(math.ceil(max(x0, x1) + pad)) + 1)
    ya, yb = max(0, int(math.floor(min(y0, y1) - pad))), min(H, int(math.ceil(max(y0, y1) + pad)) + 1)
    if xa >= xb or ya >= yb:
        return
    yy, xx = np.mgrid[ya:yb, xa:xb].astype(np.float64)
    vx, vy = x1 - x0, y1 - y0
    ll = vx * vx + vy * vy
    if ll == 0:
        t = np.zeros_like(xx)
    else:
        t = np.clip(((xx - x0) * vx + (yy - y0) * vy) / ll, 0.0, 1.0)
    px, py = x0 + t * vx, y0 + t * vy
    dist2 = (xx - px) ** 2 + (yy - py) ** 2
    inside = dist2 <= (width / 2.0) ** 2
    sub = D[ya:yb, xa:xb]
    sub[inside] = value


def _random_object(rng, W, H, scale, dmax, kind=None, centre=None, d0=None):
    """Draw one c1-statistics object; returns (sort_key, centre, painter)."""
    if kind is None:
        kind = int(rng.integers(0, 3))
    if centre is None:
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
    else:
        cx, cy = centre
    if d0 is None:
        d0 = rng.uniform(0.0, dmax)
    if kind == 0:
        w = int(round(rng.integers(32, 321) * scale))
        h = int(round(rng.integers(32, 321) * scale))
        return d0, (cx, cy), lambda D: _paint_rect(D, cx, cy, max(w, 1), max(h, 1), d0)
    if kind == 1:
        a = rng.integers(16, 161) * scale
        b = rng.integers(16, 161) * scale
        phi = rng.uniform(0.0, math.pi)
        return d0, (cx, cy), lambda D: _paint_ellipse(D, cx, cy, a, b, phi, d0)
    w = int(round(rng.integers(32, 321) * scale))
    h = int(round(rng.integers(32, 321) * scale))
    gx, gy = rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05)
    return d0, (cx, cy), lambda D: _paint_slanted(D, cx, cy, max(w, 1), max(h, 1), d0, gx, gy, dmax)


def _finish(D64: np.ndarray, rng, noise: float) -> np.ndarray:
    if noise > 0:
        D64 = D64 + rng.normal(0.0, noise, size=D64.shape)
    return np.ascontiguousarray(D64.astype(np.float32))


# ---------------------------------------------------------------------------
# views
# ---------------------------------------------------------------------------
def views_3x3():
    angles = np.arange(8, dtype=np.float64) * 45.0
    ratios = np.array([1.0 if k % 2 == 0 else SQRT2_F32 for k in range(8)], dtype=np.float32)
    return angles, ratios


def views_4x4():
    angles, ratios = [], []
    for dy in (-1, 0, 1, 2):
        for dx in (-1, 0, 1, 2):
            if dx == 0 and dy == 0:
                continue
            angles.append(math.degrees(math.atan2(dy, dx)))
            ratios.append(math.hypot(dx, dy))
    return np.asarray(angles, dtype=np.float64), np.asarray(ratios, dtype=np.float32)


# ---------------------------------------------------------------------------
# configs
# ---------------------------------------------------------------------------
def _c0(seed: int) -> Scene:
    rng = np.random.default_rng(seed)
    H, W = 192, 256
    D = _background(rng, H, W)
    objs = []
    for _ in range(4):
        w = int(rng.integers(16, 65))
        h = int(rng.integers(16, 65))
        x0 = int(rng.integers(0, W - w + 1))
        y0 = int(rng.integers(0, H - h + 1))
        d = rng.uniform(2.0, 24.0)
        objs.append((d, x0, y0, w, h))
    for d, x0, y0, w, h in sorted(objs, key=lambda o: o[0]):
        D[y0:y0 + h, x0:x0 + w] = d
    D32 = _finish(D, rng, 0.0)
    return Scene("c0", seed, D32, np.array([0.0]), np.array([1.0], dtype=np.float32),
                 np.array([32], dtype=np.int32), dict(PARAMS_C0))


def extent_scene(H: int, W: int, seed: int) -> Scene:
    """A thin frame at an extreme extent (for example 24 x 65535): a gentle
    ramp (no edges above gamma) with 400 constant rectangles of disparity
    8..40 and a band of disparity 30 along the far edge of the long side, so
    that candidates reach the largest coordinates; 8 views at 45 degree steps,
    ratios 1 / sqrt(2) alternating, L = 50 / 70."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    D = (4.0 + 0.01 * (xx % 97) + 0.01 * (yy % 89)).astype(np.float32)
    for _ in range(400):
        h, w = int(rng.integers(2, min(H, 40) + 1)), int(rng.integers(2, min(W, 40) + 1))
        y0, x0 = int(rng.integers(0, H - h + 1)), int(rng.integers(0, W - w + 1))
        D[y0:y0 + h, x0:x0 + w] = np.float32(rng.uniform(8.0, 40.0))
    if W >= H:
        D[:, -5:] = np.float32(30.0)
    if H >= W:
        D[-5:, :] = np.float32(30.0)
    angles = np.arange(8) * 45.0
    ratios = np.where(np.arange(8) % 2 == 1, np.float32(np.sqrt(2.0)), np.float32(1.0)).astype(np.float32)
    return Scene(f"extent{H}x{W}", seed, np.ascontiguousarray(D), angles, ratios,
                 np.array([50, 70] * 4, np.int32))


def make_c1_like(seed_or_rng, W: int = 1280, H: int = 960, n_objects: int = 20,
                 dmax: float = 48.0, noise: float = 0.1, name: str = "c1", seed: int = -1) -> Scene:
    """c1 statistics at any frame size (object sizes scale with W / 1280)."""
    rng = seed_or_rng if isinstance(seed_or_rng, np.random.Generator) else np.random.default_rng(seed_or_rng)
    if not isinstance(seed_or_rng, np.random.Generator):
        seed = int(seed_or_rng)
    scale = W / 1280.0
    D = _background(rng, H, W)
    objs = [_random_object(rng, W, H, scale, dmax) for _ in range(n_objects)]
    for _, _, paint in sorted(objs, key=lambda o: o[0]):
        paint(D)
    D32 = _finish(D, rng, noise)
    angles, ratios = views_3x3()
    return Scene(name, seed, D32, angles, ratios, config_scan_len(D32, ratios), dict(DEFAULT_PARAMS))


def _c2(seed: int) -> Scene:
    rng = np.random.default_rng(seed)
    H, W = 2160, 3840
    dmax = 128.0
    scale = W / 1280.0
    D = _background(rng, H, W)
    painters = []
    # 40 layered occluders: disparity rises layer by layer and every layer is
    # centred near its predecessor so that it overlaps it.
    layer_d = np.sort(rng.uniform(0.0, dmax, size=40))
    centre = (rng.uniform(0, W), rng.uniform(0, H))
    for k in range(40):
        d_k = float(layer_d[k])
        _, c, paint = _random_object(rng, W, H, scale, dmax, centre=centre, d0=d_k)
        painters.append((d_k, paint))
        step = 160.0 * scale
        centre = (float(np.clip(c[0] + rng.uniform(-step, step), 0, W)),
                  float(np.clip(c[1] + rng.uniform(-step, step), 0, H)))
    # 100 thin structures: 60 random segments and 40 vertical poles, 1-3 px wide
    for _ in range(60):
        x0, y0 = rng.uniform(0, W), rng.uniform(0, H)
        ang = rng.uniform(0, math.pi)
        ln = rng.uniform(100.0, 1500.0)
        x1, y1 = x0 + ln * math.cos(ang), y0 + ln * math.sin(ang)
        wd = int(rng.integers(1, 4))
        d = rng.uniform(0.0, dmax)
        painters.append((d, (lambda x0=x0, y0=y0, x1=x1, y1=y1, wd=wd, d=d:
                             (lambda DD: _paint_segment(DD, x0, y0, x1, y1, wd, d)))()))
    for _ in range(40):
        x0 = int(rng.integers(0, W))
        wd = int(rng.integers(1, 4))
        top = int(rng.integers(0, H))
        hgt = int(rng.integers(200, H + 1))
        d = rng.uniform(0.0, dmax)
        painters.append((d, (lambda x0=x0, wd=wd, top=top, hgt=hgt, d=d:
                             (lambda DD: DD.__setitem__((slice(top, min(H, top + hgt)), slice(x0, min(W, x0 + wd))), d)))()))
    for _, paint in sorted(painters, key=lambda p: p[0]):
        paint(D)
    D32 = _finish(D, rng, 0.1)
    angles, ratios = views_4x4()
    return Scene("c2", seed, D32, angles, ratios, config_scan_len(D32, ratios, cap=400), dict(DEFAULT_PARAMS))


C3_SIZES = ((640, 480), (1280, 960), (1920, 1080), (2048, 1536))


def make_batch(seed: int = 3000, n_frames: int = 64, sizes=C3_SIZES) -> list:
    """c3: frames of mixed size, c1 statistics, one generator for everything."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(sizes), size=n_frames)
    frames = []
    for k in range(n_frames):
        W, H = sizes[int(idx[k])]
        frames.append(make_c1_like(rng, W=W, H=H, name="c3", seed=seed * 1000 + k))
    return frames


def make_scene(cfg: str, seed: int) -> Scene:
    if cfg == "c0":
        return _c0(seed)
    if cfg == "c1":
        return make_c1_like(seed, 1280, 960, name="c1")
    if cfg == "c2":
        return _c2(seed)
    if cfg == "c4":
        return make_c1_like(seed, 1920, 1080, name="c4")
    if cfg == "paper":
        return make_c1_like(seed, 1600, 1200, name="paper")
    raise ValueError(f"unknown config {cfg!r} (c3 is a batch: use make_batch)")


def training_crops(seed: int, n_crops: int = 8, crop: int = 256, W: int = 1280, H: int = 960):
    """One c1-statistics frame plus n_crops random crop origins (y0, x0)."""
    rng = np.random.default_rng(seed)
    sc = make_c1_like(rng, W=W, H=H, name="c4-train", seed=seed)
    ys = rng.integers(0, H - crop + 1, size=n_crops)
    xs = rng.integers(0, W - crop + 1, size=n_crops)
    return sc, list(zip(ys.tolist(), xs.tolist()))


def fusion_maps(seed: int, D: np.ndarray, K: int = 8, noise: float = 0.3, outliers: float = 0.05,
                holes: float = 0.03) -> np.ndarray:
    """K noisy per-view disparity maps of a true centre map D (the input of the
    median fusion): Gaussian noise, a fraction of gross outliers (uniform over
    [0, 2 max D]) and a fraction of holes (NaN), independently per map."""
    rng = np.random.default_rng(seed)
    H, W = D.shape
    maps = np.repeat(D[None].astype(np.float32), K, axis=0)
    maps += rng.normal(0.0, noise, size=maps.shape).astype(np.float32)
    out = rng.uniform(size=maps.shape) < outliers
    maps[out] = rng.uniform(0.0, 2.0 * float(D.max()) + 1.0, size=int(out.sum())).astype(np.float32)
    maps[rng.uniform(size=maps.shape) < holes] = np.nan
    return np.ascontiguousarray(maps, dtype=np.float32)


# ---------------------------------------------------------------------------
# the limitation cases of Sec. 5, with every painted surface kept
# ---------------------------------------------------------------------------
@dataclass
class Layer:
    """One painted surface: its pixels in centre-view coordinates (they may
    lie outside the centre frame) and their disparities, including the parts
    that nearer surfaces hide in the centre view."""
    name: str
    x: np.ndarray   # int64
    y: np.ndarray   # int64
    d: np.ndarray   # float32


def _rect_layer(name, x0, x1, y0, y1, d) -> Layer:
    yy, xx = np.mgrid[y0:y1, x0:x1]
    return Layer(name, xx.ravel().astype(np.int64), yy.ravel().astype(np.int64),
                 np.full(xx.size, d, np.float32))


LIMITATION_CASES = ("occluded_occluder", "outside_border", "one_camera")


def limitation_scene(kind: str):
    """A small scene for one limitation of the method (Sec. 5) and the list
    of every surface painted into it.  The visible centre map D is what the
    painter's algorithm leaves in the frame (ascending disparity, nearer
    surfaces overwrite farther ones); surfaces outside the frame, and the
    hidden parts of overwritten ones, are in the layers only.

    Every scene is in the class where the method equals a forward-warping
    z-buffer of D exactly: integer fronto-parallel layers, views at 0 and
    180 degrees with r = 1, zeta = 1, beta = 0.5, N = 1 and
    L = 2 (max D - min D) + 4 (the layers outside D included).

    occluded_occluder  a plate (d 10) whose left four columns sit behind a
                       thin pole (d 30): in the right camera (0 degrees)
                       the hidden columns cover background that D cannot
                       explain.
    outside_border     an object (d 20) just right of the frame: in the
                       right camera it covers background inside the frame.
    one_camera         an object very close to the cameras (d 60), outside
                       the centre camera's frame and seen only by the right
                       camera.
    All three also hold an ordinary object inside the frame."""
    H, W = 96, 160
    bg = 2.0
    layers = [_rect_layer("background", -96, W + 96, -8, H + 8, bg)]
    if kind == "occluded_occluder":
        layers += [_rect_layer("object", 20, 40, 30, 60, 8.0),
                   _rect_layer("plate", 90, 130, 20, 70, 10.0),
                   _rect_layer("pole", 90, 94, 10, 80, 30.0)]
    elif kind == "outside_border":
        layers += [_rect_layer("object", 40, 70, 20, 50, 8.0),
                   _rect_layer("outside", W, W + 6, 30, 60, 20.0)]
    elif kind == "one_camera":
        layers += [_rect_layer("object", 40, 70, 20, 50, 8.0),
                   _rect_layer("near", W + 30, W + 40, 10, 50, 60.0)]
    else:
        raise ValueError(f"unknown limitation case {kind!r}")
    D = np.zeros((H, W), np.float32)
    for ly in sorted(layers, key=lambda l: float(l.d.max())):  # painter's algorithm
        inside = (ly.x >= 0) & (ly.x < W) & (ly.y >= 0) & (ly.y < H)
        D[ly.y[inside], ly.x[inside]] = ly.d[inside]
    dmax = max(float(l.d.max()) for l in layers)
    L = int(2 * (dmax - bg) + 4)
    params = dict(edge_thr=1.0, disp_thr=0.5, dist_thr=1.0, neighbours=1)
    sc = Scene(kind, 0, np.ascontiguousarray(D), np.array([0.0, 180.0]),
               np.array([1.0, 1.0], np.float32), np.array([L, L], np.int32), params)
    return sc, layers
