"""Seeded synthetic stereo pairs shaped like the paper's surgical data.

The paper evaluates on a Unity3D colon phantom and on in-vivo videos
(Section 3, first paragraph), neither of which is available here.  This
module stands in for them with rectified 8-bit grayscale pairs that carry the
two failure modes the paper designs against (Section 1, fourth paragraph):
weakly textured regions and non-Lambertian specular highlights, plus a smooth
photometric gain.  It holds none of the stereo method's arithmetic: it only
draws images, a ground-truth disparity and its validity.

Conventions: disparity d >= 0 means left pixel x is seen at right pixel x - d.
Every random draw comes from one numpy PCG64 stream in a fixed order, so a
seed fixes the pair bit for bit.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.ndimage import gaussian_filter

__all__ = ["StereoPair", "make_pair", "integer_shift_pair", "misaligned_pair", "random_pair_tiny"]


@dataclass
class StereoPair:
    left: np.ndarray       # uint8 (H, W)
    right: np.ndarray      # uint8 (H, W)
    disp: np.ndarray       # float32 (H, W), ground truth on the left grid
    valid: np.ndarray      # bool (H, W), left pixel visible in the right image
    seed: int
    d_max: float


def _bumps(rng, W, H, n, wlo, whi, alo, ahi):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    out = np.zeros((H, W))
    for _ in range(n):
        cx = rng.uniform(0, W)
        cy = rng.uniform(0, H)
        w = rng.uniform(wlo, whi)
        a = rng.uniform(alo, ahi)
        out += a * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2.0 * w * w))
    return out


def _minmax(a):
    lo, hi = a.min(), a.max()
    if hi - lo <= 0:
        return np.zeros_like(a)
    return (a - lo) / (hi - lo)


def _keys_cubic_rows(img, xs):
    """Keys cubic convolution (a = -0.5) along each row at columns xs (H, W'),
    replicate border.  A different interpolant from the method's linear one,
    so the generated pair carries no interpolation bias toward the method."""
    H, W = img.shape
    x0 = np.floor(xs).astype(np.int64)
    t = xs - x0
    a = -0.5

    def k(s):
        s = np.abs(s)
        return np.where(
            s <= 1, (a + 2) * s**3 - (a + 3) * s**2 + 1,
            np.where(s < 2, a * s**3 - 5 * a * s**2 + 8 * a * s - 4 * a, 0.0))

    rows = np.arange(H)[:, None]
    out = np.zeros_like(xs)
    for o in (-1, 0, 1, 2):
        idx = np.clip(x0 + o, 0, W - 1)
        out += k(t - o) * img[rows, idx]
    return out


def _lin_rows(f, xs):
    H, W = f.shape
    xs = np.clip(xs, 0, W - 1)
    m = np.minimum(np.floor(xs).astype(np.int64), W - 2)
    t = xs - m
    rows = np.arange(H)[:, None]
    return (1 - t) * f[rows, m] + t * f[rows, m + 1]


def make_pair(W: int, H: int, d_max: float, seed: int, *, low_contrast=True,
              gain=True, specular=True, noise=True) -> StereoPair:
    """One synthetic rectified pair (W x H) with disparity in [0, d_max].

    Recipe, in draw order:
      1. texture: uniform noise blurred with a sigma-2 Gaussian;
      2. low contrast: the 30 % of pixels where a smooth random field is lowest
         get their contrast cut to a tenth (weak texture);
      3. disparity: four random 2-D Gaussians min-max mapped to [0, d_max],
         redrawn until the horizontal slope stays below 0.5 (no occlusion);
      4. warp: each right pixel x' takes the left value at x = x' + D(x)
         (30 fixed-point steps), sampled with Keys cubic interpolation;
      5. gain: the right image times a smooth field in [0.8, 1.2];
      6. specular: five Gaussian blobs added to the right image, saturating
         at 255 in their cores;
      7. sensor noise N(0, 2^2) on the right; both images rounded half to
         even and clipped to uint8.
    The flags switch off steps 2, 5, 6 and 7 for the "diffuse" variant.
    """
    if W < 4 or H < 4:
        raise ValueError("image too small")
    rng = np.random.Generator(np.random.PCG64(seed))
    base = gaussian_filter(rng.uniform(0.0, 255.0, (H, W)), sigma=2.0,
                           mode="mirror", truncate=4.0)
    lf = base.copy()
    field = gaussian_filter(rng.uniform(0.0, 1.0, (H, W)), sigma=W / 16.0,
                            mode="mirror", truncate=4.0)
    if low_contrast:
        k = int(round(0.3 * H * W))
        thr = np.sort(field.ravel())[k - 1]
        mask = field <= thr
        mu = base.mean()
        lf[mask] = mu + 0.1 * (base[mask] - mu)

    D = None
    for _ in range(100):
        cand = _minmax(_bumps(rng, W, H, 4, W / 8.0, W / 4.0, 0.5, 1.0)) * d_max
        if W < 2 or np.abs(np.diff(cand, axis=1)).max() < 0.5:
            D = cand
            break
    if D is None:
        raise RuntimeError("no disparity field with slope < 0.5 in 100 draws")

    xp = np.broadcast_to(np.arange(W, dtype=np.float64), (H, W))
    x = xp.copy()
    for _ in range(30):
        x = xp + _lin_rows(D, x)
    rf = _keys_cubic_rows(lf, x)

    g = _minmax(_bumps(rng, W, H, 3, W / 4.0, W / 2.0, 0.5, 1.0))
    if gain:
        rf = rf * (0.8 + 0.4 * g)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    for _ in range(5):
        cx = rng.uniform(0, W)
        cy = rng.uniform(0, H)
        r = rng.uniform(W / 64.0, W / 32.0)
        if specular:
            rf = rf + 1.5 * 255.0 * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * r * r))
    nz = rng.normal(0.0, 2.0, (H, W))
    if noise:
        rf = rf + nz
    left = np.clip(np.rint(lf), 0, 255).astype(np.uint8)
    right = np.clip(np.rint(rf), 0, 255).astype(np.uint8)
    valid = (np.arange(W)[None, :] - D) >= 0
    return StereoPair(left, right, D.astype(np.float32), valid, seed, float(d_max))


def integer_shift_pair(W: int, H: int, s: int, seed: int) -> StereoPair:
    """Right image = left image shifted by an integer s (R(x') = L(x' + s),
    replicate border): no low contrast, gain, highlights or noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = gaussian_filter(rng.uniform(0.0, 255.0, (H, W)), sigma=2.0,
                           mode="mirror", truncate=4.0)
    left = np.clip(np.rint(base), 0, 255).astype(np.uint8)
    idx = np.clip(np.arange(W) + s, 0, W - 1)
    right = left[:, idx].copy()
    disp = np.full((H, W), float(s), np.float32)
    valid = (np.arange(W)[None, :] - s) >= 0
    valid = np.broadcast_to(valid, (H, W)).copy()
    return StereoPair(left, right, disp, valid, seed, float(s))


def misaligned_pair(W: int, H: int, d_max: float, seed: int, v_max: float = 1.5):
    """make_pair(W, H, d_max, seed) with an imperfect rectification: the
    right image moved vertically by vf(x') = a + b (x' / (W - 1) - 1/2), a
    small roll of the right camera, with a and b drawn uniformly from
    [-v_max / 2, v_max / 2] (|vf| <= 3/4 v_max) from the stream PCG64([seed,
    1]), and resampled with Keys bicubic interpolation.  Left (x, y) then
    matches right (x - d, y + v) with v = vf(x - d).  Returns (pair, v) with
    pair.right replaced and v the float32 vertical ground truth on the left
    grid."""
    pair = make_pair(W, H, d_max, seed)
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    a, b = (float(t) for t in rng.uniform(-0.5 * v_max, 0.5 * v_max, 2))
    xs = np.arange(W, dtype=np.float64)
    vf = a + b * (xs / max(W - 1, 1) - 0.5)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    right = _keys_cubic_2d(pair.right.astype(np.float64), xx, yy - vf[None, :])
    pair.right = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    v = (a + b * ((xx - pair.disp) / max(W - 1, 1) - 0.5)).astype(np.float32)
    return pair, v


def random_pair_tiny(W: int, H: int, seed: int, lo=0, hi=256) -> tuple[np.ndarray, np.ndarray]:
    """Two independent uniform uint8 images (edge-case inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.integers(lo, hi, (H, W), dtype=np.uint8)
    b = rng.integers(lo, hi, (H, W), dtype=np.uint8)
    return a, b


def _make_one(args):
    W, H, d, s = args[:4]
    return make_pair(W, H, d, s, **(args[4] if len(args) > 4 else {}))


def make_pairs(spec, workers: int = 0):
    """make_pair for each (W, H, d_max, seed[, flags]) of spec, in order, on a
    pool of worker processes (0 = one per CPU, at most 16); flags is a dict of
    make_pair's keyword switches.  Call it before the GPU is touched in this
    process: workers are forked."""
    import multiprocessing as mp
    import os
    spec = list(spec)
    n = workers or min(16, os.cpu_count() or 1, max(1, len(spec)))
    if n <= 1 or len(spec) <= 1:
        return [_make_one(a) for a in spec]
    with mp.get_context("fork").Pool(n) as pool:
        return pool.map(_make_one, spec, chunksize=1)


def mixed_batch_spec(seed0: int = 3000):
    """64 pairs of mixed sizes: 24 at 320x240, 24 at 640x480, 16 at 1280x720,
    disparity up to 10 % of the width, seeds seed0, seed0 + 1, ..."""
    spec = []
    for (W, H, n) in ((320, 240, 24), (640, 480, 24), (1280, 720, 16)):
        for _ in range(n):
            spec.append((W, H, 0.1 * W, seed0 + len(spec)))
    return spec


def stereo_rig(W: int, H: int, seed: int, baseline: float = 5.0) -> dict:
    """Seeded synthetic calibration of a stereo endoscope of W x H images (the
    calibration of the paper's rigs is not available): per camera a focal
    length of 0.8-1.0 W px, a principal point within 2 % of the centre,
    barrel distortion (k1 in [-0.25, -0.1], k2 in [0, 0.05]), tangential
    terms below 1e-3, and a rectifying rotation of up to 1 degree about each
    axis; both rectified cameras share a focal length and principal point.
    Returns {"left": {...}, "right": {...}, "focal": f, "baseline": B} with
    each camera's fields named as in bdis_camera.  Draw order fixed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nf = float(rng.uniform(0.8, 1.0) * W)
    ncx, ncy = (W - 1) / 2.0, (H - 1) / 2.0
    cams = {}
    for side in ("left", "right"):
        f = float(rng.uniform(0.8, 1.0) * W)
        cx = (W - 1) / 2.0 + float(rng.uniform(-0.02, 0.02) * W)
        cy = (H - 1) / 2.0 + float(rng.uniform(-0.02, 0.02) * H)
        k1, k2 = float(rng.uniform(-0.25, -0.1)), float(rng.uniform(0.0, 0.05))
        p1, p2 = (float(v) for v in rng.uniform(-1e-3, 1e-3, 2))
        a, b, c = (float(v) for v in np.deg2rad(rng.uniform(-1.0, 1.0, 3)))
        rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
        ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
        rx = np.array([[1, 0, 0], [0, np.cos(c), -np.sin(c)], [0, np.sin(c), np.cos(c)]])
        R = rz @ ry @ rx
        cams[side] = dict(fx=f, fy=f, cx=cx, cy=cy, k1=k1, k2=k2, p1=p1, p2=p2, k3=0.0,
                          R=tuple(float(v) for v in R.ravel()), nfx=nf, nfy=nf, ncx=ncx, ncy=ncy)
    return {"left": cams["left"], "right": cams["right"], "focal": nf, "baseline": float(baseline)}


def _keys_cubic_2d(img: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Keys (a = -0.5) bicubic reading of img at (xs, ys), border replicated."""
    H, W = img.shape

    def k(s):
        s = np.abs(s)
        return np.where(s <= 1, (1.5 * s - 2.5) * s * s + 1,
                        np.where(s < 2, ((-0.5 * s + 2.5) * s - 4) * s + 2, 0.0))

    x0, y0 = np.floor(xs).astype(np.int64), np.floor(ys).astype(np.int64)
    out = np.zeros(xs.shape)
    for j in range(-1, 3):
        wy = k(ys - (y0 + j))
        yy = np.clip(y0 + j, 0, H - 1)
        for i in range(-1, 3):
            xx = np.clip(x0 + i, 0, W - 1)
            out += wy * k(xs - (x0 + i)) * img[yy, xx]
    return out


def raw_capture(rect: np.ndarray, cam: dict, iters: int = 20) -> np.ndarray:
    """The raw (distorted, unrectified) uint8 image a camera with calibration
    `cam` (fields as in bdis_camera) would record of the rectified image
    `rect`: for each raw pixel, its undistorted ray (fixed-point inversion of
    the lens model, `iters` steps), rotated into the rectified frame and read
    from `rect` with Keys bicubic interpolation (not the bilinear reading of
    the rectification itself).  Rays that leave `rect` give 0.  Input
    generation only: it lets a rectification be checked against the image it
    should recover."""
    H, W = rect.shape
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    xd = (x - cam["cx"]) / cam["fx"]
    yd = (y - cam["cy"]) / cam["fy"]
    xu, yu = xd.copy(), yd.copy()
    for _ in range(iters):
        r2 = xu * xu + yu * yu
        radial = 1 + cam["k1"] * r2 + cam["k2"] * r2 * r2 + cam["k3"] * r2 ** 3
        dx = 2 * cam["p1"] * xu * yu + cam["p2"] * (r2 + 2 * xu * xu)
        dy = cam["p1"] * (r2 + 2 * yu * yu) + 2 * cam["p2"] * xu * yu
        xu, yu = (xd - dx) / radial, (yd - dy) / radial
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    X = R[0, 0] * xu + R[0, 1] * yu + R[0, 2]
    Y = R[1, 0] * xu + R[1, 1] * yu + R[1, 2]
    Z = R[2, 0] * xu + R[2, 1] * yu + R[2, 2]
    u = cam["nfx"] * X / Z + cam["ncx"]
    v = cam["nfy"] * Y / Z + cam["ncy"]
    val = _keys_cubic_2d(rect.astype(np.float64), u, v)
    inside = (u >= 0) & (v >= 0) & (u <= W - 1) & (v <= H - 1)
    return np.where(inside, np.clip(np.rint(val), 0, 255), 0).astype(np.uint8)
