"""Seeded synthetic frames (numpy PCG64 via ``default_rng``).

The paper measures on a 256x256 Lena image and on N x N test images up to
4000 x 4000 (Sec. 3, Fig. 5); neither is available, so these seeded frames
stand in for them: grayscale content in [0, ~1.05] that fills the inscribed
disk, at the workload sizes.

Draw order for one frame (all from one ``numpy.random.default_rng(seed)``):
  1. for each blob: u, v, sigma fraction, amplitude          (4 uniform draws)
  2. for each polygon: vertex count k in {3..8}, u, v, scale fraction,
     k angles, k radius fractions, intensity
  3. if noise: an H x W array of U[0, noise_max) draws
Geometry: disk radius Rpx = D/2 (D = min(H, W)) around the frame centre
((W-1)/2, (H-1)/2) in pixel-centre coordinates.  Blob / polygon centres are
area-uniform in the disk (radius Rpx*sqrt(u), angle 2 pi v).
  * blob: a * exp(-d^2 / (2 sigma^2)), sigma = U[0.02, 0.2] * Rpx, added at
    pixel centres in FP64 (evaluated as the separable outer product of the
    x and y factors, which is the same function).
  * polygon: star-shaped (sorted angles, radii s * U[0.5, 1], s = U[0.05, 0.3]
    * Rpx); pixel centres inside by the even-odd rule are SET to the
    intensity U[0, 1]; painted in draw order over the blobs.
  * noise: U[0, 0.05] added per pixel.
  * zero_outside: pixels whose centre has rho > 1 are set to 0.
The frame is finally cast to the requested dtype.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class FrameSpec:
    H: int
    W: int
    blobs: int = 8
    polygons: int = 0
    noise: bool = True
    zero_outside: bool = True
    dtype: str = "float32"


def _disk_point(rng, rpx):
    u, v = rng.random(), rng.random()
    rad = rpx * np.sqrt(u)
    phi = 2.0 * np.pi * v
    return rad * np.cos(phi), rad * np.sin(phi)


def _inside_polygon(px, py, vx, vy):
    """Even-odd rule for points (px, py) against the closed polygon (vx, vy)."""
    inside = np.zeros(px.shape, dtype=bool)
    k = len(vx)
    for e in range(k):
        x1, y1 = vx[e], vy[e]
        x2, y2 = vx[(e + 1) % k], vy[(e + 1) % k]
        cond = (y1 > py) != (y2 > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = x1 + (py - y1) * (x2 - x1) / (y2 - y1)
        inside ^= cond & (px < xint)
    return inside


def make_frame(spec: FrameSpec, seed: int) -> np.ndarray:
    """Draw one H x W frame; see the module docstring for the recipe."""
    H, W = spec.H, spec.W
    D = min(H, W)
    rpx = 0.5 * D
    cx, cy = 0.5 * (W - 1), 0.5 * (H - 1)
    rng = np.random.default_rng(seed)
    f = np.zeros((H, W), dtype=np.float64)
    # x to the right, y up: pixel (i, j) has offsets (j - cx, cy - i)
    xs = np.arange(W, dtype=np.float64) - cx
    ys = cy - np.arange(H, dtype=np.float64)
    for _ in range(spec.blobs):
        bx, by = _disk_point(rng, rpx)
        sig = rpx * (0.02 + 0.18 * rng.random())
        amp = rng.random()
        gx = np.exp(-((xs - bx) ** 2) / (2.0 * sig * sig))
        gy = np.exp(-((ys - by) ** 2) / (2.0 * sig * sig))
        f += amp * np.outer(gy, gx)
    for _ in range(spec.polygons):
        k = int(rng.integers(3, 9))
        px0, py0 = _disk_point(rng, rpx)
        s = rpx * (0.05 + 0.25 * rng.random())
        ang = np.sort(rng.random(k) * 2.0 * np.pi)
        rad = s * (0.5 + 0.5 * rng.random(k))
        inten = rng.random()
        vx = px0 + rad * np.cos(ang)
        vy = py0 + rad * np.sin(ang)
        j0 = max(0, int(np.floor(cx + vx.min())) - 1)
        j1 = min(W, int(np.ceil(cx + vx.max())) + 2)
        i0 = max(0, int(np.floor(cy - vy.max())) - 1)
        i1 = min(H, int(np.ceil(cy - vy.min())) + 2)
        if j0 >= j1 or i0 >= i1:
            continue
        gx, gy = np.meshgrid(xs[j0:j1], ys[i0:i1])
        m = _inside_polygon(gx, gy, vx, vy)
        sub = f[i0:i1, j0:j1]
        sub[m] = inten
    if spec.noise:
        f += 0.05 * rng.random((H, W))
    if spec.zero_outside:
        X = 2.0 * np.arange(W) - (W - 1)
        Y = (H - 1) - 2.0 * np.arange(H)
        out = (X[None, :] ** 2 + Y[:, None] ** 2) > float(D) * D
        f[out] = 0.0
    return f.astype(spec.dtype)


# The five workloads the library is measured on (sizes, seeds, content).
CONFIGS = {
    1: dict(spec=FrameSpec(64, 64, blobs=8, polygons=0, noise=True, zero_outside=True, dtype="float64"),
            nmax=20, rings=32, angles=128, seed=1),
    2: dict(spec=FrameSpec(1024, 1024, blobs=8, polygons=0, noise=True, zero_outside=True),
            nmax=100, rings=512, angles=1024, seed=2),
    3: dict(spec=FrameSpec(2160, 3840, blobs=32, polygons=16, noise=False, zero_outside=False),
            nmax=200, rings=1080, angles=4096, seed=3),
}


def config_frame(cfg: int, seed: int | None = None) -> np.ndarray:
    c = CONFIGS[cfg]
    return make_frame(c["spec"], c["seed"] if seed is None else seed)


BATCH_SIDES = (256, 384, 512, 768, 1024, 1536, 2048)
BATCH_NMAX = (30, 50, 100)


def batch_sides(count: int = 64, seed: int = 4):
    """Mixed-size batch: (side, nmax, frame seed) per image, sides and N_max uniform."""
    rng = np.random.default_rng(seed)
    sides = rng.choice(BATCH_SIDES, size=count)
    nmaxs = rng.choice(BATCH_NMAX, size=count)
    return [(int(s), int(n), 1000 + i) for i, (s, n) in enumerate(zip(sides, nmaxs))]


SERVE_SIZES = ((480, 640, 0.50), (1080, 1920, 0.35), (2160, 3840, 0.15))
SERVE_NMAX = (30, 100, 200)


def request_stream(count: int, qps: float, seed: int = 5):
    """Poisson arrivals at rate qps: list of (t_arrival_s, H, W, nmax, frame seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps)
    probs = np.array([p for _, _, p in SERVE_SIZES])
    kinds = rng.choice(len(SERVE_SIZES), size=count, p=probs)
    nm = rng.choice(SERVE_NMAX, size=count)
    out = []
    for i in range(count):
        H, W, _ = SERVE_SIZES[kinds[i]]
        out.append((float(t[i]), H, W, int(nm[i]), 5000 + i))
    return out


def dedup_set(side: int, n_distinct: int = 5, seed: int = 31):
    """A synthetic image set with planted duplicates (stands in for a computer
    vision dataset with repeated images, Sec. 2.7).  Original k (seed + k,
    blob + polygon content, zero outside the disk) is followed by its planted
    variants, each an exact pixel permutation of the original that keeps the
    content: a copy, a quarter turn, a half turn and a left-right mirror for
    even k; a copy only for odd k.  One more frame is original 0 shifted by
    one pixel (different content at the pixel level: must not be grouped).
    Returns (frames, groups): groups lists the indices of each original and
    its variants, in order."""
    frames, groups = [], []
    spec = FrameSpec(side, side, blobs=6, polygons=3, noise=False, zero_outside=True)
    for k in range(n_distinct):
        f = make_frame(spec, seed + k)
        members = [len(frames)]
        frames.append(f)
        variants = [f.copy(), np.rot90(f, 1), np.rot90(f, 2), f[:, ::-1]] if k % 2 == 0 else [f.copy()]
        for v in variants:
            members.append(len(frames))
            frames.append(np.ascontiguousarray(v))
        groups.append(members)
    shifted = np.roll(frames[0], 1, axis=1)
    frames.append(np.ascontiguousarray(shifted))
    return frames, groups
