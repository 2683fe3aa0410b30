"""Seeded synthetic stereo pairs -- the only module shared by the HIP path's
tests and the oracle's tests.  It holds none of the method's arithmetic
(no census, cost, aggregation or disparity selection): it only draws images.

Recipe (stands in for the KITTI 2015 / VGA / Middlebury-Q pairs of the paper's
experiments, whose data is not used here; only their shapes are):

* left image: uniform noise U[0, 255], Gaussian-smoothed (sigma = 1 px),
  re-stretched to its original spread, plus a linear gradient of up to +-48
  grey levels across the frame, rounded and clipped to uint8;
* ground-truth left disparity: piecewise-planar over a Voronoi partition into
  K random planes d = a + b x + c y (a uniform in the disparity range,
  |b|, |c| <= 0.05), rounded and clipped to [0, D-1];
* right image: every left pixel is forward-warped to x - d; where several land
  on one pixel the larger disparity wins (a z-buffer); holes get fresh
  smoothed noise; optional blobs covering a fraction of the right image are
  replaced by noise; then Gaussian noise sigma = 2 is added, rounded, clipped;
* occlusion mask: left pixels that lose the z-test or land in a noise blob.

Every pair is a pure function of (width, height, ndisp, seed, options).
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

# The five workloads.  Seeds are 2106 + configuration index.
CONFIGS = {
    "c1_320x240_d64_r4": dict(width=320, height=240, ndisp=64, win_w=5, win_h=5,
                              npaths=4, p1=7, p2=86, lr_tolerance=-1, median3x3=False,
                              planes=(8, 8), occlusion=0.0, seed=2106),
    "c2_1242x375_d128_r8": dict(width=1242, height=375, ndisp=128, win_w=9, win_h=7,
                                npaths=8, p1=10, p2=120, lr_tolerance=1, median3x3=True,
                                planes=(8, 16), occlusion=0.05, seed=2107),
    "c3_1920x1080_d256_r8": dict(width=1920, height=1080, ndisp=256, win_w=9, win_h=7,
                                 npaths=8, p1=10, p2=120, lr_tolerance=1, median3x3=True,
                                 planes=(8, 16), occlusion=0.05, seed=2108),
}
BATCH_SIZES = ((320, 240), (640, 512), (1242, 375), (1920, 1080))
BATCH_NDISP = (64, 128, 256)
SERVE_SIZES = ((640, 512), (1242, 375), (1920, 1080))
SERVE_NDISP = (128, 256)


def _texture(rng: np.random.Generator, height: int, width: int) -> np.ndarray:
    noise = rng.uniform(0.0, 255.0, size=(height, width))
    smooth = gaussian_filter(noise, sigma=1.0, mode="reflect")
    spread = smooth.std()
    if spread > 0:
        smooth = (smooth - smooth.mean()) * (noise.std() / spread) * 0.6 + 127.5
    return smooth


def left_image(rng: np.random.Generator, width: int, height: int) -> np.ndarray:
    tex = _texture(rng, height, width)
    gx, gy = rng.uniform(-48.0, 48.0, size=2)
    xs = np.linspace(-0.5, 0.5, width)[None, :]
    ys = np.linspace(-0.5, 0.5, height)[:, None]
    img = tex + gx * xs + gy * ys
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def planar_disparity(rng: np.random.Generator, width: int, height: int,
                     ndisp: int, n_planes: int) -> np.ndarray:
    """Integer ground truth, piecewise planar over a Voronoi partition."""
    seeds = np.stack([rng.uniform(0, width, n_planes), rng.uniform(0, height, n_planes)], 1)
    a = rng.uniform(0, ndisp - 1, n_planes)
    b = rng.uniform(-0.05, 0.05, n_planes)
    c = rng.uniform(-0.05, 0.05, n_planes)
    ys, xs = np.mgrid[0:height, 0:width]
    best = np.full((height, width), np.inf)
    label = np.zeros((height, width), np.int64)
    for k in range(n_planes):
        dist = (xs - seeds[k, 0]) ** 2 + (ys - seeds[k, 1]) ** 2
        closer = dist < best
        best[closer] = dist[closer]
        label[closer] = k
    cx = xs - seeds[label, 0]
    cy = ys - seeds[label, 1]
    d = a[label] + b[label] * cx + c[label] * cy
    return np.clip(np.rint(d), 0, ndisp - 1).astype(np.int64)


def warp_right(rng: np.random.Generator, left: np.ndarray, disp: np.ndarray,
               occlusion: float = 0.0, noise_sigma: float = 2.0):
    """Forward warp with a z-buffer; returns (right uint8, occluded bool)."""
    height, width = left.shape
    ys, xs = np.mgrid[0:height, 0:width]
    xr = xs - disp
    valid = xr >= 0
    zbuf = np.full((height, width), -1, np.int64)
    np.maximum.at(zbuf, (ys[valid], xr[valid]), disp[valid])
    winner = np.zeros((height, width), bool)
    winner[valid] = disp[valid] == zbuf[ys[valid], xr[valid]]
    right = _texture(rng, height, width)            # hole fill
    right[ys[winner], xr[winner]] = left[winner]
    occluded = ~winner
    if occlusion > 0:
        blob = np.zeros((height, width), bool)
        target = occlusion * width * height
        covered = 0
        while covered < target:
            r = rng.uniform(3, max(4.0, 0.04 * min(width, height)))
            cx, cy = rng.uniform(0, width), rng.uniform(0, height)
            x0, x1 = max(0, int(cx - r)), min(width, int(cx + r) + 2)
            y0, y1 = max(0, int(cy - r)), min(height, int(cy + r) + 2)
            if x0 >= x1 or y0 >= y1:
                continue
            sub = blob[y0:y1, x0:x1]
            before = int(sub.sum())
            sub |= (xs[y0:y1, x0:x1] - cx) ** 2 + (ys[y0:y1, x0:x1] - cy) ** 2 <= r * r
            covered += int(sub.sum()) - before
        fill = _texture(rng, height, width)
        right[blob] = fill[blob]
        hit = np.zeros((height, width), bool)
        hit[winner] = blob[ys[winner], xr[winner]]
        occluded |= hit
    right = right + rng.normal(0.0, noise_sigma, size=right.shape)
    return np.clip(np.rint(right), 0, 255).astype(np.uint8), occluded


def make_pair(width: int, height: int, ndisp: int, seed: int,
              planes=(8, 16), occlusion: float = 0.0) -> dict:
    """A seeded synthetic pair with its integer ground truth."""
    rng = np.random.Generator(np.random.PCG64(seed))
    left = left_image(rng, width, height)
    n_planes = int(rng.integers(planes[0], planes[1] + 1))
    disp = planar_disparity(rng, width, height, ndisp, n_planes)
    right, occluded = warp_right(rng, left, disp, occlusion)
    return {"left": left, "right": right, "disp_gt": disp.astype(np.uint16),
            "occluded": occluded}


def pure_shift_pair(width: int, height: int, d0: int, seed: int) -> dict:
    """R(x, y) = L(x + d0, y), fresh noise where x + d0 >= W."""
    rng = np.random.Generator(np.random.PCG64(seed))
    left = left_image(rng, width, height)
    right = np.empty_like(left)
    if d0 < width:
        right[:, : width - d0] = left[:, d0:]
    fill = left_image(rng, width, height)
    right[:, max(0, width - d0):] = fill[:, max(0, width - d0):]
    return {"left": left, "right": right}


def config_pair(name: str) -> dict:
    cfg = CONFIGS[name]
    return make_pair(cfg["width"], cfg["height"], cfg["ndisp"], cfg["seed"],
                     cfg["planes"], cfg["occlusion"])


def random_images(width: int, height: int, seed: int):
    """Two unrelated noise images (edge-case tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.integers(0, 256, (height, width), dtype=np.uint8),
            rng.integers(0, 256, (height, width), dtype=np.uint8))


def random_cost(width: int, height: int, ndisp: int, seed: int, high: int = 64):
    """Uniform random uint8 cost volume (aggregation edge cases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, high, (height, width, ndisp), dtype=np.uint8)


def batch_specs(n: int = 64, seed: int = 2109):
    """(width, height, ndisp, seed) of the mixed batch workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(n):
        w, h = BATCH_SIZES[int(rng.integers(0, len(BATCH_SIZES)))]
        nd = BATCH_NDISP[int(rng.integers(0, len(BATCH_NDISP)))]
        specs.append((w, h, nd, seed * 1000 + i))
    return specs


def stream_specs(n_streams: int = 16, seed: int = 2110):
    """(width, height, ndisp, seed) of each simulated camera stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(n_streams):
        w, h = SERVE_SIZES[int(rng.integers(0, len(SERVE_SIZES)))]
        nd = SERVE_NDISP[int(rng.integers(0, len(SERVE_NDISP)))]
        specs.append((w, h, nd, seed * 1000 + i))
    return specs


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process on [0, duration)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.asarray(out)
        out.append(t)
