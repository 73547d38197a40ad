"""Seeded generators for the five synthetic workloads and for random test problems.

The paper's own data (high-resolution photographs with user seeds, an MRI volume with CNN unaries, an ink
drawing for the curvature experiment) is not available, so these generators stand in for it with the same
structure: Gaussian log-likelihood-ratio unaries (Eq. 2), contrast-sensitive or constant Potts weights
(Sec. 1, the Potts paragraph), 2D 4/8-connected and 3D 6-connected grids (the "kernel size 3" square /
spherical neighbourhoods of the experimental setup), and a non-submodular grid with repulsive edges
(the submodularity footnote of Sec. 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# ADMM schedule defaults in input-energy units (weights and unaries are x1000 integers).  The paper's
# mu0 = 100 (2D) / 500 (3D) are in unstated units; with x1000 inputs the oracle's sweep (oracle/sweep_mu.py,
# results in oracle/mu_sweep.json) picks these: in 2D mu0 = 1000 stops the 512x512 image after 2 iterations with
# no energy gap; in 3D no mu0 meets the stopping rule within 50 iterations on the 128x128x64 volume, and mu0 = 5000
# keeps its gap to the global cut at 0.27 % (1500 reaches 0.05 % but leaves twice as many nodes to the block
# max-flows: 7.4 instead of 4.2 ms per solve on MI355X; 15000 and above lose 4 %).
DEFAULT_MU0_2D = 1000
DEFAULT_MU0_3D = 5000
BALL_MU0 = 5000
DEFAULT_EPS_Q16 = 6554  # eps = 0.1 in Q16.16
DEFAULT_MAX_ITER = 50


def half_stencil(ndim: int, conn: int) -> List[Tuple[int, int, int]]:
    """Half-stencil offsets (dx, dy, dz); the full stencil is these and their negations."""
    if ndim == 2 and conn == 4:
        return [(1, 0, 0), (0, 1, 0)]
    if ndim == 2 and conn == 8:
        return [(1, 0, 0), (0, 1, 0), (1, 1, 0), (-1, 1, 0)]
    if ndim == 2 and conn in (24, 48, 80):   # 5x5, 7x7, 9x9 squares: (dx, 0) for dx = 1..r, then rows dy = 1..r
        r = {24: 2, 48: 3, 80: 4}[conn]
        out = [(dx, 0, 0) for dx in range(1, r + 1)]
        for dy in range(1, r + 1):
            for dx in range(-r, r + 1):
                out.append((dx, dy, 0))
        return out
    if ndim == 3 and conn == 6:
        return [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    if ndim == 3 and conn in (32, 122, 256):   # balls of radius 2 / 3 / 4; first nonzero coordinate (z, y, x) positive
        r = {32: 2, 122: 3, 256: 4}[conn]
        out = []
        for dz in range(0, r + 1):
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    if dx * dx + dy * dy + dz * dz > r * r or (dx, dy, dz) == (0, 0, 0):
                        continue
                    if dz > 0 or (dz == 0 and dy > 0) or (dz == 0 and dy == 0 and dx > 0):
                        out.append((dx, dy, dz))
        return out
    raise ValueError(f"unsupported stencil ndim={ndim} conn={conn}")


def lambda_q8(lam: float) -> int:
    """lambda quantised to 1/256, rounded half away from zero."""
    v = abs(lam) * 256.0
    q = int(math.floor(v + 0.5))
    return q if lam >= 0 else -q


def _round(x: np.ndarray) -> np.ndarray:
    return np.floor(x + 0.5)


@dataclasses.dataclass
class Problem:
    name: str
    dims: Tuple[int, int, int]          # (W, H, D); D = 1 in 2D
    ndim: int
    conn: int
    u: np.ndarray                       # int32[n]
    w: np.ndarray                       # int32[h, n]
    lam_q8: int
    block: Tuple[int, int, int]
    overlap: Tuple[int, int, int]
    mu0: int
    mu_num: int = 21
    mu_den: int = 20
    eps_q16: int = DEFAULT_EPS_Q16
    max_iter: int = DEFAULT_MAX_ITER
    solver: str = "maxflow"             # "maxflow" | "exhaustive"
    truth: Optional[np.ndarray] = None  # generating foreground mask (for reporting only)

    @property
    def n(self) -> int:
        return int(self.dims[0] * self.dims[1] * self.dims[2])

    def offsets(self):
        return half_stencil(self.ndim, self.conn)


def _weights_from_features(feat: np.ndarray, ndim: int, conn: int, sigma_w: float,
                           scale: float = 1000.0) -> np.ndarray:
    """Contrast-sensitive weights w = round(scale * exp(-|dx|^2 / (2 sigma^2)) / d) on the half-stencil.

    feat has shape (D, H, W, C).  d is the Euclidean length of the offset."""
    D, H, W, _ = feat.shape
    offs = half_stencil(ndim, conn)
    n = W * H * D
    out = np.zeros((len(offs), n), dtype=np.int64)
    for o, (dx, dy, dz) in enumerate(offs):
        wv = np.zeros((D, H, W), dtype=np.float64)
        z0, z1 = max(0, -dz), D - max(0, dz)
        y0, y1 = max(0, -dy), H - max(0, dy)
        x0, x1 = max(0, -dx), W - max(0, dx)
        a = feat[z0:z1, y0:y1, x0:x1]
        b = feat[z0 + dz:z1 + dz, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
        d2 = np.sum((a - b) ** 2, axis=-1)
        dist = math.sqrt(dx * dx + dy * dy + dz * dz)
        wv[z0:z1, y0:y1, x0:x1] = _round(scale * np.exp(-d2 / (2.0 * sigma_w ** 2)) / dist)
        out[o] = wv.reshape(-1)
    return out.astype(np.int32)


def _constant_weights(dims, ndim, conn, value) -> np.ndarray:
    W, H, D = dims
    offs = half_stencil(ndim, conn)
    out = np.zeros((len(offs), W * H * D), dtype=np.int32)
    zz, yy, xx = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    for o, (dx, dy, dz) in enumerate(offs):
        ok = ((xx + dx >= 0) & (xx + dx < W) & (yy + dy >= 0) & (yy + dy < H)
              & (zz + dz >= 0) & (zz + dz < D))
        out[o] = np.where(ok.reshape(-1), value, 0)
    return out


def _gauss_llr(img: np.ndarray, mu_fg: float, mu_bg: float, sigma: float, channels: bool = False) -> np.ndarray:
    """u = 1000 * (log p(bg|x) - log p(fg|x)) for equal-variance Gaussians (summed over a last channel axis)."""
    llr = ((img - mu_fg) ** 2 - (img - mu_bg) ** 2) / (2.0 * sigma ** 2)
    if channels:
        llr = llr.sum(axis=-1)
    return _round(1000.0 * llr).reshape(-1).astype(np.int64)


def config1(seed: int = 0, size: int = 64, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """64x64 grey disk (r = 20) + N(0, 0.15^2); 4-connected contrast Potts; lambda = 1; 16x16 blocks, o = 1."""
    rng = np.random.default_rng(seed)
    c = size / 2.0
    r = 20.0 * size / 64.0
    yy, xx = np.mgrid[0:size, 0:size]
    fg = (xx - c) ** 2 + (yy - c) ** 2 <= r * r
    img = np.where(fg, 0.7, 0.3) + rng.normal(0.0, 0.15, size=(size, size))
    u = _gauss_llr(img, 0.7, 0.3, 0.15)
    w = _weights_from_features(img[None, :, :, None], 2, 4, 0.1)
    return Problem("config1_disk64_4conn", (size, size, 1), 2, 4, u.astype(np.int32), w,
                   lambda_q8(1.0), (16, 16, 1), (1, 1, 0), mu0, max_iter=50,
                   truth=fg.reshape(-1).astype(np.uint8))


def _ellipse_mask(rng, W, H, count):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    fg = np.zeros((H, W), dtype=bool)
    for _ in range(count):
        cx, cy = rng.uniform(0.0, W), rng.uniform(0.0, H)
        a, b = rng.uniform(20.0, 120.0), rng.uniform(20.0, 120.0)
        th = rng.uniform(0.0, math.pi)
        dx, dy = xx - cx, yy - cy
        xr = dx * math.cos(th) + dy * math.sin(th)
        yr = -dx * math.sin(th) + dy * math.cos(th)
        fg |= (xr / a) ** 2 + (yr / b) ** 2 <= 1.0
    return fg


def config2(seed: int = 0, W: int = 512, H: int = 512, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """512x512x3 image of 5 random ellipses + N(0, 0.1^2) per channel; 8-connected contrast weights
    (scale 1000, diagonals / sqrt 2); lambda = 2; 32x32 blocks, o = 2."""
    rng = np.random.default_rng(seed)
    fg = _ellipse_mask(rng, W, H, 5)
    base = np.where(fg, 0.7, 0.3)[:, :, None]
    img = base + rng.normal(0.0, 0.1, size=(H, W, 3))
    u = _gauss_llr(img, 0.7, 0.3, 0.1, channels=True)
    w = _weights_from_features(img[None], 2, 8, 0.1)
    return Problem(f"config2_ellipses{W}x{H}_8conn", (W, H, 1), 2, 8, u.astype(np.int32), w,
                   lambda_q8(2.0), (32, 32, 1), (2, 2, 0), mu0,
                   truth=fg.reshape(-1).astype(np.uint8))


def config2_even(K: int, seed: int = 0, W: int = 512, H: int = 512, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """The config2 image split into K even blocks (the 2D experiments' partitions into 32, 64 or 128 blocks):
    8 x 4, 8 x 8 or 16 x 8 blocks with o = 2, each the smallest size whose partition has that many blocks per
    axis (66 x 130, 66 x 66 or 34 x 66 at 512 x 512).  With 32 and 64 blocks the max-flow state of a block
    exceeds the LDS."""
    nbx, nby = {32: (8, 4), 64: (8, 8), 128: (16, 8)}[K]
    o = 2
    base = config2(seed=seed, W=W, H=H, mu0=mu0)
    size = lambda N, nb: -(-(N + (nb - 1) * o) // nb)   # noqa: E731
    return dataclasses.replace(base, name=f"config2_even{K}_ellipses{W}x{H}_8conn",
                               block=(size(W, nbx), size(H, nby), 1), overlap=(o, o, 0))


def _sized_axis(N: int, nb: int, pct: int) -> Tuple[int, int]:
    """Block edge and overlap of nb even blocks along an axis of length N grown by pct percent: stride s = N / nb
    (Size_00 blocks, each pixel in one block), B = round(s (1 + pct / 100)), o = B - s."""
    if N % nb:
        raise ValueError("the axis must split into equal blocks")
    s = N // nb
    B = int(_round(np.float64(s * (1.0 + pct / 100.0)))) if pct else s
    return B, B - s


def config2_sized(K: int, pct: int, seed: int = 0, W: int = 512, H: int = 512, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """The config2 image in the 2D experiments' partitions (Sec. 3 set-up): K = 32, 64 or 128 even blocks (8 x 4,
    8 x 8 or 16 x 8 along x, y) that cover the image without overlap (Size_00, pct = 0), then grown by 10 % or 25 %
    per axis (Size_10, Size_25), so that neighbouring blocks overlap by the growth."""
    nbx, nby = {32: (8, 4), 64: (8, 8), 128: (16, 8)}[K]
    Bx, ox = _sized_axis(W, nbx, pct)
    By, oy = _sized_axis(H, nby, pct)
    base = config2(seed=seed, W=W, H=H, mu0=mu0)
    return dataclasses.replace(base, name=f"config2_K{K}_size{pct:02d}_ellipses{W}x{H}_8conn",
                               block=(Bx, By, 1), overlap=(ox, oy, 0))


def config3_sized(K: int = 128, pct: int = 10, seed: int = 0, dims=(128, 128, 64), mu0: int = DEFAULT_MU0_3D) -> Problem:
    """The config3 volume in the 3D experiments' partition: K = 64 or 128 even blocks (4 x 4 x 4 or 8 x 4 x 4 along
    x, y, z), grown by pct percent per axis (Size_10 in the paper's 3D setting)."""
    nb = {64: (4, 4, 4), 128: (8, 4, 4)}[K]
    blk, ovl = zip(*[_sized_axis(N, n, pct) for N, n in zip(dims, nb)])
    base = config3(seed=seed, dims=dims, mu0=mu0)
    W, H, D = dims
    return dataclasses.replace(base, name=f"config3_K{K}_size{pct:02d}_spheres{W}x{H}x{D}_6conn",
                               block=tuple(blk), overlap=tuple(ovl))


def config3(seed: int = 0, dims=(128, 128, 64), mu0: int = DEFAULT_MU0_3D) -> Problem:
    """128x128x64 volume with 3 random spheres (r in U[8, 24]) + N(0, 0.2^2); 6-connected constant Potts
    w = 1000; lambda = 1.5; 16^3 blocks, o = 1."""
    W, H, D = dims
    rng = np.random.default_rng(seed)
    zz, yy, xx = np.mgrid[0:D, 0:H, 0:W].astype(np.float64)
    fg = np.zeros((D, H, W), dtype=bool)
    for _ in range(3):
        cx, cy, cz = rng.uniform(0, W), rng.uniform(0, H), rng.uniform(0, D)
        r = rng.uniform(8.0, 24.0)
        fg |= (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2 <= r * r
    img = np.where(fg, 0.7, 0.3) + rng.normal(0.0, 0.2, size=(D, H, W))
    u = _gauss_llr(img, 0.7, 0.3, 0.2)
    w = _constant_weights(dims, 3, 6, 1000)
    return Problem(f"config3_spheres{W}x{H}x{D}_6conn", (W, H, D), 3, 6, u.astype(np.int32), w,
                   lambda_q8(1.5), (16, 16, 16), (1, 1, 1), mu0,
                   truth=fg.reshape(-1).astype(np.uint8))


def config4(seed: int = 0, size: int = 256, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """Non-submodular 256x256 4-connected grid: u ~ U{-1000..1000}; each edge repulsive with p = 0.3
    (w ~ U{-500..-50}) else attractive (w ~ U{50..500}); lambda = 1; 4x4 blocks, o = 1; exhaustive solver."""
    rng = np.random.default_rng(seed)
    n = size * size
    u = rng.integers(-1000, 1001, size=n).astype(np.int32)
    offs = half_stencil(2, 4)
    w = np.zeros((len(offs), n), dtype=np.int32)
    yy, xx = np.mgrid[0:size, 0:size]
    for o, (dx, dy, _) in enumerate(offs):
        rep = rng.random(n) < 0.3
        neg = rng.integers(-500, -49, size=n)
        pos = rng.integers(50, 501, size=n)
        ok = ((xx + dx < size) & (yy + dy < size) & (xx + dx >= 0)).reshape(-1)
        w[o] = np.where(ok, np.where(rep, neg, pos), 0)
    return Problem(f"config4_nonsubmodular{size}_4conn", (size, size, 1), 2, 4, u, w, lambda_q8(1.0),
                   (4, 4, 1), (1, 1, 0), mu0, solver="exhaustive")


SERVE_SIDES = (128, 256, 512, 1024, 2048)


def config4_lsatr(seed: int = 0, size: int = 256, B: int = 16, o: int = 1, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """The non-submodular grid of config4 (30 % repulsive edges) in B x B blocks with o-pixel overlap, too large to
    enumerate: every block is solved by the trust-region local submodular approximation (LSA-TR)."""
    p = config4(seed=seed, size=size, mu0=mu0)
    return dataclasses.replace(p, name=f"config4_lsatr{B}_nonsubmodular{size}_4conn", block=(B, B, 1),
                               overlap=(o, o, 0), solver="lsatr")


def config5_request(r: int, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """Serving request r (seed r + 1): grey disk image as config 1 at H in {128..2048}, W = round(H * U[0.5, 2]),
    disk radius 20 * min(H, W) / 64 centred; 8-connected contrast weights (sigma_w = 0.1, diagonals / sqrt 2);
    lambda ~ U[0.5, 3].  The block partition is left to the caller (block = overlap = 0)."""
    rng = np.random.default_rng(r + 1)
    H = int(rng.choice(SERVE_SIDES))
    W = int(_round(np.float64(H * rng.uniform(0.5, 2.0))))
    lam = float(rng.uniform(0.5, 3.0))
    return _disk_request(rng, W, H, lam, f"config5_req{r}_{W}x{H}", mu0)


def config5_image(W: int, H: int, lam: float = 1.5, seed: int = 0, mu0: int = DEFAULT_MU0_2D,
                  conn: int = 8) -> Problem:
    """A serving-style image of a chosen size and 2D stencil (used to tune the block partition per image shape)."""
    return _disk_request(np.random.default_rng(seed), W, H, lam, f"config5_image_{W}x{H}_{conn}conn", mu0, conn)


def _disk_request(rng, W, H, lam, name, mu0, conn=8) -> Problem:
    cx, cy = W / 2.0, H / 2.0
    rad = 20.0 * min(H, W) / 64.0
    yy, xx = np.mgrid[0:H, 0:W]
    fg = (xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad
    img = np.where(fg, 0.7, 0.3) + rng.normal(0.0, 0.15, size=(H, W))
    u = _gauss_llr(img, 0.7, 0.3, 0.15)
    w = _weights_from_features(img[None, :, :, None], 2, conn, 0.1)
    return Problem(name, (W, H, 1), 2, conn, u.astype(np.int32), w, lambda_q8(lam),
                   (0, 0, 0), (0, 0, 0), mu0, truth=fg.reshape(-1).astype(np.uint8))


def config5_trace(n_requests: int = 2000, mean_gap_s: float = 0.005, seed: int = 0) -> np.ndarray:
    """Poisson arrival times (seconds) for the serving workload: exponential gaps, mean 5 ms (200 req/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(mean_gap_s, size=n_requests))


def config_kernel(k: int, seed: int = 0, W: int = 512, H: int = 512, mu0: int = DEFAULT_MU0_2D) -> Problem:
    """The image of config2 with the k x k square neighbourhood (k = 5, 7 or 9) of the paper's larger-kernel
    experiments: contrast weights on every offset of the square (scale 1000, divided by the offset's length);
    lambda = 0.5 (k = 5), 0.6 (k = 7) or 0.4 (k = 9), which keep the total smoothing per pixel at or below
    config2's and converge within a few iterations (with k = 5 and lambda = 1 a pixel keeps oscillating between its
    blocks and the stopping rule never holds in 50 iterations); 32x32 blocks with o = 2 for k = 5, 16x16 blocks
    with o = 2 for k = 7 and 9 (LDS per block node grows with the stencil)."""
    if k not in (5, 7, 9):
        raise ValueError("k must be 5, 7 or 9")
    conn = {5: 24, 7: 48, 9: 80}[k]
    rng = np.random.default_rng(seed)
    fg = _ellipse_mask(rng, W, H, 5)
    base = np.where(fg, 0.7, 0.3)[:, :, None]
    img = base + rng.normal(0.0, 0.1, size=(H, W, 3))
    u = _gauss_llr(img, 0.7, 0.3, 0.1, channels=True)
    w = _weights_from_features(img[None], 2, conn, 0.1)
    B = 32 if k == 5 else 16
    return Problem(f"kernel{k}_ellipses{W}x{H}_{conn}conn", (W, H, 1), 2, conn, u.astype(np.int32), w,
                   lambda_q8({5: 0.5, 7: 0.6, 9: 0.4}[k]), (B, B, 1), (2, 2, 0), mu0,
                   truth=fg.reshape(-1).astype(np.uint8))


def config3_kernel5(seed: int = 0, dims=(128, 128, 64), mu0: int = BALL_MU0, k: int = 5) -> Problem:
    """The volume of config3 with the spherical kernel of size k: the radius-2 ball (k = 5, 32 neighbours), the
    radius-3 ball (k = 7, 122 neighbours) or the radius-4 ball (k = 9, 256 neighbours), distance-weighted Potts
    w = round(1000 / |offset|), lambda = 0.4, 0.16 or 25/256 (total smoothing per voxel near config3's
    1.5 x 6 x 1000); 8^3, 6^3 or 5^3 blocks with o = 1 (141, 513 or 1065 LDS bytes per block node)."""
    if k not in (5, 7, 9):
        raise ValueError("k must be 5, 7 or 9")
    conn = {5: 32, 7: 122, 9: 256}[k]
    base = config3(seed=seed, dims=dims, mu0=mu0)
    W, H, D = dims
    zz, yy, xx = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    offs = half_stencil(3, conn)
    w = np.zeros((len(offs), W * H * D), dtype=np.int32)
    for o, (dx, dy, dz) in enumerate(offs):
        ok = ((xx + dx >= 0) & (xx + dx < W) & (yy + dy >= 0) & (yy + dy < H)
              & (zz + dz >= 0) & (zz + dz < D))
        w[o] = np.where(ok.reshape(-1), int(_round(1000.0 / math.sqrt(dx * dx + dy * dy + dz * dz))), 0)
    B = {5: 8, 7: 6, 9: 5}[k]
    lam_q = {5: lambda_q8(0.4), 7: lambda_q8(0.16), 9: 25}[k]
    return Problem(f"kernel{k}_spheres{W}x{H}x{D}_{conn}conn", (W, H, D), 3, conn, base.u, w,
                   lam_q, (B, B, B), (1, 1, 1), mu0, truth=base.truth)


def random_problem(seed: int, dims, conn: int, block, overlap, lam_q8: int = 256,
                   u_range=(-3000, 3000), w_range=(0, 1000), neg_frac: float = 0.0,
                   mu0: int = DEFAULT_MU0_2D, solver: str = "maxflow") -> Problem:
    """Uniform random integer unaries and weights (a fraction neg_frac of edges negated) on any grid."""
    rng = np.random.default_rng(seed)
    W, H, D = dims
    ndim = 3 if conn in (6, 32, 122, 256) else 2
    n = W * H * D
    u = rng.integers(u_range[0], u_range[1] + 1, size=n).astype(np.int32)
    offs = half_stencil(ndim, conn)
    zz, yy, xx = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    w = np.zeros((len(offs), n), dtype=np.int32)
    for o, (dx, dy, dz) in enumerate(offs):
        ok = ((xx + dx >= 0) & (xx + dx < W) & (yy + dy >= 0) & (yy + dy < H)
              & (zz + dz >= 0) & (zz + dz < D)).reshape(-1)
        vals = rng.integers(w_range[0], w_range[1] + 1, size=n)
        if neg_frac > 0:
            vals = np.where(rng.random(n) < neg_frac, -vals, vals)
        w[o] = np.where(ok, vals, 0)
    return Problem(f"random{seed}_{W}x{H}x{D}_{conn}", (W, H, D), ndim, conn, u, w, lam_q8,
                   tuple(block), tuple(overlap), mu0, solver=solver)
