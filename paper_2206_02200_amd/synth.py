"""Seeded synthetic inputs shaped like the paper's workloads.

The paper evaluates GridShift on BSDS500 colour images (Section 3.2) and on
UCI/HAR-style low-dimensional clustering sets (Table 2, supplement Table 5).
Those datasets are not available here, so these generators stand in for them:

* Voronoi images: R random seed points split a H x W image into regions; each
  region has a mean colour, an optional linear colour ramp and i.i.d. Gaussian
  noise, clipped to [0, 255].  Pixels are emitted in raster order.
* Features: RGB, or (s*x, s*y, L*, a*, b*) with CIE L*a*b* computed in FP64
  from sRGB (IEC 61966-2-1, D65 white) before the cast to float32.
* Gaussian mixtures: isotropic components, means uniform in [0, 100]^d,
  sigma uniform in [1, 3], Dirichlet(1) weights, multinomial counts, points
  shuffled by a seeded permutation.

All randomness comes from explicit seeds: numpy PCG64, plus a seeded torch
generator for the pixel noise of the device-side variants used for the large
batched workloads.  This module holds no GridShift arithmetic; both the oracle
side and the GPU side read its output.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# --------------------------------------------------------------------------
# colour conversion (sRGB -> XYZ (D65) -> CIE L*a*b*), FP64
# --------------------------------------------------------------------------
_SRGB_TO_XYZ = np.array(
    [[0.4124, 0.3576, 0.1805], [0.2126, 0.7152, 0.0722], [0.0193, 0.1192, 0.9505]],
    dtype=np.float64,
)
_WHITE_D65 = np.array([0.95047, 1.0, 1.08883], dtype=np.float64)
_LAB_EPS = 216.0 / 24389.0
_LAB_KAPPA = 24389.0 / 27.0


def srgb_to_lab(rgb: np.ndarray) -> np.ndarray:
    """rgb in [0, 255] (float64, [..., 3]) -> L*a*b* (float64)."""
    c = np.asarray(rgb, dtype=np.float64) / 255.0
    lin = np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)
    xyz = lin @ _SRGB_TO_XYZ.T
    t = xyz / _WHITE_D65
    f = np.where(t > _LAB_EPS, np.cbrt(t), (_LAB_KAPPA * t + 16.0) / 116.0)
    L = 116.0 * f[..., 1] - 16.0
    a = 500.0 * (f[..., 0] - f[..., 1])
    b = 200.0 * (f[..., 1] - f[..., 2])
    return np.stack([L, a, b], axis=-1)


# --------------------------------------------------------------------------
# Voronoi images
# --------------------------------------------------------------------------
def voronoi_rgb(H: int, W: int, regions: int, sigma: float, ramp: float, seed: int) -> np.ndarray:
    """[H*W, 3] float64 RGB in raster order (row-major, x = column)."""
    rng = np.random.default_rng(seed)
    sx = rng.uniform(0.0, W, size=regions)
    sy = rng.uniform(0.0, H, size=regions)
    mu = rng.uniform(0.0, 255.0, size=(regions, 3))
    G = rng.uniform(-ramp, ramp, size=(regions, 3, 2)) if ramp > 0 else np.zeros((regions, 3, 2))
    ys = np.arange(H, dtype=np.float64)[:, None]
    xs = np.arange(W, dtype=np.float64)[None, :]
    best = np.full((H, W), np.inf)
    lab = np.zeros((H, W), dtype=np.int64)
    for r in range(regions):  # ties go to the lowest region index
        dist = (xs - sx[r]) ** 2 + (ys - sy[r]) ** 2
        closer = dist < best
        best = np.where(closer, dist, best)
        lab = np.where(closer, r, lab)
    lab = lab.reshape(-1)
    X = np.broadcast_to(xs, (H, W)).reshape(-1)
    Y = np.broadcast_to(ys, (H, W)).reshape(-1)
    u = (X - sx[lab]) / W
    v = (Y - sy[lab]) / H
    col = mu[lab] + G[lab, :, 0] * u[:, None] + G[lab, :, 1] * v[:, None]
    col = col + sigma * rng.standard_normal(size=(H * W, 3))
    return np.clip(col, 0.0, 255.0)


def xy_lab_features(H: int, W: int, rgb: np.ndarray, s: float) -> np.ndarray:
    """(s*x, s*y, L, a, b) as float32, [H*W, 5]."""
    lab = srgb_to_lab(rgb)
    X = np.broadcast_to(np.arange(W, dtype=np.float64)[None, :], (H, W)).reshape(-1)
    Y = np.broadcast_to(np.arange(H, dtype=np.float64)[:, None], (H, W)).reshape(-1)
    f = np.column_stack([s * X, s * Y, lab])
    return f.astype(np.float32)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    x: np.ndarray  # [n, d]
    h: float
    max_iter: int


def image_rgb_f64(seed: int = 1, H: int = 120, W: int = 160, regions: int = 8, sigma: float = 8.0) -> Workload:
    """160x120 Voronoi image, 8 regions, noise 8, RGB float64 (d=3), h=24."""
    rgb = voronoi_rgb(H, W, regions, sigma, 0.0, seed)
    return Workload(f"voronoi{W}x{H}_rgb_f64", rgb, 24.0, 100)


def image_xylab_f32(seed: int = 2, H: int = 1080, W: int = 1920, regions: int = 40, sigma: float = 6.0,
                    s: float = 0.25, h: float = 16.0, ramp: float = 64.0) -> Workload:
    """1920x1080 Voronoi image with colour ramps; (s*x, s*y, L, a, b) float32, h=16."""
    rgb = voronoi_rgb(H, W, regions, sigma, ramp, seed)
    return Workload(f"voronoi{W}x{H}_xylab_s{s:g}_f32", xy_lab_features(H, W, rgb, s), h, 100)


def gmm_f32(n: int, d: int, seed: int, components: int = 50, h: float = 4.0) -> Workload:
    """Isotropic Gaussian mixture in [0,100]^d, float32, shuffled."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(components))
    mu = rng.uniform(0.0, 100.0, size=(components, d))
    sig = rng.uniform(1.0, 3.0, size=components)
    cnt = rng.multinomial(n, w)
    comp = np.repeat(np.arange(components), cnt)
    x = mu[comp] + sig[comp][:, None] * rng.standard_normal(size=(n, d))
    perm = rng.permutation(n)
    return Workload(f"gmm{components}_n{n}_d{d}_f32", x[perm].astype(np.float32), h, 100)


def unit_gmm_f32(n: int, d: int, seed: int, components: int = 12) -> np.ndarray:
    """A clustering set scaled into [0,1]^d (the range the bandwidth tuning of
    Section 4.1 scans): an isotropic Gaussian mixture (means U[0,1]^d, sigma
    U[0.02,0.06], Dirichlet(1) weights), each coordinate mapped affinely onto
    [0,1] by its own minimum and maximum, float32, shuffled."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(components))
    mu = rng.uniform(0.0, 1.0, size=(components, d))
    sig = rng.uniform(0.02, 0.06, size=components)
    cnt = rng.multinomial(n, w)
    comp = np.repeat(np.arange(components), cnt)
    x = mu[comp] + sig[comp][:, None] * rng.standard_normal(size=(n, d))
    lo, hi = x.min(axis=0), x.max(axis=0)
    x = (x - lo) / np.where(hi > lo, hi - lo, 1.0)
    return x[rng.permutation(n)].astype(np.float32)


def hsweep_grid(count: int = 20) -> np.ndarray:
    """Bandwidths 1/count, 2/count, ..., 1: an even grid over (0,1]."""
    return np.arange(1, count + 1, dtype=np.float64) / count


def moving_blob_video(T: int = 120, H: int = 480, W: int = 640, radius: float = 28.0, seed: int = 7,
                      sigma: float = 6.0, dtype=np.float32, discs: int = 1):
    """A synthetic tracking sequence (stand-in for OTB100): textured discs of
    distinct colour families moving over a smooth two-colour background ramp.

    Each disc starts at a random point of the central half, moves with a
    random velocity of 2-5 px per frame plus a slow sinusoidal wobble, and
    bounces off the borders; the first disc's colour is (215, 60, 45), the
    others' U[120,255] x U[0,80] x U[0,255] (red-dominant, away from the
    background), each plus N(0, sigma^2) per pixel; the background is a
    diagonal ramp between (20, 90, 160) and (60, 170, 90) plus the same noise;
    clipped to [0, 255]; later discs are drawn over earlier ones.  Returns
    (frames [T][H][W][3], centres [T][discs][2] as (x, y), squeezed to [T][2]
    for one disc)."""
    rng = np.random.default_rng(seed)
    state = []
    for j in range(discs):
        cx, cy = rng.uniform(0.25 * W, 0.75 * W), rng.uniform(0.25 * H, 0.75 * H)
        ang = rng.uniform(0, 2 * np.pi)
        sp = rng.uniform(2.0, 5.0)
        col = np.array([215.0, 60.0, 45.0]) if j == 0 else np.array(
            [rng.uniform(120, 255), rng.uniform(0, 80), rng.uniform(0, 255)])
        state.append([cx, cy, sp * np.cos(ang), sp * np.sin(ang), col, rng.uniform(0, 6.28) if j else 0.0])
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    t_ramp = (xx / W + yy / H) / 2.0
    bg = np.stack([20 + 40 * t_ramp, 90 + 80 * t_ramp, 160 - 70 * t_ramp], axis=-1)
    frames = np.empty((T, H, W, 3), dtype=dtype)
    centres = np.empty((T, discs, 2), dtype=np.float64)
    for t in range(T):
        img = bg + sigma * rng.standard_normal(size=(H, W, 3))
        for j, st in enumerate(state):
            ph = 0.0 if j == 0 else st[5]
            ox = st[0] + 6.0 * np.sin(0.15 * t + ph)
            oy = st[1] + 6.0 * np.cos(0.11 * t + ph)
            centres[t, j] = (ox, oy)
            disc = (xx - ox) ** 2 + (yy - oy) ** 2 <= radius * radius
            img[disc] = st[4] + sigma * rng.standard_normal(size=(int(disc.sum()), 3))
            st[0], st[1] = st[0] + st[2], st[1] + st[3]
            if not (radius < st[0] < W - radius):
                st[2] = -st[2]
            if not (radius < st[1] < H - radius):
                st[3] = -st[3]
        frames[t] = np.clip(img, 0, 255).astype(dtype)
    return frames, (centres[:, 0] if discs == 1 else centres)


def gmm_truth(n: int, d: int, seed: int, components: int = 50) -> np.ndarray:
    """Component id of every point of gmm_f32(n, d, seed) (same draws)."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(components))
    rng.uniform(0.0, 100.0, size=(components, d))
    rng.uniform(1.0, 3.0, size=components)
    cnt = rng.multinomial(n, w)
    comp = np.repeat(np.arange(components), cnt)
    rng.standard_normal(size=(n, d))
    perm = rng.permutation(n)
    return comp[perm]


@dataclass
class BatchSpec:
    H: int
    W: int
    regions: int
    sigma: float
    h: float
    seed: int


def batch_specs(B: int = 256, seed: int = 3, hmin: int = 240, hmax: int = 1080, wmin: int = 320,
                wmax: int = 1920) -> list[BatchSpec]:
    """Per-image sizes, region counts, noise levels and bandwidths of a batch."""
    rng = np.random.default_rng(seed)
    Hs = rng.integers(hmin, hmax + 1, size=B)
    Ws = rng.integers(wmin, wmax + 1, size=B)
    Rs = rng.integers(5, 61, size=B)
    sig = rng.uniform(4.0, 12.0, size=B)
    hs = rng.choice(np.array([12.0, 16.0, 24.0]), size=B)
    return [BatchSpec(int(Hs[b]), int(Ws[b]), int(Rs[b]), float(sig[b]), float(hs[b]), 3000 + b) for b in range(B)]


def batch_image(spec: BatchSpec) -> np.ndarray:
    """One batched instance: RGB float32 [H*W, 3]."""
    return voronoi_rgb(spec.H, spec.W, spec.regions, spec.sigma, 0.0, spec.seed).astype(np.float32)


def diff_image(b: int, H: int = 512, W: int = 512, regions: int = 30, sigma: float = 6.0) -> np.ndarray:
    """Differentiable-form instance b: (x, y, L, a, b) float32 with s = 1."""
    rgb = voronoi_rgb(H, W, regions, sigma, 64.0, 5000 + b)
    return xy_lab_features(H, W, rgb, 1.0)


# --------------------------------------------------------------------------
# small inputs for tests
# --------------------------------------------------------------------------
def dyadic(x: np.ndarray, bits: int = 8) -> np.ndarray:
    """Round to multiples of 2^-bits (float64); with |x| < 2^16 sums stay exact."""
    s = float(2 ** bits)
    return np.round(np.asarray(x, dtype=np.float64) * s) / s


def separated_blobs(k: int, d: int, per: int, h: float, seed: int, spacing: float = 8.0,
                    sigma_frac: float = 0.25) -> tuple[np.ndarray, np.ndarray]:
    """k Gaussian blobs on a lattice with spacing*h between centres, sigma =
    sigma_frac*h, truncated at 3 sigma.  Returns (x float64 [k*per, d], truth)."""
    rng = np.random.default_rng(seed)
    side = int(np.ceil(k ** (1.0 / d)))
    centres = []
    for c in range(k):
        idx, cc = c, []
        for _ in range(d):
            cc.append(idx % side)
            idx //= side
        centres.append(cc)
    centres = (np.array(centres, dtype=np.float64) + 0.5) * spacing * h + rng.uniform(0, h, size=(1, d))
    z = rng.standard_normal(size=(k * per, d))
    z = np.clip(z, -3.0, 3.0)
    truth = np.repeat(np.arange(k), per)
    x = centres[truth] + sigma_frac * h * z
    perm = rng.permutation(k * per)
    return x[perm], truth[perm]


# --------------------------------------------------------------------------
# device-side generation of the large batched workloads (same recipe; the
# region parameters come from numpy PCG64, the pixel noise from a seeded
# torch generator on the device)
# --------------------------------------------------------------------------
def voronoi_rgb_torch(H: int, W: int, regions: int, sigma: float, ramp: float, seed: int, device):
    """[H*W, 3] float64 RGB in raster order, computed with torch on `device`."""
    import torch

    rng = np.random.default_rng(seed)
    sx = torch.tensor(rng.uniform(0.0, W, size=regions), dtype=torch.float64, device=device)
    sy = torch.tensor(rng.uniform(0.0, H, size=regions), dtype=torch.float64, device=device)
    mu = torch.tensor(rng.uniform(0.0, 255.0, size=(regions, 3)), dtype=torch.float64, device=device)
    G = torch.tensor(rng.uniform(-ramp, ramp, size=(regions, 3, 2)) if ramp > 0 else np.zeros((regions, 3, 2)),
                     dtype=torch.float64, device=device)
    ys = torch.arange(H, dtype=torch.float64, device=device)[:, None]
    xs = torch.arange(W, dtype=torch.float64, device=device)[None, :]
    best = torch.full((H, W), float("inf"), dtype=torch.float64, device=device)
    lab = torch.zeros((H, W), dtype=torch.int64, device=device)
    for r in range(regions):  # ties go to the lowest region index
        dist = (xs - sx[r]) ** 2 + (ys - sy[r]) ** 2
        closer = dist < best
        best = torch.where(closer, dist, best)
        lab = torch.where(closer, torch.full_like(lab, r), lab)
    lab = lab.reshape(-1)
    X = xs.expand(H, W).reshape(-1)
    Y = ys.expand(H, W).reshape(-1)
    u = (X - sx[lab]) / W
    v = (Y - sy[lab]) / H
    col = mu[lab] + G[lab, :, 0] * u[:, None] + G[lab, :, 1] * v[:, None]
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    col = col + sigma * torch.randn((H * W, 3), dtype=torch.float64, device=device, generator=gen)
    return col.clamp(0.0, 255.0)


def srgb_to_lab_torch(rgb):
    """torch version of srgb_to_lab (float64)."""
    import torch

    c = rgb / 255.0
    lin = torch.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)
    M = torch.tensor(_SRGB_TO_XYZ, dtype=torch.float64, device=rgb.device)
    xyz = lin @ M.T
    t = xyz / torch.tensor(_WHITE_D65, dtype=torch.float64, device=rgb.device)
    f = torch.where(t > _LAB_EPS, torch.pow(t.clamp_min(0.0), 1.0 / 3.0), (_LAB_KAPPA * t + 16.0) / 116.0)
    L = 116.0 * f[:, 1] - 16.0
    a = 500.0 * (f[:, 0] - f[:, 1])
    b = 200.0 * (f[:, 1] - f[:, 2])
    return torch.stack([L, a, b], dim=1)


def batch_rgb_torch(specs: list[BatchSpec], device):
    """Concatenated float32 RGB points of a batch, row offsets and bandwidths."""
    import torch

    xs = [voronoi_rgb_torch(s.H, s.W, s.regions, s.sigma, 0.0, s.seed, device).to(torch.float32) for s in specs]
    off = np.concatenate([[0], np.cumsum([s.H * s.W for s in specs])]).astype(np.int64)
    return torch.cat(xs, dim=0), off, np.array([s.h for s in specs])


def diff_batch_torch(B: int, device, H: int = 512, W: int = 512, regions: int = 30, sigma: float = 6.0):
    """B images of (x, y, L, a, b) float32 features with s = 1, concatenated."""
    import torch

    out = []
    X = torch.arange(W, dtype=torch.float64, device=device)[None, :].expand(H, W).reshape(-1)
    Y = torch.arange(H, dtype=torch.float64, device=device)[:, None].expand(H, W).reshape(-1)
    for b in range(B):
        rgb = voronoi_rgb_torch(H, W, regions, sigma, 64.0, 5000 + b, device)
        lab = srgb_to_lab_torch(rgb)
        out.append(torch.cat([X[:, None], Y[:, None], lab], dim=1).to(torch.float32))
    off = np.arange(B + 1, dtype=np.int64) * (H * W)
    return torch.cat(out, dim=0), off
