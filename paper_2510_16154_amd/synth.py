"""Seeded synthetic images that stand in for the paper's test pictures.

The paper's images (an MRI scan from a cited publication and private photos,
Sec. 3.2 and Sec. 4.2) are not available, so every input here is a seeded
Voronoi mosaic with the value range the paper uses (colours in [0,1], Sec. 2).
This module is shared input plumbing only: it holds none of the method's
arithmetic and is imported both by the tests that drive the CPU oracle and by
the GPU path's tests and benchmark.

Recipe (numpy PCG64, ``default_rng(seed)``; draws in this fixed order):
  1. sites: ``regions x 2`` uniform in [0,W) x [0,H) (pixel units, (x, y));
  2. region colours: U[0,1]^C, or smooth spectra when ``spectra=True``;
  3. per-region linear colour gradient (only when ``gradient_amp > 0``):
     direction angle U[0,2pi), colour direction U[-1,1]^C;
  4. i.i.d. Gaussian noise N(0, sigma^2) per pixel and channel.
Each pixel takes the region whose site is nearest to its centre
(q+1/2, r+1/2) (ties: lowest site index), adds the region's gradient term
``amp * d_s * ((x, y) - site_s) . u_s`` in normalised coordinates (x=(q+1/2)/W,
y=(r+1/2)/H), adds noise, is clipped to [0,1] and stored as float32, HWC
(channel fastest), row 0 first in memory.
"""
from __future__ import annotations

import numpy as np

__all__ = ["voronoi_image", "voronoi_labels", "batch_shapes", "wsnet_init", "hashed_block", "patched_block"]


def _nearest_site(H: int, W: int, sites: np.ndarray) -> np.ndarray:
    xs = np.arange(W, dtype=np.float64) + 0.5
    ys = np.arange(H, dtype=np.float64) + 0.5
    best = np.full((H, W), np.inf)
    lab = np.zeros((H, W), dtype=np.int32)
    for s, (sx, sy) in enumerate(sites):
        d2 = (ys[:, None] - sy) ** 2 + (xs[None, :] - sx) ** 2
        closer = d2 < best  # strict: earlier sites win ties
        best = np.where(closer, d2, best)
        lab = np.where(closer, s, lab)
    return lab


def voronoi_image(H: int, W: int, C: int, regions: int, noise_sigma: float,
                  seed: int, gradient_amp: float = 0.0, spectra: bool = False,
                  return_labels: bool = False):
    """Return an ``(H, W, C)`` float32 Voronoi image (and its labels if asked)."""
    if H < 1 or W < 1 or C < 1 or regions < 1:
        raise ValueError("H, W, C and regions must be >= 1")
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, size=(regions, 2)) * np.array([W, H], dtype=np.float64)
    if spectra:
        m = rng.uniform(0.2, 0.8, size=regions)
        qs = np.arange(1, 4, dtype=np.float64)
        amp = rng.uniform(-1.0, 1.0, size=(regions, 3)) * (0.3 / qs)[None, :]
        ph = rng.uniform(0.0, 2.0 * np.pi, size=(regions, 3))
        band = np.arange(C, dtype=np.float64) / max(C - 1, 1) * 30.0
        spec = m[:, None] + np.sum(
            amp[:, :, None] * np.cos(np.pi * qs[None, :, None] * band[None, None, :] / 30.0
                                     + ph[:, :, None]), axis=1)
        colours = np.clip(spec, 0.0, 1.0)
    else:
        colours = rng.uniform(0.0, 1.0, size=(regions, C))
    lab = _nearest_site(H, W, sites)
    img = colours[lab]  # (H, W, C) float64
    if gradient_amp > 0.0:
        theta = rng.uniform(0.0, 2.0 * np.pi, size=regions)
        cdir = rng.uniform(-1.0, 1.0, size=(regions, C))
        x = (np.arange(W, dtype=np.float64) + 0.5) / W
        y = (np.arange(H, dtype=np.float64) + 0.5) / H
        sxn = sites[:, 0] / W
        syn = sites[:, 1] / H
        proj = ((x[None, :] - sxn[lab]) * np.cos(theta)[lab]
                + (y[:, None] - syn[lab]) * np.sin(theta)[lab])
        img = img + gradient_amp * cdir[lab] * proj[:, :, None]
    if noise_sigma > 0.0:
        img = img + rng.normal(0.0, noise_sigma, size=(H, W, C))
    img = np.clip(img, 0.0, 1.0).astype(np.float32)
    if return_labels:
        return img, lab
    return img


def voronoi_labels(H: int, W: int, regions: int, seed: int) -> np.ndarray:
    """Ground-truth region labels of ``voronoi_image`` with the same seed."""
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, size=(regions, 2)) * np.array([W, H], dtype=np.float64)
    return _nearest_site(H, W, sites)


def batch_shapes(n: int, seed: int, lo: int = 128, hi: int = 1024):
    """Uneven, non-square image specs for the batched workload.

    Returns ``n`` tuples ``(H, W, regions, sigma, image_seed)`` with sides
    uniform in [lo, hi] (redrawn when H == W), 4-16 regions, noise sigma
    uniform in [0.02, 0.1]; image ``i`` uses seed ``seed * 1000 + i``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        while True:
            H = int(rng.integers(lo, hi + 1))
            W = int(rng.integers(lo, hi + 1))
            if H != W:
                break
        regions = int(rng.integers(4, 17))
        sigma = float(rng.uniform(0.02, 0.1))
        out.append((H, W, regions, sigma, seed * 1000 + i))
    return out


# Convolution shapes (input, output channels) of the warm-start network, in order.
WSNET_CONVS = [(3, 16), (16, 32), (32, 64), (80, 32), (32, 6)]


def wsnet_init(K: int, seed: int) -> np.ndarray:
    """Seeded starting weights of the warm-start network, flat FP32: per 3 x 3
    convolution He-normal weights (std sqrt(2 / (9 Cin))) then zero biases;
    then the control head's 64 x 2K weights (std 1/8) and zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in WSNET_CONVS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), size=9 * cin * cout))
        parts.append(np.zeros(cout))
    parts.append(rng.normal(0.0, 0.125, size=64 * 2 * K))
    parts.append(np.zeros(2 * K))
    return np.concatenate(parts).astype(np.float32)


# ---------------------------------------------------------------------------
# Images too large to hold on the host (up to 4e9 elements): every element is a
# function of its index, so any rectangle can be made on its own, on the GPU for
# the whole image or on the CPU for a small crop, with the same bits.
#   element (y, x, ch) of an image W wide with C channels has index
#   e = (y W + x) C + ch;  u = hash32(lo32(e) ^ hash32(hi32(e) + seed)) >> 8, a
#   24-bit integer, and the value is lo + (hi - lo) u / 2^24 in FP32.
# hash32 is the two-round xor-shift-multiply integer mixer (multiplier 0x45d9f3b),
# evaluated in int64 with every product below 2^63, so CPU and GPU agree exactly.

_MASK32 = 0xFFFFFFFF


def _hash32(x):
    x = ((x >> 16) ^ x) * 0x45D9F3B & _MASK32
    x = ((x >> 16) ^ x) * 0x45D9F3B & _MASK32
    return (x >> 16) ^ x


def hashed_block(y0: int, h: int, x0: int, w: int, W: int, C: int, seed: int, lo: float = -1.0, hi: float = 1.0,
                 device="cpu"):
    """Rows y0..y0+h-1, columns x0..x0+w-1 (all channels) of the hashed image
    of width W: an ``h x w x C`` FP32 torch tensor on ``device`` with values in
    [lo, hi)."""
    import torch
    ys = torch.arange(y0, y0 + h, dtype=torch.int64, device=device).view(h, 1, 1)
    xs = torch.arange(x0, x0 + w, dtype=torch.int64, device=device).view(1, w, 1)
    cs = torch.arange(C, dtype=torch.int64, device=device).view(1, 1, C)
    e = (ys * W + xs) * C + cs
    u = _hash32((e & _MASK32) ^ _hash32((e >> 32) + (seed & _MASK32))) >> 8
    return (lo + (hi - lo) * (u.to(torch.float64) / float(1 << 24))).to(torch.float32)


def patched_block(y0: int, h: int, x0: int, w: int, W: int, C: int, seed: int, patches, background: float = 0.5,
                  amp: float = 0.5, device="cpu"):
    """The same rectangle of an image that is ``background`` everywhere except in
    the square patches ``(py, px, side)``, where it takes the hashed values in
    [background - amp, background + amp) (``hashed_block`` with ``seed``)."""
    import torch
    out = torch.full((h, w, C), background, dtype=torch.float32, device=device)
    for py, px, side in patches:
        ya, yb = max(py, y0), min(py + side, y0 + h)
        xa, xb = max(px, x0), min(px + side, x0 + w)
        if ya < yb and xa < xb:
            out[ya - y0:yb - y0, xa - x0:xb - x0] = hashed_block(ya, yb - ya, xa, xb - xa, W, C, seed, background - amp,
                                                                 background + amp, device)
    return out
