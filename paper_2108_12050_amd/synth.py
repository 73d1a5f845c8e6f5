"""Seeded synthetic inputs for the MHFD detector.

The paper measures on a private SEM focal series of ATUM-collected sections
(section 5); those images are not available, so these generators stand in for
them with the shapes, value ranges and structure of the five workloads the
detector is measured on.  Every generator draws from
``numpy.random.default_rng(seed)`` in the order written in its docstring, so a
(seed, shape) pair always gives the same array.

This module renders test images only.  It holds none of the detector's
arithmetic (no LoG, maxima, thresholds or pruning) and is shared by the
oracle-side tests, the GPU tests and the benchmark.
"""
from __future__ import annotations

import math

import numpy as np

BACKGROUND = 0.1


def _gauss_window(c: float, t: float, n: int, halfwidth: float):
    """Integer pixel range [lo, hi) within `halfwidth` of c and the 1-D
    Gaussian profile exp(-(p - c)^2 / (2 t^2)) on it."""
    lo = max(0, int(math.floor(c - halfwidth)))
    hi = min(n, int(math.ceil(c + halfwidth)) + 1)
    p = np.arange(lo, hi, dtype=np.float64)
    return lo, hi, np.exp(-((p - c) ** 2) / (2.0 * t * t))


def render_blobs(img: np.ndarray, cy, cx, t, amp, halfwidth_t: float = 6.0) -> None:
    """Add isotropic Gaussian blobs amp * exp(-((y-cy)^2 + (x-cx)^2) / (2 t^2)),
    evaluated at integer pixel centres within halfwidth_t * t of the centre
    (beyond 6 t a blob is below 2e-8 of its amplitude)."""
    H, W = img.shape
    for y0, x0, s, a in zip(cy, cx, t, amp):
        hw = halfwidth_t * s
        ylo, yhi, gy = _gauss_window(y0, s, H, hw)
        xlo, xhi, gx = _gauss_window(x0, s, W, hw)
        if yhi > ylo and xhi > xlo:
            img[ylo:yhi, xlo:xhi] += a * np.outer(gy, gx)


def render_ridges(img: np.ndarray, cy, cx, length, angle, amp, width_std: float = 1.0) -> None:
    """Add straight ridge segments: amp * exp(-d^2 / (2 width_std^2)), d the
    distance from the pixel centre to the segment of the given length centred
    at (cy, cx) with direction `angle`."""
    H, W = img.shape
    m = 4.0 * width_std
    for y0, x0, L, th, a in zip(cy, cx, length, angle, amp):
        dy, dx = math.sin(th), math.cos(th)
        ya, xa = y0 - 0.5 * L * dy, x0 - 0.5 * L * dx
        yb, xb = y0 + 0.5 * L * dy, x0 + 0.5 * L * dx
        ylo = max(0, int(math.floor(min(ya, yb) - m)))
        yhi = min(H, int(math.ceil(max(ya, yb) + m)) + 1)
        xlo = max(0, int(math.floor(min(xa, xb) - m)))
        xhi = min(W, int(math.ceil(max(xa, xb) + m)) + 1)
        if yhi <= ylo or xhi <= xlo:
            continue
        py = np.arange(ylo, yhi, dtype=np.float64)[:, None]
        px = np.arange(xlo, xhi, dtype=np.float64)[None, :]
        # projection onto the segment, clamped to its ends
        u = np.clip((py - ya) * dy + (px - xa) * dx, 0.0, L)
        qy, qx = ya + u * dy, xa + u * dx
        d2 = (py - qy) ** 2 + (px - qx) ** 2
        img[ylo:yhi, xlo:xhi] += a * np.exp(-d2 / (2.0 * width_std * width_std))


def blob_field(seed: int, H: int = 512, W: int = 512, n_blobs: int | None = None,
               t_range=(2.0, 8.0), amp_range=(0.2, 1.0), noise_std: float = 0.02,
               psf_sigma: float = 0.0) -> np.ndarray:
    """Bright blobs on a 0.1 background with additive Gaussian noise, fp32.

    Draw order: centres cy, cx ~ U[0, H), U[0, W) (continuous); std t ~
    U[t_range]; amplitude ~ U[amp_range]; then, if psf_sigma > 0, nothing is
    drawn for the blur (a Gaussian PSF, reflect borders); last the noise
    N(0, noise_std) per pixel.  The default blob count is 200 per 512 x 512
    pixels, scaled by area."""
    rng = np.random.default_rng(seed)
    if n_blobs is None:
        n_blobs = int(round(200 * H * W / (512 * 512)))
    cy = rng.uniform(0.0, H, n_blobs)
    cx = rng.uniform(0.0, W, n_blobs)
    t = rng.uniform(t_range[0], t_range[1], n_blobs)
    amp = rng.uniform(amp_range[0], amp_range[1], n_blobs)
    img = np.full((H, W), BACKGROUND, dtype=np.float64)
    render_blobs(img, cy, cx, t, amp)
    if psf_sigma > 0.0:
        from scipy.ndimage import gaussian_filter
        img = gaussian_filter(img, psf_sigma, mode="reflect", truncate=4.0)
    img += rng.normal(0.0, noise_std, size=(H, W))
    return img.astype(np.float32)


def plain_tile(seed: int = 0, H: int = 512, W: int = 512) -> np.ndarray:
    """512 x 512 fp32 workload: 200 blobs (std U[2,8] px, amplitude
    U[0.2,1]) on background 0.1 with N(0, 0.02) noise."""
    return blob_field(seed, H, W)


def sem_tile(seed: int = 0, psf_sigma: float = 0.0, H: int = 4096, W: int = 4096,
             poisson_lambda: float = 250.0) -> np.ndarray:
    """SEM-tile-shaped 8-bit workload.

    Texture: one Gaussian blob per 400 px^2 (std U[1.5, 6], amplitude
    U[0.1, 0.6]) and one ridge segment per 4000 px^2 (length U[16, 128],
    angle U[0, pi), cross-profile std 1 px, amplitude U[0.1, 0.6]) on
    background 0.1.  Defocus: Gaussian PSF of std psf_sigma (none if 0).
    Then clip to [0, 1], Poisson-like shot noise Poisson(lambda v)/lambda,
    clip again and quantise to round(255 v).

    Draw order: blob cy, cx, t, amp; ridge cy, cx, length, angle, amp; then
    the Poisson draws.  The texture does not depend on psf_sigma, so one seed
    gives the same scene at every defocus."""
    rng = np.random.default_rng(seed)
    nb = int(round(H * W / 400.0))
    nr = int(round(H * W / 4000.0))
    bcy = rng.uniform(0.0, H, nb)
    bcx = rng.uniform(0.0, W, nb)
    bt = rng.uniform(1.5, 6.0, nb)
    ba = rng.uniform(0.1, 0.6, nb)
    rcy = rng.uniform(0.0, H, nr)
    rcx = rng.uniform(0.0, W, nr)
    rl = rng.uniform(16.0, 128.0, nr)
    rth = rng.uniform(0.0, math.pi, nr)
    ra = rng.uniform(0.1, 0.6, nr)
    img = np.full((H, W), BACKGROUND, dtype=np.float64)
    render_blobs(img, bcy, bcx, bt, ba)
    render_ridges(img, rcy, rcx, rl, rth, ra)
    if psf_sigma > 0.0:
        from scipy.ndimage import gaussian_filter
        img = gaussian_filter(img, psf_sigma, mode="reflect", truncate=4.0)
    np.clip(img, 0.0, 1.0, out=img)
    img = rng.poisson(poisson_lambda * img) / poisson_lambda
    np.clip(img, 0.0, 1.0, out=img)
    return np.rint(255.0 * img).astype(np.uint8)


MIXED_SIZES = ((1024, 1024), (2048, 1536), (3072, 2048), (4096, 4096))


def mixed_batch_shapes(seed: int = 0, n: int = 64, sizes=MIXED_SIZES):
    """Sizes of the uneven batch (uniform over `sizes`) and a defocus
    psf_sigma ~ U[0, 4] per tile.  Draw order: size index, psf_sigma."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(sizes), n)
    psf = rng.uniform(0.0, 4.0, n)
    return [(sizes[i][0], sizes[i][1], float(p)) for i, p in zip(idx, psf)]


def mixed_batch(seed: int = 0, n: int = 64, sizes=MIXED_SIZES, scale: float = 1.0):
    """Uneven batch of fp32 tiles rendered like the plain workload (blob count
    scaled by area) with a per-tile PSF.  `scale` shrinks every side (tests use
    it to keep sizes small); tile i uses seed 1000 * seed + i."""
    tiles = []
    for i, (h, w, p) in enumerate(mixed_batch_shapes(seed, n, sizes)):
        hh, ww = max(1, int(round(h * scale))), max(1, int(round(w * scale)))
        tiles.append(blob_field(1000 * seed + i, hh, ww, psf_sigma=p))
    return tiles


def grad_batch(seed: int = 0, B: int = 8, H: int = 2048, W: int = 2048) -> np.ndarray:
    """B x H x W fp32 batch for the differentiable score, rendered like the
    plain workload; image b uses seed 100 * seed + b."""
    return np.stack([blob_field(100 * seed + b, H, W) for b in range(B)])


SERVE_SIZES = (512, 1024, 2048, 4096, 8192)
SERVE_PROBS = (0.1, 0.2, 0.3, 0.3, 0.1)


def arrivals(seed: int = 0, rate_hz: float = 50.0, duration_s: float = 60.0,
             sizes=SERVE_SIZES, probs=SERVE_PROBS):
    """Poisson request stream: exponential inter-arrival gaps at rate_hz over
    duration_s and a square size per request.  Draw order: all gaps (drawn in
    blocks until the horizon is passed), then one size index per request."""
    rng = np.random.default_rng(seed)
    times = []
    t = 0.0
    while True:
        gaps = rng.exponential(1.0 / rate_hz, 1024)
        for gap in gaps:
            t += gap
            if t >= duration_s:
                break
            times.append(t)
        if t >= duration_s:
            break
    idx = rng.choice(len(sizes), size=len(times), p=np.asarray(probs) / np.sum(probs))
    return np.asarray(times), [int(sizes[i]) for i in idx]
