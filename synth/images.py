"""Seeded synthetic images shaped like the paper's workloads.

The paper's test image (a 256 x 256 photograph, Section 5) is not available, so a
seeded generator stands in for it: piecewise-constant shapes (edges are what RL
sharpens) over a smooth low-amplitude background, blurred with the job's PSF under
the half-sample-symmetric ("reflect") boundary, plus Poisson or Gaussian noise
(Section 1, eq. 1 and the noise types named after it).

Recipe of ``latent_image(H, W, seed)``:
  * g = 0.1 everywhere;
  * max(8, H*W // 4096) shapes painted in order, each an axis-aligned rectangle
    (sides U[4, min(H,W)/3]) or a disc (radius U[3, min(H,W)/6]) with value U[0.1, 1];
  * plus 0.05 sin(2 pi (x/Px + y/Py) + phi), Px, Py ~ U[32, 256], phi ~ U[0, 2 pi);
  * clipped to [0.02, 1].
All draws come from numpy's PCG64 seeded with ``seed``.
"""
import numpy as np
from scipy import signal


def latent_image(H, W, seed):
    rng = np.random.default_rng(seed)
    H, W = int(H), int(W)
    g = np.full((H, W), 0.1, dtype=np.float64)
    m = min(H, W)
    n_shapes = max(8, (H * W) // 4096)
    for _ in range(n_shapes):
        val = rng.uniform(0.1, 1.0)
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        if rng.uniform() < 0.5:
            hi = max(4.0, m / 3.0)
            sy = rng.uniform(4.0, hi)
            sx = rng.uniform(4.0, hi)
            y0, y1 = int(max(0, cy - sy / 2)), int(min(H, cy + sy / 2))
            x0, x1 = int(max(0, cx - sx / 2)), int(min(W, cx + sx / 2))
            g[y0:y1, x0:x1] = val
        else:
            rad = rng.uniform(3.0, max(3.0, m / 6.0))
            y0, y1 = int(max(0, cy - rad)), int(min(H, cy + rad + 1))
            x0, x1 = int(max(0, cx - rad)), int(min(W, cx + rad + 1))
            if y1 <= y0 or x1 <= x0:
                continue
            yy, xx = np.mgrid[y0:y1, x0:x1]
            inside = (yy + 0.5 - cy) ** 2 + (xx + 0.5 - cx) ** 2 <= rad * rad
            g[y0:y1, x0:x1][inside] = val
    px = rng.uniform(32, 256)
    py = rng.uniform(32, 256)
    phi = rng.uniform(0, 2 * np.pi)
    yy, xx = np.mgrid[0:H, 0:W]
    g += 0.05 * np.sin(2 * np.pi * (xx / px + yy / py) + phi)
    return np.clip(g, 0.02, 1.0)


def blur_reflect(g, h):
    """b = g * h with the half-sample-symmetric boundary, in float64.

    The image is padded by the PSF extent with numpy's 'symmetric' mode (c b a | a b c,
    i.e. period-2N folding) and convolved with ``scipy.signal.fftconvolve`` ('valid'),
    so the result at (y, x) is sum_ij h[i][j] g[fold(y-(i-oy))][fold(x-(j-ox))].
    """
    g = np.asarray(g, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    kh, kw = h.shape
    oy, ox = kh // 2, kw // 2
    pad = ((kh - 1 - oy, oy), (kw - 1 - ox, ox))
    gp = np.pad(g, pad, mode="symmetric")
    return signal.fftconvolve(gp, h, mode="valid")


def observe(g, h, noise, seed, peak=255.0, sigma=0.01):
    """Observed image f = g*h + noise as float32 (non-negative).

    noise = "poisson": f = Poisson(peak * b) / peak; "gaussian": f = max(b + N(0, sigma^2), 0);
    "none": f = b.
    """
    rng = np.random.default_rng(seed + 7919)
    b = np.maximum(blur_reflect(g, h), 0.0)
    if noise == "poisson":
        f = rng.poisson(peak * b) / peak
    elif noise == "gaussian":
        f = np.maximum(b + rng.normal(0.0, sigma, size=b.shape), 0.0)
    elif noise == "none":
        f = b
    else:
        raise ValueError(noise)
    return np.ascontiguousarray(f, dtype=np.float32)
