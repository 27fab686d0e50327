"""Point-spread-function constructors (Section 3, Figure 1 (a)-(e); Section 5 test PSFs).

Every constructor builds the PSF in float64, normalises it to unit sum in float64 and
casts to float32.  The float32 array is *the* PSF handed to both the oracle and the GPU
library, so both sides see exactly the same taps (their sum differs from 1 by a few ulp,
which is part of the input, not an error of either side).

Array convention: a kh x kw float32 array, origin (oy, ox) = (kh // 2, kw // 2).  A tap
h[i][j] sits at offset (i - oy, j - ox).
"""
import math

import numpy as np


def normalise_to_f32(h64):
    h64 = np.asarray(h64, dtype=np.float64)
    s = h64.sum()
    if not s > 0:
        raise ValueError("PSF must have a positive sum")
    return (h64 / s).astype(np.float32)


def delta():
    """The identity PSF [1]."""
    return np.ones((1, 1), dtype=np.float32)


def box_h(length):
    """Linear motion blur along scan-lines (Figure 1(a)): a 1 x L box."""
    return normalise_to_f32(np.ones((1, int(length))))


def box_v(length):
    """Linear motion blur along columns: an L x 1 box."""
    return normalise_to_f32(np.ones((int(length), 1)))


def box_rect(my, mx):
    """Rectangular PSF of constant density (Figure 1(b))."""
    return normalise_to_f32(np.ones((int(my), int(mx))))


def disc(radius):
    """Uniform defocus disc (Figure 1(c)).

    Support {(dy, dx): dx^2 + dy^2 <= r^2}, diameter d = 2r + 1.  This reading of the
    paper's "diameter 9 / 17" test PSFs (Section 5) gives 49 and 197 support pixels,
    which is what the list-filter timings of Table 1 imply.
    """
    r = int(radius)
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    return normalise_to_f32((xx * xx + yy * yy <= r * r).astype(np.float64))


def disc_support_size(radius):
    """Number of support pixels of ``disc(radius)`` (counted from the array)."""
    return int(np.count_nonzero(disc(radius)))


def oblique_line(length, angle_deg, samples_per_px=64):
    """Antialiased linear motion blur of ``length`` pixels at ``angle_deg`` (Figure 1(e)).

    The paper gives no rasteriser for oblique lines.  This one splats S = 64 * L equally
    spaced midpoint samples t in (-L/2, L/2) along the direction (cos a, -sin a) in
    (column, row) coordinates bilinearly onto the grid, accumulates in float64,
    normalises and casts to float32.  The bounding box has half-extents
    ceil(L/2 |cos a|) + 1 columns and ceil(L/2 |sin a|) + 1 rows, so the array is odd-sized
    and centred on the origin.
    """
    L = float(length)
    a = math.radians(float(angle_deg))
    c, s = math.cos(a), math.sin(a)
    hx = int(math.ceil(L / 2 * abs(c))) + 1
    hy = int(math.ceil(L / 2 * abs(s))) + 1
    h = np.zeros((2 * hy + 1, 2 * hx + 1), dtype=np.float64)
    n = int(samples_per_px * L)
    t = (np.arange(n, dtype=np.float64) + 0.5) / n * L - L / 2
    px = t * c          # column offset
    py = -t * s         # row offset (rows grow downwards)
    x0 = np.floor(px).astype(np.int64)
    y0 = np.floor(py).astype(np.int64)
    fx = px - x0
    fy = py - y0
    for dyi, dxi, wgt in ((0, 0, (1 - fy) * (1 - fx)), (0, 1, (1 - fy) * fx),
                          (1, 0, fy * (1 - fx)), (1, 1, fy * fx)):
        np.add.at(h, (y0 + dyi + hy, x0 + dxi + hx), wgt)
    # trim all-zero border rows / columns while keeping the array centred
    while h.shape[0] > 1 and not h[0].any() and not h[-1].any():
        h = h[1:-1]
    while h.shape[1] > 1 and not h[:, 0].any() and not h[:, -1].any():
        h = h[:, 1:-1]
    return normalise_to_f32(h)


def dense_random(size, seed):
    """Dense non-negative random PSF (size x size, U[0,1] entries), normalised."""
    rng = np.random.default_rng(seed)
    return normalise_to_f32(rng.uniform(0.0, 1.0, size=(int(size), int(size))))
