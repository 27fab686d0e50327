"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formulas: each compares it with a library
routine (scipy.ndimage, numpy.fft, numpy.pad), a closed form, an invariant, an exact
rational brute force on tiny inputs, or a value/trend the paper prints.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def _asym_psfs():
    return [synth.dense_random(5, 3), synth.oblique_line(11, 30.0), synth.dense_random(3, 9),
            synth.box_h(7), synth.box_v(5), synth.disc(4),
            np.array([[0.0, 0.25, 0.0], [0.5, 0.125, 0.0], [0.0, 0.0, 0.125]], np.float32)]


# ---- P1: convolution / correlation == scipy.ndimage (library routine) -------------------
@pytest.mark.parametrize("bc,mode", [("reflect", "reflect"), ("replicate", "nearest")])
@pytest.mark.parametrize("shape", [(37, 53), (5, 3), (1, 9), (12, 1)])
def test_p1_conv_corr_match_scipy(orc, bc, mode, shape):
    u = RNG.uniform(0.05, 1.0, shape)
    for h in _asym_psfs():
        h64 = h.astype(np.float64)
        ref_c = ndimage.convolve(u, h64, mode=mode)
        ref_r = ndimage.correlate(u, h64, mode=mode)
        np.testing.assert_allclose(orc.conv(u, h64, bc), ref_c, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(orc.corr(u, h64, bc), ref_r, rtol=1e-13, atol=1e-15)


# ---- P6: brute force with numpy.pad continuation, tiny images, deep folds, even sizes ----
@pytest.mark.parametrize("bc,padmode", [("reflect", "symmetric"), ("replicate", "edge")])
def test_p6_bruteforce_tiny_deep_folds(orc, bc, padmode):
    for H in range(1, 6):
        for W in range(1, 7):
            u = RNG.integers(0, 256, size=(H, W)).astype(np.float64)
            for (kh, kw) in [(1, 1), (1, 2), (2, 1), (3, 4), (1, 11), (9, 1), (4, 4), (2, 13)]:
                h = RNG.integers(0, 4, size=(kh, kw)).astype(np.float64)
                oy, ox = kh // 2, kw // 2
                P = 20
                up = np.pad(u, P, mode=padmode)
                ref_c = np.zeros((H, W))
                ref_r = np.zeros((H, W))
                for i in range(kh):
                    for j in range(kw):
                        dy, dx = i - oy, j - ox
                        ref_c += h[i, j] * up[P - dy:P - dy + H, P - dx:P - dx + W]
                        ref_r += h[i, j] * up[P + dy:P + dy + H, P + dx:P + dx + W]
                # integer data and weights: every sum is exact in FP64
                assert np.array_equal(orc.conv(u, h, bc), ref_c), (H, W, kh, kw)
                assert np.array_equal(orc.corr(u, h, bc), ref_r), (H, W, kh, kw)


def test_fold_matches_numpy_pad(orc):
    for n in range(1, 7):
        i = np.arange(-25, n + 25)
        sym = np.pad(np.arange(n), 25, mode="symmetric")
        edge = np.pad(np.arange(n), 25, mode="edge")
        assert [orc.fold(k, n, "reflect") for k in i] == list(sym)
        assert [orc.fold(k, n, "replicate") for k in i] == list(edge)


# ---- P12: direct convolution == FFT convolution of the padded image (library routine) ---
def test_p12_conv_matches_fft(orc):
    u = RNG.uniform(0.0, 1.0, (64, 48))
    for h in [synth.disc(7), synth.oblique_line(21, 65.0), synth.dense_random(15, 1)]:
        h64 = h.astype(np.float64)
        kh, kw = h.shape
        oy, ox = kh // 2, kw // 2
        up = np.pad(u, ((kh - 1 - oy, oy), (kw - 1 - ox, ox)), mode="symmetric")
        Hp, Wp = up.shape
        F = np.fft.rfft2(up) * np.fft.rfft2(h64, s=(Hp, Wp))
        full = np.fft.irfft2(F, s=(Hp, Wp))
        ref = full[kh - 1:kh - 1 + u.shape[0], kw - 1:kw - 1 + u.shape[1]]
        np.testing.assert_allclose(orc.conv(u, h64), ref, rtol=0, atol=1e-12)


# ---- P2: delta PSF is the identity (closed form) ------------------------------------------
@pytest.mark.parametrize("bc", ["reflect", "replicate"])
def test_p2_delta_identity(orc, bc):
    f = synth.observe(synth.latent_image(40, 33, 3), synth.delta(), "poisson", 3)
    u = orc.rl(f, synth.delta(), 7, bc)
    assert np.array_equal(u, f.astype(np.float64))


# ---- P3: 1x1 image and constant images (closed forms) -----------------------------------
@pytest.mark.parametrize("bc", ["reflect", "replicate"])
def test_p3_single_pixel_and_constant(orc, bc):
    for h in _asym_psfs():
        f = np.array([[0.37]], np.float32)
        u0 = np.array([[0.81]])
        u1 = orc.rl(f, h, 1, bc, u0=u0)
        assert abs(u1[0, 0] - float(f[0, 0])) < 1e-15
        c = np.full((9, 14), 0.25, np.float32)
        np.testing.assert_allclose(orc.rl(c, h, 5, bc), 0.25, rtol=1e-14)


# ---- P4: u = g is a fixed point when f = g*h exactly (blur made by scipy) ----------------
@pytest.mark.parametrize("bc,mode", [("reflect", "reflect"), ("replicate", "nearest")])
def test_p4_fixed_point(orc, bc, mode):
    g = synth.latent_image(48, 40, 4)
    for h in _asym_psfs():
        h64 = h.astype(np.float64)
        f = ndimage.convolve(g, h64, mode=mode)
        u = orc.rl(f, h64, 6, bc, u0=g)
        # first step: r = f/(g*h) = 1 and h^* * 1 = s = sum(h) at every pixel, so u^1 = s g;
        # later steps: r = 1/s, h^* * r = 1, so u^K = s g for all K >= 1 (the float32 taps
        # sum to 1 only up to a few ulp)
        np.testing.assert_allclose(u, g * h64.sum(), rtol=1e-12)


# ---- P5: flux preservation (invariant) ---------------------------------------------------
def test_p5_flux_reflect_symmetric(orc):
    f = synth.observe(synth.latent_image(50, 61, 5), synth.disc(5), "poisson", 5)
    for h in [synth.disc(5), synth.box_h(9), synth.box_v(13), synth.box_rect(3, 5)]:
        u = orc.rl(f, h, 20, "reflect")
        assert abs(u.sum() - f.astype(np.float64).sum()) < 1e-11 * f.sum()


def test_p5_flux_zero_margin_any_psf(orc):
    f = np.zeros((60, 64))
    f[15:45, 16:48] = RNG.uniform(0.1, 1.0, (30, 32))
    for h in [synth.oblique_line(11, 30.0), synth.dense_random(7, 2)]:
        # support stays away from the border for these few iterations: K * radius < margin
        u = orc.rl(f, h, 2, "reflect")
        assert abs(u.sum() - f.sum()) < 1e-12 * f.sum()


# ---- P7: adjointness <u*h, r> = <u, h^* * r> (invariant) --------------------------------
def test_p7_adjoint(orc):
    u = RNG.uniform(0, 1, (31, 29))
    r = RNG.uniform(0, 1, (31, 29))
    for h in [synth.disc(4), synth.box_h(9), synth.box_rect(5, 3)]:
        lhs = np.vdot(orc.conv(u, h), r)
        rhs = np.vdot(u, orc.corr(r, h))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # asymmetric PSF away from the border
    u2 = np.zeros((40, 40))
    u2[12:28, 12:28] = RNG.uniform(0, 1, (16, 16))
    r2 = np.zeros((40, 40))
    r2[12:28, 12:28] = RNG.uniform(0, 1, (16, 16))
    h = synth.dense_random(7, 5)
    assert abs(np.vdot(orc.conv(u2, h), r2) - np.vdot(u2, orc.corr(r2, h))) < 1e-12


# ---- exact rational brute force of plain RL on tiny inputs --------------------------------
def _exact_rl(f, h, K, padmode):
    H, W = f.shape
    kh, kw = h.shape
    oy, ox = kh // 2, kw // 2
    P = 12
    yi = np.pad(np.arange(H), P, mode=padmode)
    xi = np.pad(np.arange(W), P, mode=padmode)
    F = [[Fraction(float(f[y, x])) for x in range(W)] for y in range(H)]
    Hf = [[Fraction(float(h[i, j])) for j in range(kw)] for i in range(kh)]
    u = [row[:] for row in F]
    for _ in range(K):
        r = [[None] * W for _ in range(H)]
        for y in range(H):
            for x in range(W):
                v = sum((Hf[i][j] * u[yi[P + y - (i - oy)]][xi[P + x - (j - ox)]]
                         for i in range(kh) for j in range(kw)), Fraction(0))
                r[y][x] = F[y][x] / v if v > 0 else Fraction(0)
        u = [[u[y][x] * sum((Hf[i][j] * r[yi[P + y + (i - oy)]][xi[P + x + (j - ox)]]
                             for i in range(kh) for j in range(kw)), Fraction(0))
              for x in range(W)] for y in range(H)]
    return np.array([[float(v) for v in row] for row in u])


@pytest.mark.parametrize("bc,padmode", [("reflect", "symmetric"), ("replicate", "edge")])
def test_exact_rational_rl_tiny(orc, bc, padmode):
    f = np.array([[0.5, 0.25, 1.0, 0.0], [0.75, 0.125, 0.5, 0.375], [1.0, 0.625, 0.25, 0.5]],
                 np.float32)
    for h in [np.array([[0.25, 0.5, 0.125, 0.125]], np.float32),
              np.array([[0.0, 0.25], [0.5, 0.125], [0.125, 0.0]], np.float32),
              np.array([[0.5], [0.25], [0.25], [0.0], [0.0]], np.float32)]:
        ref = _exact_rl(f, h, 2, padmode)
        np.testing.assert_allclose(orc.rl(f, h, 2, bc), ref, rtol=1e-14, atol=1e-300)


# ---- thinning: the float32 convergence test on hand-picked values (closed form) -----------
def test_below_closed_form(orc):
    e = 2.0 ** -13
    # ABS: |a-b| < tau, strict
    assert not orc.below(1.0 + e, 1.0, "abs", e)
    assert orc.below(1.0 + e, 1.0, "abs", e * 1.5)
    assert orc.below(1.0, 1.0 + e, "abs", e * 1.5)
    # REL: |a-b| < tau * b
    assert orc.below(4.0 + 4 * e, 4.0, "rel", 1.5 * e)
    assert not orc.below(4.0 + 4 * e, 4.0, "rel", e)
    assert not orc.below(2.0, 1.0, "abs", 0.5)
    # tau = 0 never freezes, even an unchanged pixel; a pixel stuck at zero is converged
    assert not orc.below(1.0, 1.0, "abs", 0.0)
    assert orc.below(0.0, 0.0, "rel", 1e-4)
    assert orc.below(0.5, 0.5, "rel", 1e-4)


# ---- thinned step: what frozen pixels keep (Section 4, eq. 4-5) -----------------------------
def _thin_state(shape, hyst, seed):
    """A seeded mid-run state: positive u^k and stale r, counters with a block of frozen
    pixels and scattered frozen ones (cnt >= hyst) among active ones."""
    rng = np.random.default_rng(seed)
    H, W = shape
    u = rng.uniform(0.1, 1.0, shape)
    r = rng.uniform(0.5, 1.5, shape)
    f = rng.uniform(0.05, 1.0, shape)
    frozen = rng.random(shape) < 0.35
    frozen[H // 4:H // 2, W // 3:2 * W // 3] = True
    cnt = np.where(frozen, rng.integers(hyst, 60, shape), rng.integers(0, hyst, shape))
    return f, u, r, cnt.astype(np.uint8)


def _thin_step_expected(f, u_prev, r_old, cnt0, h, active, thin, mode):
    """eq. 4-5 written with scipy: active pixels get a fresh ratio and update, computed with
    the stale ratio of the frozen neighbours; frozen pixels keep u, r and cnt."""
    h64 = h.astype(np.float64)
    v = ndimage.convolve(u_prev, h64, mode=mode)
    r_mixed = np.where(active, np.where(v > 0, f / np.where(v > 0, v, 1.0), 0.0), r_old)
    u_new = np.where(active, u_prev * ndimage.correlate(r_mixed, h64, mode=mode), u_prev)
    a32, b32 = u_new.astype(np.float32), u_prev.astype(np.float32)
    d = np.abs((a32 - b32).astype(np.float32))
    t = (np.float32(thin["tau"]) * b32).astype(np.float32) if thin["mode"] == "rel" \
        else np.float32(thin["tau"])
    below = (d < t) | ((a32 == 0) & (b32 == 0))
    cnt = np.where(active, np.where(below, np.minimum(cnt0.astype(int) + 1, 255), 0), cnt0)
    return u_new, r_mixed, cnt.astype(np.uint8)


@pytest.mark.parametrize("bc,mode", [("reflect", "reflect"), ("replicate", "nearest")])
@pytest.mark.parametrize("k", [13, 20])
def test_thin_step_frozen_pixels(orc, bc, mode, k):
    thin = dict(mode="rel", tau=0.06, hysteresis=3, reset_period=10, compact_period=10)
    for h in (synth.disc(3), synth.oblique_line(9, 30.0), synth.dense_random(5, 3)):
        f, u0, r0, c0 = _thin_state((41, 37), thin["hysteresis"], 77 + k)
        full = oracle.is_full(k, thin["reset_period"])
        active = np.ones(f.shape, bool) if full else c0 < thin["hysteresis"]
        assert full or 0 < active.sum() < f.size
        want_u, want_r, want_c = _thin_step_expected(f, u0, r0, c0, h, active, thin, mode)
        u, r, c = u0.copy(), r0.copy(), c0.copy()
        n = orc.thin_step(f, u, r, c, h, k, thin, bc)
        assert n == int(active.sum())
        # frozen pixels: u, r and counter untouched, bit for bit
        assert np.array_equal(u[~active], u0[~active])
        assert np.array_equal(r[~active], r0[~active])
        assert np.array_equal(c[~active], c0[~active])
        np.testing.assert_allclose(u, want_u, rtol=1e-13, atol=0)
        np.testing.assert_allclose(r, want_r, rtol=1e-13, atol=0)
        # the decisions are far from the threshold at this tau on random data, and both
        # outcomes occur
        assert np.array_equal(c, want_c)
        assert 0 < np.count_nonzero(c[active] == 0) < active.sum()


# ---- thinned step under the block rule (freeze decisions per B x B block) ------------------
def _block_state(shape, B, hyst, seed):
    """A seeded mid-run state whose counters are constant on B x B blocks: some blocks
    frozen (cnt >= hyst), the others active."""
    rng = np.random.default_rng(seed)
    H, W = shape
    f = rng.uniform(0.05, 1.0, shape)
    u = rng.uniform(0.1, 1.0, shape)
    r = rng.uniform(0.5, 1.5, shape)
    TY, TX = -(-H // B), -(-W // B)
    tc = np.where(rng.random((TY, TX)) < 0.4, rng.integers(hyst, 60, (TY, TX)),
                  rng.integers(0, hyst, (TY, TX))).astype(np.uint8)
    cnt = np.kron(tc, np.ones((B, B), np.uint8))[:H, :W].copy()
    return f, u, r, cnt, tc


def _block_step_expected(f, u_prev, r_old, tc, B, h, thin, mode, full):
    """The block rule written with scipy: every pixel of an active block gets a fresh ratio
    and update (computed with the stale ratio of frozen blocks); a block's counter counts up
    only if the float32 test holds on all of its pixels."""
    H, W = f.shape
    tact = np.ones(tc.shape, bool) if full else tc < thin["hysteresis"]
    active = np.kron(tact, np.ones((B, B), bool))[:H, :W]
    h64 = h.astype(np.float64)
    v = ndimage.convolve(u_prev, h64, mode=mode)
    r_mixed = np.where(active, np.where(v > 0, f / np.where(v > 0, v, 1.0), 0.0), r_old)
    u_new = np.where(active, u_prev * ndimage.correlate(r_mixed, h64, mode=mode), u_prev)
    a32, b32 = u_new.astype(np.float32), u_prev.astype(np.float32)
    d = np.abs((a32 - b32).astype(np.float32))
    t = (np.float32(thin["tau"]) * b32).astype(np.float32) if thin["mode"] == "rel" \
        else np.float32(thin["tau"])
    below = (d < t) | ((a32 == 0) & (b32 == 0))
    tc_new = tc.copy()
    for ty in range(tc.shape[0]):
        for tx in range(tc.shape[1]):
            if tact[ty, tx]:
                ok = below[ty * B:(ty + 1) * B, tx * B:(tx + 1) * B].all()
                tc_new[ty, tx] = min(int(tc[ty, tx]) + 1, 255) if ok else 0
    cnt = np.kron(tc_new, np.ones((B, B), np.uint8))[:H, :W]
    return u_new, r_mixed, cnt, active


@pytest.mark.parametrize("bc,mode", [("reflect", "reflect"), ("replicate", "nearest")])
@pytest.mark.parametrize("k", [13, 20])
def test_block_rule_step(orc, bc, mode, k):
    B = 4
    # a large tau so that both block decisions occur on random data
    thin = dict(mode="rel", tau=0.25, hysteresis=3, reset_period=10, compact_period=10,
                block=B)
    for h in (synth.disc(2), synth.oblique_line(9, 30.0)):
        f, u0, r0, c0, tc = _block_state((23, 30), B, thin["hysteresis"], 91 + k)
        full = oracle.is_full(k, thin["reset_period"])
        want_u, want_r, want_c, active = _block_step_expected(f, u0, r0, tc, B, h, thin,
                                                               mode, full)
        u, r, c = u0.copy(), r0.copy(), c0.copy()
        n = orc.thin_step(f, u, r, c, h, k, thin, bc)
        assert n == int(active.sum())
        assert np.array_equal(u[~active], u0[~active])
        assert np.array_equal(r[~active], r0[~active])
        np.testing.assert_allclose(u, want_u, rtol=1e-13, atol=0)
        np.testing.assert_allclose(r, want_r, rtol=1e-13, atol=0)
        assert np.array_equal(c, want_c)
        # both decisions occur among the active blocks
        ca = c[active]
        assert 0 < np.count_nonzero(ca == 0) < ca.size


def test_block_rule_of_1x1_blocks_is_the_pixel_rule(orc):
    """Blocks of one pixel decide exactly as the per-pixel rule (Section 4)."""
    thin = dict(mode="rel", tau=1e-3, hysteresis=2, reset_period=5, compact_period=5)
    h = synth.disc(3)
    f = synth.observe(synth.latent_image(30, 41, 12), h, "poisson", 12)
    fd = f.astype(np.float64)
    a = [fd.copy(), np.zeros_like(fd), np.zeros(f.shape, np.uint8)]
    b = [fd.copy(), np.zeros_like(fd), np.zeros(f.shape, np.uint8)]
    for k in range(23):
        na = orc.thin_step(fd, a[0], a[1], a[2], h, k, thin)
        nb = orc.thin_step_blocks(fd, b[0], b[1], b[2], h, k, thin, 1)
        assert na == nb
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert 0 < np.count_nonzero(a[2] >= 2) < f.size


def test_block_rule_tau_zero_is_plain_rl(orc):
    h = synth.disc(2)
    f = synth.observe(synth.latent_image(37, 29, 13), h, "poisson", 13)
    thin = dict(mode="abs", tau=0.0, hysteresis=1, reset_period=10, compact_period=10,
                block=8)
    out = orc.rl_thin(f, h, 12, thin)
    assert np.array_equal(out["u"], orc.rl(f, h, 12))
    assert (out["active"] == f.size).all()


def test_below_many_matches_below(orc):
    rng = np.random.default_rng(9)
    b = rng.uniform(0.0, 2.0, 400).astype(np.float32)
    a = (b * (1 + rng.uniform(-3e-4, 3e-4, 400))).astype(np.float32)
    a[:5] = 0.0
    b[:3] = 0.0
    for mode, tau in (("rel", 1e-4), ("abs", 1e-4), ("rel", 0.0)):
        got = orc.below_many(a, b, mode, tau)
        want = [orc.below(x, y, mode, tau) for x, y in zip(a, b)]
        assert got.tolist() == want


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---- thinning schedule, closed form with the delta PSF -------------------------------------
def test_thin_schedule_delta_closed_form(orc):
    rows = _golden_rows("thin_schedule_delta.txt")
    f = synth.observe(synth.latent_image(12, 17, 6), synth.delta(), "poisson", 6)
    N = f.size
    for hyst, row in zip((5, 1), rows):
        want = np.array([int(v) for v in row]) * N
        out = orc.rl_thin(f, synth.delta(), len(want), dict(mode="rel", tau=1e-4,
                          hysteresis=hyst, reset_period=10, compact_period=10))
        assert np.array_equal(out["active"], want)
        assert np.array_equal(out["u"], f.astype(np.float64))


# ---- P8: threshold 0 is exactly plain RL (Table 2, first two rows) -------------------------
@pytest.mark.parametrize("mode", ["abs", "rel"])
def test_p8_tau_zero_is_plain(orc, mode):
    h = synth.disc(3)
    f = synth.observe(synth.latent_image(30, 26, 7), h, "poisson", 7)
    plain = orc.rl(f, h, 12)
    th = orc.rl_thin(f, h, 12, dict(mode=mode, tau=0.0, hysteresis=1, reset_period=10,
                                     compact_period=1))
    assert np.array_equal(th["u"], plain)
    assert (th["active"] == f.size).all()


# ---- P9: omitted fraction bounded by the reset rule, monotone in tau (Table 2 trends) ------
def test_p9_table2_trends(orc):
    rows = _golden_rows("table2_trends.txt")
    omitted_paper = [float(r[1]) for r in rows]
    assert omitted_paper[0] == 0.0 and max(omitted_paper) < 90.0
    assert all(b >= a for a, b in zip(omitted_paper, omitted_paper[1:]))
    h = synth.disc(4)
    f = synth.observe(synth.latent_image(48, 48, 8), h, "poisson", 8)
    ref = orc.rl(f, h, 100)
    prev_omit, prev_err = -1.0, -1.0
    for tau in [0.0, 0.005, 0.02, 0.1, 0.5]:
        # paper mode: absolute threshold on the 0..255 grey scale, images scaled to [0, 1]
        th = orc.rl_thin(f, h, 100, dict(mode="abs", tau=tau / 255.0, hysteresis=1,
                                          reset_period=10, compact_period=1))
        omit = 100.0 * (1.0 - th["active"].sum() / (100 * f.size))
        err = float(np.abs(th["u"] - ref).max())
        assert omit < 90.0
        assert omit >= prev_omit
        assert err >= prev_err
        prev_omit, prev_err = omit, err
    assert prev_omit > 50.0


# ---- P10: disc support sizes (Table 1 / Section 5 reading) --------------------------------
def test_p10_disc_support():
    for r, n in _golden_rows("disc_support.txt"):
        h = synth.disc(int(r))
        assert np.count_nonzero(h) == int(n)
        ints, _ = oracle.psf_runs(h)
        assert len(ints) == 2 * int(r) + 1
        # half-width of row dy is floor(sqrt(r^2 - dy^2))
        for dy, x0, x1 in ints:
            hw = int(np.floor(np.sqrt(int(r) ** 2 - dy * dy)))
            assert (x0, x1) == (-hw, hw)


def test_psf_runs_definition():
    h = np.array([[0, 1, 1, 2, 0, 3], [0, 0, 0, 0, 0, 0], [5, 5, 5, 5, 5, 5]], np.float32)
    ints, ws = oracle.psf_runs(h)
    assert ints.tolist() == [[-1, -2, -1], [-1, 0, 0], [-1, 2, 2], [1, -3, 2]]
    assert ws.tolist() == [1.0, 2.0, 3.0, 5.0]


def test_rebuild_schedule():
    ks = [k for k in range(35) if oracle.is_rebuild(k, 10, 10)]
    assert ks == [1, 11, 21, 31]
    ks = [k for k in range(13) if oracle.is_rebuild(k, 10, 1)]
    assert ks == [1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 12]
    ks = [k for k in range(25) if oracle.is_rebuild(k, 0, 10)]
    assert ks == [1, 11, 21]


# ---- mutation check: every planted mistake in the oracle is caught by some pin ------------
def _pins_pass(o):
    """A compact subset of the pins above, run against an oracle variant."""
    u = RNG.uniform(0.05, 1.0, (11, 13))
    try:
        for h in _asym_psfs()[:3] + [_asym_psfs()[-1]]:
            h64 = h.astype(np.float64)
            if not np.allclose(o.conv(u, h64), ndimage.convolve(u, h64, mode="reflect"),
                               rtol=1e-13):
                return False
            if not np.allclose(o.corr(u, h64), ndimage.correlate(u, h64, mode="reflect"),
                               rtol=1e-13):
                return False
            f = ndimage.convolve(u, h64, mode="reflect")
            if not np.allclose(o.rl(f, h64, 3, u0=u), u * h64.sum(), rtol=1e-12):
                return False
        # robust variant: weights against the gradient of its energy (scipy rel_entr)
        from scipy.special import rel_entr
        h = _unit(synth.disc(2))
        f = ndimage.convolve(u, h, mode="reflect") * RNG.uniform(0.7, 1.3, u.shape)
        uu = RNG.uniform(0.2, 1.0, u.shape)

        def energy(x):
            v = ndimage.convolve(x, h, mode="reflect")
            return float(np.sum(2.0 * np.sqrt(v - f + rel_entr(f, v) + 0.0025)))

        num, den = o.robust_terms(f, uu, h, 0.05)
        ep = np.zeros_like(uu)
        ep[5, 6] = 1e-6
        g = (energy(uu + ep) - energy(uu - ep)) / 2e-6
        if not abs((den - num)[5, 6] - g) <= 1e-5 * max(1.0, abs(g)):
            return False
        # thinned step: frozen pixels keep u and their stale ratio (eq. 4-5)
        thin = dict(mode="rel", tau=0.06, hysteresis=3, reset_period=10, compact_period=10)
        hd = synth.disc(2)
        f, u0, r0, c0 = _thin_state((17, 15), 3, 5)
        active = c0 < 3
        want_u, want_r, _ = _thin_step_expected(f, u0, r0, c0, hd, active, thin, "reflect")
        uu, rr, cc = u0.copy(), r0.copy(), c0.copy()
        o.thin_step(f, uu, rr, cc, hd, 13, thin)
        if not (np.array_equal(uu[~active], u0[~active]) and
                np.array_equal(rr[~active], r0[~active]) and
                np.allclose(uu, want_u, rtol=1e-13, atol=0)):
            return False
        # block rule: a block counts up only when all of its pixels pass the test
        tb = dict(mode="rel", tau=0.25, hysteresis=3, reset_period=10, compact_period=10,
                  block=4)
        f, u0, r0, c0, tc = _block_state((23, 30), 4, 3, 104)
        _, _, want_c, _ = _block_step_expected(f, u0, r0, tc, 4, hd, tb, "reflect", False)
        uu, rr, cc = u0.copy(), r0.copy(), c0.copy()
        o.thin_step(f, uu, rr, cc, hd, 13, tb)
        if not np.array_equal(cc, want_c):
            return False
        e = 2.0 ** -13
        if o.below(1.0 + e, 1.0, "abs", e) or not o.below(1.0 + e, 1.0, "abs", 1.5 * e):
            return False
        if o.below(4.0 + 4 * e, 4.0, "rel", e) or not o.below(4.0 + 4 * e, 4.0, "rel", 1.5 * e):
            return False
    except Exception:
        return False
    return True


def test_planted_mistakes_are_caught():
    assert _pins_pass(oracle.Oracle(0))
    for m in range(1, 13):
        assert not _pins_pass(oracle.Oracle(m)), f"mutant {m} passed the pins"


# ---- TV-regularised variant (Dey et al. 2006; named as carrying over in Section 2) --------
def test_tv_zero_lambda_is_plain_rl(orc):
    h = synth.disc(3)
    f = synth.observe(synth.latent_image(40, 33, 8), h, "poisson", 8)
    assert np.array_equal(orc.rl_tv(f, h, 6, 0.0, 1e-3), orc.rl(f, h, 6))


def test_tv_div_closed_forms(orc):
    eps = 1e-3
    # constant image: no gradient anywhere
    assert np.array_equal(orc.tv_div(np.full((6, 7), 0.3), eps), np.zeros((6, 7)))
    # ramp along x with slope a: the flux a/m leaves the first column and enters the last
    H, W, a = 5, 9, 0.2
    u = np.tile(a * np.arange(W, dtype=np.float64), (H, 1))
    m = np.sqrt(a * a + eps * eps)
    want = np.zeros((H, W))
    want[:, 0] = a / m
    want[:, -1] = -a / m
    assert np.allclose(orc.tv_div(u, eps), want, rtol=0, atol=1e-15)
    # single spike in a flat image: hand-derived values at the spike and its neighbours
    u = np.zeros((7, 8))
    u[3, 4] = 1.0
    d = orc.tv_div(u, eps)
    s1, s2 = np.sqrt(1 + eps * eps), np.sqrt(2 + eps * eps)
    # n = (-1/s2, -1/s2) at the spike, (1/s1, 0) left of it, (0, 1/s1) above it, else 0
    assert abs(d[3, 4] - (-2 / s2 - 2 / s1)) < 1e-14
    assert abs(d[3, 3] - 1 / s1) < 1e-14                 # left neighbour: its own nx
    assert abs(d[2, 4] - 1 / s1) < 1e-14                 # upper neighbour: its own ny
    assert abs(d[3, 5] - 1 / s2) < 1e-14                 # right: minus the spike's nx
    assert abs(d[4, 4] - 1 / s2) < 1e-14                 # lower: minus the spike's ny
    others = np.ones(d.shape, bool)
    others[3, 3:6] = False
    others[2, 4] = others[4, 4] = False
    assert np.abs(d[others]).max() < 1e-15
    assert abs(d.sum()) < 1e-14                          # zero flux: the sum telescopes


def test_tv_summation_by_parts(orc):
    """Backward divergence is the negative adjoint of the forward gradient with zero flux at
    the edges: sum div(n) v = -sum n . grad v, for n = grad u / |grad u|_eps."""
    rng = np.random.default_rng(5)
    u = rng.random((13, 11))
    v = rng.random((13, 11))
    eps = 0.05
    div = orc.tv_div(u, eps)
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    gx[:, :-1] = np.diff(u, axis=1)
    gy[:-1, :] = np.diff(u, axis=0)
    m = np.sqrt(gx ** 2 + gy ** 2 + eps ** 2)
    vx = np.zeros_like(v)
    vy = np.zeros_like(v)
    vx[:, :-1] = np.diff(v, axis=1)
    vy[:-1, :] = np.diff(v, axis=0)
    lhs = float((div * v).sum())
    rhs = -float(((gx / m) * vx + (gy / m) * vy).sum())
    assert abs(lhs - rhs) < 1e-12


def test_tv_constant_fixed_point(orc):
    h = synth.disc(4)
    f = np.full((30, 26), 0.4)
    u = orc.rl_tv(f, h, 5, 0.1, 1e-3)
    assert np.allclose(u, f, rtol=0, atol=1e-15)


# ---- robustified data term: I-divergence weights ---------------------------------------
def test_robust_idiv_matches_rel_entr(orc):
    """d(v, f) = v - f - f ln(v/f) is v - f + rel_entr(f, v) (scipy), also at f = 0."""
    from scipy.special import rel_entr
    v = RNG.uniform(1e-3, 3.0, 200)
    f = np.concatenate([RNG.uniform(1e-3, 3.0, 150), np.zeros(50)])
    for vi, fi in zip(v, f):
        want = vi - fi + float(rel_entr(fi, vi))
        assert abs(orc.idiv(vi, fi) - want) <= 1e-12 * max(1.0, abs(want))
    assert orc.idiv(0.7, 0.7) == 0.0
    assert orc.idiv(0.0, 0.5) == 0.0  # v <= 0: no information


def _unit(h):
    h = np.asarray(h, np.float64)
    return h / h.sum()


def test_robust_constant_weights_are_plain_rl(orc):
    """eps far above every divergence: the weights are constant and cancel, so the update
    is plain RL's (PSFs normalised in FP64: a sum off 1 would scale every step by it)."""
    for h in [synth.disc(3), synth.oblique_line(9, 40.0), synth.box_rect(3, 5)]:
        h = _unit(h)
        f = synth.observe(synth.latent_image(40, 36, 8), h, "poisson", 8).astype(np.float64)
        a = orc.rl_robust(f, h, 4, 1e8)
        b = orc.rl(f, h, 4)
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


def test_robust_fixed_points(orc):
    """Constant images, and the true image of noise-free data (f = g*h by scipy, u^0 = g):
    d = 0 everywhere, constant weights, u^1 = u^0."""
    h = _unit(synth.disc(3))
    c = np.full((30, 34), 0.37)
    np.testing.assert_allclose(orc.rl_robust(c, h, 3, 0.05), c, rtol=1e-13)
    g = RNG.uniform(0.2, 1.0, (30, 34))
    f = ndimage.convolve(g, h, mode="reflect")
    np.testing.assert_allclose(orc.rl_robust(f, h, 1, 0.05, u0=g), g, rtol=1e-12)


@pytest.mark.parametrize("psf,points", [
    ("disc2", [(0, 0), (5, 7), (12, 21), (23, 3), (17, 17)]),       # mirror-symmetric: all
    ("oblique7", [(6, 6), (10, 14), (15, 9)]),                      # interior only
])
def test_robust_gradient_identity(orc, psf, points):
    """den - num is the gradient of E(u) = sum 2 sqrt(d(u*h, f) + eps^2), checked against
    central differences of E computed with scipy (convolve, rel_entr).  The correlation is
    the exact adjoint of the reflected convolution for mirror-symmetric PSFs everywhere,
    for others away from the image edges."""
    from scipy.special import rel_entr
    h = _unit(synth.disc(2) if psf == "disc2" else synth.oblique_line(7, 30.0))
    eps = 0.05
    f = synth.observe(synth.latent_image(24, 22, 9), synth.disc(2), "poisson", 9).astype(np.float64)
    u = RNG.uniform(0.1, 1.0, f.shape)

    def energy(uu):
        v = ndimage.convolve(uu, h, mode="reflect")
        d = v - f + rel_entr(f, v)
        return float(np.sum(2.0 * np.sqrt(d + eps * eps)))

    num, den = orc.robust_terms(f, u, h, eps)
    for (y, x) in points:
        e = np.zeros_like(u)
        e[y, x] = 1e-6
        g = (energy(u + e) - energy(u - e)) / 2e-6
        assert abs((den - num)[y, x] - g) <= 1e-5 * max(1.0, abs(g)), (y, x, (den - num)[y, x], g)
