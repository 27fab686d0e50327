"""GPU parity of plain RL (Section 2, eq. 3) against the FP64 oracle, through the C ABI.

Bar: delta PSF bit-exact (P2); box/run kernels bit-exact on integer images with 0/1
weights where every float32 sum is exact (P6); everything else within RTOL = 1e-5 of the
oracle under the max-relative metric of gpu_util.
"""
import numpy as np
import pytest

import synth
from gpu_util import RTOL, rel_err, run_gpu, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def _obs(H, W, h, seed, noise="poisson"):
    return synth.observe(synth.latent_image(H, W, seed), h, noise, seed)


# ---- P2: the delta PSF is the identity, bit for bit -------------------------------------
@pytest.mark.parametrize("bc", ["reflect", "replicate"])
@pytest.mark.parametrize("shape", [(1, 1), (7, 300), (130, 67)])
def test_delta_bit_exact(bc, shape):
    f = _obs(*shape, synth.delta(), 5)
    u, info = run_gpu(f, synth.delta(), 6, boundary=bc)
    assert info["path"] == 1  # AUTO routes a 1x1 PSF to DIRECT
    assert np.array_equal(u, f.astype(np.float64))


# ---- every path x PSF family x boundary at ragged sizes (several tiles + tails) ----------
CASES = [
    ("box_h15", lambda: synth.box_h(15), ["direct", "box_axis", "runs"]),
    ("box_v41", lambda: synth.box_v(41), ["direct", "box_axis", "runs"]),
    ("box_v6_even", lambda: synth.box_v(6), ["direct", "box_axis", "runs"]),
    ("disc10", lambda: synth.disc(10), ["direct", "runs"]),
    ("oblique31", lambda: synth.oblique_line(31, 30.0), ["direct", "runs"]),
    ("oblique47_steep", lambda: synth.oblique_line(47, 75.0), ["runs"]),
    ("dense15", lambda: synth.dense_random(15, 2), ["direct", "runs"]),
    ("rect5x7", lambda: synth.box_rect(5, 7), ["runs", "box_rect", "box_sat"]),
    ("rect4x6_even", lambda: synth.box_rect(4, 6), ["direct", "box_rect", "box_sat"]),
    ("rect2x2", lambda: synth.box_rect(2, 2), ["box_rect", "box_sat"]),
    ("rect31x17", lambda: synth.box_rect(31, 17), ["runs", "box_rect", "box_sat"]),
    ("rect_margin", lambda: np.pad(synth.box_rect(3, 6), ((2, 0), (0, 3))), ["box_rect", "box_sat"]),
]


@pytest.mark.parametrize("name,mk,paths", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("bc", ["reflect", "replicate"])
def test_paths_match_oracle(orc, name, mk, paths, bc):
    h = mk()
    f = _obs(147, 203, h, 17)
    K = 8
    ref = orc.rl(f, h, K, bc)
    for path in paths:
        scheds = ["two_pass", "resident"] if path == "box_axis" else ["auto"]
        for sched in scheds:
            u, info = run_gpu(f, h, K, boundary=bc, path=path, schedule=sched)
            err = rel_err(u, ref)
            print(f"{name} {bc} {path}/{sched}: err {err:.3g} {info}")
            assert err <= RTOL, (path, sched, err)


# ---- tiny images: folds deeper than the image --------------------------------------------
@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (3, 2), (5, 9)])
def test_tiny_deep_folds(orc, shape):
    for h in [synth.box_h(15), synth.box_v(9), synth.disc(4), synth.oblique_line(11, 30.0),
              synth.box_rect(5, 7)]:
        f = _obs(*shape, synth.delta(), 3)
        f = np.maximum(f, 0.05).astype(np.float32)
        ref = orc.rl(f, h, 4)
        for path in (["direct", "runs"] + (["box_axis"] if min(h.shape) == 1 else [])
                     + (["box_rect", "box_sat"] if min(h.shape) > 1 and h.min() > 0 else [])):
            u, _ = run_gpu(f, h, 4, path=path)
            assert rel_err(u, ref) <= RTOL, (shape, h.shape, path)


# ---- P6: integer images, 0/1 weights: sums are exact, so kernels are bit-exact ------------
def test_integer_images_bit_exact(orc):
    rng = np.random.default_rng(4)
    f = rng.integers(1, 256, size=(70, 90)).astype(np.float32)
    for h01 in [np.ones((1, 9), np.float32), np.ones((7, 1), np.float32),
                (synth.disc(3) > 0).astype(np.float32), np.ones((5, 7), np.float32)]:
        # one conv only: v = f*h with integer weights; with K=1 u^1 = u^0 * corr(f/v)
        # ratio and update round, so compare the forward convolution through a lock-step
        # property: for u0 = f and f' = f*h (exact integers), r = 1 exactly and
        # u^1 = f * sum(h) exactly.
        fb = orc.conv(f.astype(np.float64), h01).astype(np.float32)
        assert np.array_equal(fb.astype(np.float64), orc.conv(f.astype(np.float64), h01))
        rect = min(h01.shape) > 1 and h01.min() > 0
        for path in (["direct", "runs"] + (["box_axis"] if min(h01.shape) == 1 else [])
                     + (["box_rect", "box_sat"] if rect else [])):
            scheds = ["two_pass", "resident"] if path == "box_axis" else ["auto"]
            for sched in scheds:
                u, _ = run_gpu(fb, h01, 1, path=path, schedule=sched, u0=to_dev(f))
                assert np.array_equal(u, f.astype(np.float64) * h01.sum()), (h01.shape, path, sched)


# ---- configuration 1: 128 x 128, box 15, Poisson 255, 50 iterations, direct path ----------
def test_config1_full(orc):
    job = synth.job_for_config(1)[0]
    ref = orc.rl(job["f"], job["psf"], job["iters"])
    for path in ["direct", "box_axis", "runs"]:
        u, info = run_gpu(job["f"], job["psf"], job["iters"], path=path)
        err = rel_err(u, ref)
        print(f"config1 {path}: err {err:.3g}")
        assert err <= RTOL


# ---- determinism: the same inputs give bit-identical outputs ------------------------------
def test_deterministic():
    h = synth.oblique_line(31, 30.0)
    f = _obs(300, 257, h, 9)
    a, _ = run_gpu(f, h, 5)
    b, _ = run_gpu(f, h, 5)
    assert np.array_equal(a, b)


# ---- statistics: FP64 flux and the f check ------------------------------------------------
def test_stats_flux_and_invalid_f(orc):
    from paper_1304_7211_amd.job import Job
    h = synth.disc(5)
    f = _obs(120, 100, h, 12)
    job = Job(to_dev(f), h)
    job.iterate(7)
    u, st = job.result(stats=True)
    assert st.iters_done == 7 and st.f_invalid == 0
    assert abs(st.flux - float(u.double().sum().item())) < 1e-9 * st.flux
    # REFLECT with a mirror-symmetric PSF preserves the flux (P5)
    assert abs(st.flux - float(f.astype(np.float64).sum())) < 1e-5 * st.flux
    job.close()
    bad = f.copy()
    bad[3, 4] = -1.0
    job = Job(to_dev(bad), h)
    job.iterate(1)
    from paper_1304_7211_amd._abi import RLError
    with pytest.raises(RLError):
        job.result(stats=True)
    job.close()


# ---- fused iteration kernel (conv, ratio, corr, update in one launch) ---------------------
FUSED_PSFS = [synth.disc(6), synth.oblique_line(21, 30.0), synth.dense_random(15, 4),
              synth.box_h(9), synth.box_v(12),
              np.array([[0.0, 0.3, 0.0, 0.0], [0.1, 0.2, 0.0, 0.25], [0.0, 0.0, 0.0, 0.15]],
                       np.float32)]


@pytest.mark.parametrize("bc", ["reflect", "replicate"])
@pytest.mark.parametrize("K", [1, 6, 7])
def test_fused_matches_oracle(orc, bc, K):
    for h in FUSED_PSFS:
        f = _obs(147, 203, h, 19)
        ref = orc.rl(f, h, K, bc)
        u, info = run_gpu(f, h, K, boundary=bc, schedule="fused")
        assert info["schedule"] == 3
        assert rel_err(u, ref) <= RTOL, (h.shape, bc, K)


def test_fused_state_roundtrip_and_split_iterations(orc):
    from paper_1304_7211_amd.job import Job
    h = synth.oblique_line(15, 120.0)
    f = _obs(96, 130, h, 23)
    a = Job(to_dev(f), h, schedule="fused")
    a.iterate(5)
    st = a.get_state()
    assert st["k"] == 5
    b = Job(to_dev(f), h, schedule="fused")
    b.set_state(u=st["u"], k=5)
    b.iterate(4)
    a.iterate(4)
    ua, ub = a.result().cpu().numpy(), b.result().cpu().numpy()
    assert np.array_equal(ua, ub)
    assert rel_err(ua, orc.rl(f, h, 9)) <= RTOL
    a.close()
    b.close()


def test_fused_rejects_small_images():
    from paper_1304_7211_amd._abi import RLError
    from paper_1304_7211_amd.job import Job
    h = synth.disc(3)
    f = _obs(40, 100, h, 2)
    with pytest.raises(RLError):
        Job(to_dev(f), h, schedule="fused")
