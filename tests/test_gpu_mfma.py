"""GPU parity of the matrix-core path (RL_PATH_MFMA: PSF rows as banded matrices on
v_mfma_f32_16x16x32_bf16, values and weights split into three bfloat16 parts) against the
FP64 oracle, through the C ABI.

Cases: dense PSFs of every width the path takes (1 .. 17 taps per row, up to 64 rows), even
sizes, a PSF larger than the image (folds deeper than the image), ragged images (several
64 x 64 tiles plus tails, and images smaller than one tile), both boundaries, exact zeros,
full length (150 iterations), the thinned, TV and robust epilogues, and batch membership.
Bar: RTOL (1e-5) against the oracle; lock-step thinning counters bit for bit with the
float32 test taken on the GPU's own values; batches bit-identical to the job alone.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import RTOL, rel_err, run_gpu, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd import _abi as A  # noqa: E402
from paper_1304_7211_amd.job import BatchRunner, Job  # noqa: E402


def _obs(H, W, h, seed, noise="poisson"):
    return synth.observe(synth.latent_image(H, W, seed), h, noise, seed)


def _dense(kh, kw, seed):
    rng = np.random.default_rng(seed)
    h = rng.random((kh, kw))
    return (h / h.sum()).astype(np.float32)


PSFS = [
    ("dense15", lambda: synth.dense_random(15, 2)),
    ("dense9", lambda: synth.dense_random(9, 4)),
    ("dense4x6_even", lambda: _dense(4, 6, 5)),
    ("wide17x5", lambda: _dense(5, 17, 6)),
    ("line1x17", lambda: _dense(1, 17, 7)),
    ("tall64x3", lambda: _dense(64, 3, 8)),
    ("column9x1", lambda: _dense(9, 1, 9)),
    ("gaps", lambda: np.array([[0, .1, 0, .2, 0], [0, 0, 0, 0, 0], [.3, 0, 0, 0, .4]],
                              np.float32)),
]


@pytest.mark.parametrize("name,mk", PSFS, ids=[p[0] for p in PSFS])
@pytest.mark.parametrize("bc", ["reflect", "replicate"])
def test_mfma_matches_oracle(orc, name, mk, bc):
    h = mk()
    f = _obs(147, 203, h, 21)
    K = 8
    u, info = run_gpu(f, h, K, path="mfma", boundary=bc)
    assert info["path"] == A.RL_PATH_MFMA
    ref = orc.rl(f, h, K, bc)
    err = rel_err(u, ref)
    print(f"{name} {bc}: {err:.3g}")
    assert err <= RTOL


@pytest.mark.parametrize("shape", [(1, 1), (5, 3), (64, 64), (65, 129), (200, 17)])
def test_mfma_small_and_ragged_images(orc, shape):
    h = synth.dense_random(15, 3)  # larger than the smallest images: deep folds
    f = _obs(*shape, h, 22)
    u, info = run_gpu(f, h, 6, path="mfma")
    assert info["path"] == A.RL_PATH_MFMA
    assert rel_err(u, orc.rl(f, h, 6)) <= RTOL


def test_auto_picks_mfma_for_dense_and_not_for_sparse():
    f = to_dev(_obs(96, 80, synth.disc(3), 23))
    for h, want in ((synth.dense_random(15, 1), A.RL_PATH_MFMA),
                    (synth.oblique_line(31, 30.0), A.RL_PATH_RUNS),
                    (synth.disc(16), A.RL_PATH_RUNS)):
        job = Job(f, h)
        assert job.describe()["path"] == want
        job.close()


def test_mfma_full_length(orc):
    h = synth.dense_random(15, 11)
    f = _obs(300, 257, h, 24)
    K = 150
    u, _ = run_gpu(f, h, K)
    err = rel_err(u, orc.rl(f, h, K))
    print(f"dense15 K={K}: {err:.3g}")
    assert err <= RTOL


def test_mfma_exact_zeros(orc):
    h = synth.dense_random(9, 12)
    f = _obs(150, 140, h, 25)
    f[20:60, 30:90] = 0.0  # windows inside are all zero: r and u exactly 0 there
    u, _ = run_gpu(f, h, 5, path="mfma")
    ref = orc.rl(f, h, 5)
    assert np.array_equal(u == 0.0, ref == 0.0)
    assert rel_err(u, ref) <= RTOL


def test_mfma_close_to_the_vector_path():
    h = synth.dense_random(15, 13)
    f = _obs(190, 230, h, 26)
    a, _ = run_gpu(f, h, 20, path="mfma")
    b, _ = run_gpu(f, h, 20, path="runs")
    assert rel_err(a, b) <= RTOL


THIN = dict(mode="rel", tau=1e-3, hysteresis=3, reset_period=10, compact_period=10)


@pytest.mark.parametrize("k0", [10, 11, 13])
def test_mfma_thinned_lockstep(orc, k0):
    h = synth.dense_random(9, 14)
    f = _obs(150, 131, h, 27)
    st0 = orc.rl_thin(f, h, k0, THIN)
    u32, r32, cnt = st0["u"].astype(np.float32), st0["r"].astype(np.float32), st0["cnt"].copy()
    u, r, c = u32.astype(np.float64), r32.astype(np.float64), cnt.copy()
    full = O.is_full(k0, THIN["reset_period"])
    active = np.ones(f.shape, bool) if full else cnt < THIN["hysteresis"]
    n_act = orc.thin_step(f, u, r, c, h, k0, THIN)
    job = Job(to_dev(f), h, thin=THIN, path="mfma")
    assert job.describe()["path"] == A.RL_PATH_MFMA
    job.set_state(u=to_dev(u32), r=to_dev(r32), cnt=to_dev(cnt), k=k0)
    job.iterate(1)
    st = job.get_state()
    sched = job.thin_schedule()
    gu, gr, gc = st["u"].cpu().numpy(), st["r"].cpu().numpy(), st["cnt"].cpu().numpy()
    job.close()
    assert rel_err(gu, u) <= RTOL
    assert rel_err(gr[active], r[active]) <= RTOL
    assert np.array_equal(gu[~active], u32[~active])
    assert np.array_equal(gr[~active], r32[~active])
    assert sched[-1] == n_act
    below = orc.below_many(gu, u32, THIN["mode"], THIN["tau"])
    up = np.minimum(cnt.astype(np.int32) + 1, 255).astype(np.uint8)
    want = np.where(active, np.where(below, up, np.uint8(0)), cnt).astype(np.uint8)
    assert np.array_equal(gc, want)


def test_mfma_tv_and_robust(orc):
    h = synth.dense_random(9, 15)
    f = _obs(140, 150, h, 28)
    u, info = run_gpu(f, h, 8, path="mfma", tv=dict(lam=0.2, eps=1.0))
    assert info["path"] == A.RL_PATH_MFMA
    assert rel_err(u, orc.rl_tv(f, h, 8, 0.2, 1.0)) <= RTOL
    u, _ = run_gpu(f, h, 6, path="mfma", robust=dict(eps=0.05))
    assert rel_err(u, orc.rl_robust(f, h, 6, 0.05)) <= RTOL


def test_mfma_in_a_batch_is_bit_identical_to_alone():
    """Batch launches run the kernel with four wavefronts per tile, a job's own launches with
    eight (two blocks per wavefront instead of four): every block sees the same products in
    the same order, so the two shapes must agree bit for bit."""
    specs = [(synth.dense_random(15, 31), (300, 257), 12), (synth.disc(5), (128, 200), 9),
             (synth.dense_random(15, 32), (97, 131), 17), (synth.oblique_line(21, 60.0), (150, 150), 5)]
    fs = [to_dev(_obs(H, W, h, 40 + i)) for i, (h, (H, W), _) in enumerate(specs)]
    js = [Job(f, h) for f, (h, _, _) in zip(fs, specs)]
    BatchRunner(len(js)).iterate(js, [k for _, _, k in specs])
    outs = [j.result().cpu().numpy() for j in js]
    for j in js:
        j.close()
    for f, (h, _, K), o in zip(fs, specs, outs):
        a, _ = run_gpu(f.cpu().numpy(), h, K)
        assert np.array_equal(o.astype(np.float64), a)
