"""GPU parity of thinned RL under the block rule (a refinement of Section 4's adaptive
update rule: freeze decisions per B x B block aligned at (0, 0), every pixel of an active
block updated, frozen blocks keep u and their stale ratio, eq. 4-5).

Lock-step protocol as for the per-pixel rule: a float32 state (u^k, r, counters, k) goes to
both sides and each performs one iteration.  Floats agree within RTOL.  The decision of
each active block is the float32 convergence test of Section 4 taken on the GPU's own
u^{k+1} and u^k for every pixel of the block (oracle ``below_many``), so the expected block
counters follow from the GPU's floats and must match bit for bit everywhere.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import RTOL, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd.job import Job  # noqa: E402

HYST = 3


def block_view(a, B):
    """(TY, TX, B, B) view of a per-pixel array padded with True (edge blocks are cut)."""
    H, W = a.shape
    TY, TX = -(-H // B), -(-W // B)
    pad = np.ones((TY * B, TX * B), dtype=bool)
    pad[:H, :W] = a
    return pad.reshape(TY, B, TX, B).transpose(0, 2, 1, 3)


def expand(cb, B, shape):
    return np.kron(cb, np.ones((B, B), dtype=np.uint8))[:shape[0], :shape[1]].astype(np.uint8)


def seeded_state(orc, f, h, B, k0, seed):
    """u, r after k0 block-rule iterations of the oracle (float32), and block counters
    drawn at random in [0, HYST + 1] so that frozen and active blocks both occur."""
    thin = dict(mode="rel", tau=1e-3, hysteresis=HYST, reset_period=10, compact_period=10,
                block=B)
    out = orc.rl_thin(f, h, k0, thin)
    H, W = f.shape
    rng = np.random.default_rng(seed)
    cb = rng.integers(0, HYST + 2, size=(-(-H // B), -(-W // B))).astype(np.uint8)
    return out["u"].astype(np.float32), out["r"].astype(np.float32), cb


def pick_tau(orc, f, h, u32, r32, cnt, k0, B):
    """A relative threshold near the median of the active blocks' largest relative change in
    one step, so that blocks pass and fail the test (float32, from the oracle's step)."""
    u = u32.astype(np.float64)
    r = r32.astype(np.float64)
    c = cnt.copy()
    thin = dict(mode="rel", tau=1e-30, hysteresis=HYST, reset_period=10, compact_period=10,
                block=B)
    orc.thin_step(f, u, r, c, h, k0, thin)
    rel = np.abs(u - u32) / np.maximum(u32.astype(np.float64), 1e-30)
    H, W = f.shape
    TY, TX = -(-H // B), -(-W // B)
    pad = np.zeros((TY * B, TX * B))
    pad[:H, :W] = rel
    bmax = pad.reshape(TY, B, TX, B).max(axis=(1, 3))
    return float(np.float32(np.median(bmax[bmax > 0])))


def lockstep(orc, B, k0, h, shape, path="auto", seed=0):
    H, W = shape
    f = synth.observe(synth.latent_image(H, W, 40 + seed), h, "poisson", 40 + seed)
    u32, r32, cb = seeded_state(orc, f, h, B, k0, seed)
    cnt = expand(cb, B, f.shape)
    tau = pick_tau(orc, f, h, u32, r32, cnt, k0, B)
    thin = dict(mode="rel", tau=tau, hysteresis=HYST, reset_period=10, compact_period=10,
                block=B)
    full = O.is_full(k0, thin["reset_period"])
    act_b = np.ones(cb.shape, bool) if full else cb < HYST
    active = expand(act_b.astype(np.uint8), B, f.shape).astype(bool)
    # oracle side: one step from the float32 state
    u = u32.astype(np.float64)
    r = r32.astype(np.float64)
    c = cnt.copy()
    n_act = orc.thin_step(f, u, r, c, h, k0, thin)
    assert n_act == int(active.sum())
    # GPU side
    job = Job(to_dev(f), h, thin=thin, path=path)
    job.set_state(u=to_dev(u32), r=to_dev(r32), cnt=to_dev(cnt), k=k0)
    job.iterate(1)
    st = job.get_state()
    sched = job.thin_schedule()
    info = job.describe()
    torch.cuda.synchronize()
    gu = st["u"].cpu().numpy()
    gr = st["r"].cpu().numpy()
    gc = st["cnt"].cpu().numpy()
    job.close()
    assert info["tile_h"] == 64 and info["tile_w"] == 64
    assert rel_err(gu, u) <= RTOL
    assert rel_err(gr[active], r[active]) <= RTOL
    assert np.array_equal(gu[~active], u32[~active])
    assert np.array_equal(gr[~active], r32[~active])
    assert sched[-1] == n_act
    # expected block counters from the float32 test on the GPU's own values
    below = orc.below_many(gu, u32, "rel", tau)
    passed = block_view(below, B).all(axis=(2, 3))
    up = np.minimum(cb.astype(np.int32) + 1, 255).astype(np.uint8)
    want_b = np.where(act_b, np.where(passed, up, np.uint8(0)), cb)
    want = expand(want_b, B, f.shape)
    mism = gc != want
    assert not mism.any(), f"{int(mism.sum())} counters differ from the float32 block decision"
    n_pass = int((act_b & passed).sum())
    n_fail = int((act_b & ~passed).sum())
    print(f"B={B} k0={k0} path={info['path']} active blocks {int(act_b.sum())} "
          f"(pass {n_pass}, fail {n_fail}), frozen {int((~act_b).sum())}")
    assert n_pass > 0 and n_fail > 0
    if not full:
        assert (~act_b).any()


@pytest.mark.parametrize("B", [8, 16, 32, 64])
@pytest.mark.parametrize("k0", [9, 10, 13])
def test_lockstep_disc(orc, B, k0):
    """Sliding kernel (disc runs), a ragged image whose width is not a multiple of 4
    (per-output epilogue)."""
    lockstep(orc, B, k0, synth.disc(4), (150, 131), seed=B + k0)


@pytest.mark.parametrize("B", [8, 16, 64])
def test_lockstep_four_wide(orc, B):
    """Width a multiple of 4: the four-wide epilogue carries the block rule."""
    lockstep(orc, B, 13, synth.disc(3), (136, 200), seed=100 + B)


@pytest.mark.parametrize("path,h", [
    ("auto", "oblique"), ("auto", "vbox"), ("direct", "disc"), ("box_rect", "rect"),
    ("box_sat", "rect"), ("mfma", "dense")], ids=["span", "cols", "direct", "rect", "sat", "mfma"])
def test_lockstep_kernels(orc, path, h):
    psf = {"oblique": synth.oblique_line(9, 30.0), "vbox": synth.box_v(9),
           "disc": synth.disc(3), "rect": synth.box_rect(5, 7),
           "dense": synth.dense_random(7, 5)}[h]
    lockstep(orc, 16, 13, psf, (131, 150), path=path, seed=200)


@pytest.mark.parametrize("B", [8, 64])
def test_free_running(orc, B):
    """K iterations from u^0 = f.  Decisions near the threshold may differ between the
    float32 run and the FP64 oracle, so masks are compared by disagreement rate."""
    h = synth.disc(4)
    # tau 2e-2: the oracle freezes 70 % (B = 8) and 14 % (B = 64) of pixel-iterations
    thin = dict(mode="rel", tau=2e-2, hysteresis=3, reset_period=10, compact_period=10,
                block=B)
    f = synth.observe(synth.latent_image(160, 144, 41), h, "poisson", 41, peak=1000.0)
    K = 40
    ref = orc.rl_thin(f, h, K, thin)
    job = Job(to_dev(f), h, thin=thin)
    job.iterate(K)
    st = job.get_state()
    u = st["u"].cpu().numpy()
    cnt = st["cnt"].cpu().numpy()
    sched = np.array(job.thin_schedule())
    stats = job.stats()
    job.close()
    frozen = ref["cnt"] >= thin["hysteresis"]
    mask_dis = float(np.mean((cnt >= thin["hysteresis"]) != frozen))
    omitted = 1.0 - ref["active"].sum() / (K * f.size)
    err = rel_err(u, ref["u"])
    print(f"B={B} free-running: max err {err:.3g}, mask disagreement {mask_dis:.3g}, "
          f"omitted {omitted:.3f}")
    assert omitted > 0.05
    assert stats.skipped_px_iters == K * f.size - int(sched.sum())
    assert mask_dis < 2e-2
    # as for the per-pixel rule: a block that freezes on one side only misses at most
    # R - 1 updates before the next full step, each below tau relative; two such episodes
    # plus a 2 tau margin for the neighbours: 2 (R - 1) tau + 2 tau
    bound = 2 * (thin["reset_period"] - 1) * thin["tau"] + 2 * thin["tau"]
    assert err < bound, (err, bound)


def test_tau_zero_is_plain_bit_exact(orc):
    """tau = 0 never freezes: the block rule equals plain RL bit for bit (same strip)."""
    h = synth.disc(5)
    f = synth.observe(synth.latent_image(190, 172, 42), h, "poisson", 42)
    a = Job(to_dev(f), h, tuning=dict(strip=8))
    b = Job(to_dev(f), h, thin=dict(mode="rel", tau=0.0, hysteresis=1, reset_period=10,
                                    compact_period=1, block=16))
    a.iterate(25)
    b.iterate(25)
    ua, ub = a.result(), b.result()
    torch.cuda.synchronize()
    assert torch.equal(ua, ub)
    assert rel_err(ub.cpu().numpy(), orc.rl(f, h, 25)) <= RTOL
    a.close()
    b.close()


def test_state_roundtrip_and_list():
    """rl_set_state takes each block's counter from its top-left pixel; rl_get_state returns
    every pixel with its block's counter; the kept pixel list is flatnonzero of the
    expanded mask."""
    B = 16
    h = synth.disc(3)
    f = synth.observe(synth.latent_image(100, 90, 43), h, "poisson", 43)
    thin = dict(mode="rel", tau=1e-3, hysteresis=2, reset_period=10, compact_period=10,
                block=B, keep_list=True)
    job = Job(to_dev(f), h, thin=thin)
    rng = np.random.default_rng(5)
    cnt = rng.integers(0, 4, size=f.shape).astype(np.uint8)
    job.set_state(cnt=to_dev(cnt), k=11)
    got = job.get_state()["cnt"].cpu().numpy()
    want = expand(cnt[::B, ::B], B, f.shape)
    assert np.array_equal(got, want)
    job.set_state(cnt=to_dev(want), k=1)
    job.iterate(1)  # k = 1 is a rebuild point
    lst = job.active_list().cpu().numpy()
    assert np.array_equal(lst, np.flatnonzero(want.reshape(-1) < 2))
    job.close()


def test_batch_equals_alone():
    """A block-rule job advanced inside a batch is bit-identical to the job alone."""
    from paper_1304_7211_amd.job import iterate_batch
    h1, h2 = synth.disc(4), synth.oblique_line(11, 60.0)
    f1 = synth.observe(synth.latent_image(140, 170, 44), h1, "poisson", 44)
    f2 = synth.observe(synth.latent_image(200, 120, 45), h2, "poisson", 45)
    thin = dict(mode="rel", tau=2e-3, hysteresis=3, reset_period=10, compact_period=10,
                block=32)
    alone = []
    for f, h in ((f1, h1), (f2, h2)):
        j = Job(to_dev(f), h, thin=thin)
        j.iterate(30)
        alone.append(j.get_state())
        j.close()
    jobs = [Job(to_dev(f1), h1, thin=thin), Job(to_dev(f2), h2, thin=thin)]
    iterate_batch(jobs, [30, 30])
    for j, a in zip(jobs, alone):
        s = j.get_state()
        assert torch.equal(s["u"], a["u"]) and torch.equal(s["cnt"], a["cnt"])
        j.close()
