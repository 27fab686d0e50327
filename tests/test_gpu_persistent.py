"""GPU checks of the persistent schedule (one launch per rl_iterate call, tiles ordered by
an atomic ticket and synchronised through per-tile step counters).

Each tile is computed by the same code as in the two-pass schedule, so results must be
bit-identical to it; they must also match the FP64 oracle within RTOL.  Cases cover
ragged tile grids, halos deeper than the image (every tile depends on every other),
both boundaries, split iteration counts, and the rejection of thinned jobs.
"""
import numpy as np
import pytest

import synth
from gpu_util import RTOL, rel_err, run_gpu, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd._abi import RLError  # noqa: E402
from paper_1304_7211_amd.job import Job  # noqa: E402


def _obs(H, W, h, seed):
    return synth.observe(synth.latent_image(H, W, seed), h, "poisson", seed)


PSFS = [("disc6", lambda: synth.disc(6), "runs"),
        ("oblique31", lambda: synth.oblique_line(31, 30.0), "runs"),
        ("box_h15", lambda: synth.box_h(15), "box_axis"),
        ("box_v21", lambda: synth.box_v(21), "box_axis"),
        ("dense9", lambda: synth.dense_random(9, 6), "direct"),
        ("rect5x7", lambda: synth.box_rect(5, 7), "runs")]


@pytest.mark.parametrize("name,mk,path", PSFS, ids=[p[0] for p in PSFS])
@pytest.mark.parametrize("bc", ["reflect", "replicate"])
def test_persistent_equals_two_pass(orc, name, mk, path, bc):
    h = mk()
    for shape in [(147, 203), (64, 64), (300, 41), (5, 9)]:
        f = _obs(*shape, h, 13)
        K = 7
        u_p, info = run_gpu(f, h, K, boundary=bc, path=path, schedule="persistent")
        assert info["schedule"] == 4
        u_t, _ = run_gpu(f, h, K, boundary=bc, path=path, schedule="two_pass")
        assert np.array_equal(u_p, u_t), (name, bc, shape)
        assert rel_err(u_p, orc.rl(f, h, K, bc)) <= RTOL, (name, bc, shape)


def test_persistent_split_calls_and_stats(orc):
    h = synth.oblique_line(25, 110.0)
    f = _obs(520, 333, h, 5)
    fd = to_dev(f)
    a = Job(fd, h, schedule="persistent")
    b = Job(fd, h, schedule="two_pass")
    for n in (3, 1, 8, 2):
        a.iterate(n)
        b.iterate(n)
    ua, st = a.result(stats=True)
    ub = b.result()
    assert st.iters_done == 14 and st.schedule == 4
    assert torch.equal(ua, ub)
    assert rel_err(ua.cpu().numpy(), orc.rl(f, h, 14)) <= RTOL
    a.close()
    b.close()


def test_persistent_large_image_strips(orc):
    # strips of 4 (small image default) and 8 (explicit), several hundred tiles
    h = synth.disc(10)
    f = _obs(1024, 768, h, 21)
    fd = to_dev(f)
    ref_t = Job(fd, h, schedule="two_pass", tuning=dict(strip=8))
    ref_t.iterate(6)
    ut = ref_t.result().cpu().numpy()
    ref_t.close()
    for strip in (4, 8):
        j = Job(fd, h, schedule="persistent", tuning=dict(strip=strip))
        j.iterate(6)
        u = j.result().cpu().numpy()
        j.close()
        if strip == 8:
            assert np.array_equal(u, ut)
        assert rel_err(u, orc.rl(f, h, 6)) <= RTOL, strip


def test_persistent_rejects_thinning():
    h = synth.disc(4)
    f = _obs(100, 90, h, 3)
    with pytest.raises(RLError):
        Job(to_dev(f), h, schedule="persistent", thin=dict(mode="rel", tau=1e-3))


def test_wait_limit_failure_surfaces():
    """Failure path, forced from the host: with a negative wait limit every dependency
    wait of a persistent launch gives up at once (the kernel's own bounded wait: the launch
    raises its abort flag and every workgroup leaves, so the kernel ends normally).  The
    incomplete result must be reported by rl_result (with and without statistics) and by
    rl_get_state, i.e. by Job.result(), Job.stats() and Job.get_state()."""
    from paper_1304_7211_amd import _abi as A
    h = synth.disc(6)
    f = _obs(300, 280, h, 95)
    prev = A.rl_debug_spin_limit(-1)
    try:
        job = Job(to_dev(f), h, path="runs", schedule="persistent")
        job.iterate(4)
        with pytest.raises(RLError) as e:
            job.result()
        assert e.value.status == A.RL_E_DEVICE and "wait limit" in str(e.value)
        with pytest.raises(RLError):
            job.stats()
        with pytest.raises(RLError):
            job.get_state()
        job.close()
    finally:
        A.rl_debug_spin_limit(prev)
    torch.cuda.synchronize()
    # the limit is restored: a new job completes and matches two-pass bit for bit
    ok = Job(to_dev(f), h, path="runs", schedule="persistent")
    ok.iterate(4)
    u = ok.result().cpu().numpy()
    ok.close()
    ref, _ = run_gpu(f, h, 4, path="runs", schedule="two_pass")
    assert np.array_equal(u.astype(np.float64), ref)
