"""GPU parity of RL with the robustified data term (weights 1/sqrt(d + eps^2) of the
I-divergence d of u*h from f) against the FP64 oracle.

* one iteration from a seeded state on every tiled path (lock-step: both sides start from
  the same float32 u), and a few free-running iterations;
* a huge eps reduces to plain RL;
* batches and graph replay change nothing (bit-identical to the job alone);
* exact zeros in f.
"""
import numpy as np
import pytest

import synth
from gpu_util import RTOL, rel_err, run_gpu, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd.job import BatchRunner, Job  # noqa: E402

CASES = [("disc5", lambda: synth.disc(5), ["runs", "direct"]),
         ("oblique21", lambda: synth.oblique_line(21, 40.0), ["runs"]),
         ("box_h15", lambda: synth.box_h(15), ["box_axis"]),
         ("rect5x7", lambda: synth.box_rect(5, 7), ["box_rect", "box_sat"]),
         ("dense9", lambda: synth.dense_random(9, 3), ["direct"])]


def _obs(H, W, h, seed):
    return synth.observe(synth.latent_image(H, W, seed), h, "poisson", seed)


@pytest.mark.parametrize("name,mk,paths", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("bc", ["reflect", "replicate"])
def test_robust_lockstep_and_free(orc, name, mk, paths, bc):
    h = mk()
    f = _obs(110, 140, h, 61)
    rng = np.random.default_rng(61)
    u0 = (f * (1.0 + 0.2 * rng.standard_normal(f.shape))).clip(0.01).astype(np.float32)
    eps = 0.05
    ref1 = orc.rl_robust(f, h, 1, eps, bc, u0=u0)
    ref6 = orc.rl_robust(f, h, 6, eps, bc)
    for path in paths:
        u, info = run_gpu(f, h, 1, boundary=bc, path=path, u0=to_dev(u0), robust=dict(eps=eps))
        e1 = rel_err(u, ref1)
        u, _ = run_gpu(f, h, 6, boundary=bc, path=path, robust=dict(eps=eps))
        e6 = rel_err(u, ref6)
        print(f"{name} {bc} {path}: one step {e1:.3g}, 6 free-running {e6:.3g}")
        assert e1 <= RTOL, (path, e1)
        assert e6 <= RTOL, (path, e6)


def test_robust_huge_eps_is_plain_rl(orc):
    h = synth.disc(4)
    f = _obs(90, 100, h, 62)
    ref = orc.rl(f, h, 8)
    for path in ["runs", "direct"]:
        u, _ = run_gpu(f, h, 8, path=path, robust=dict(eps=1e6))
        # the weights' factor cancels, up to the PSF's float32 sum per step
        assert rel_err(u, ref) <= RTOL, path


def test_robust_batch_and_graph_identical():
    h = synth.oblique_line(15, 20.0)
    f = _obs(150, 170, h, 63)
    fd = to_dev(f)
    alone = Job(fd, h, robust=dict(eps=0.05))
    alone.iterate(9)
    ua = alone.result().cpu().numpy()
    alone.close()
    g = Job(fd, h, robust=dict(eps=0.05), tuning=dict(graph_iters=4))
    g.iterate(9)
    assert np.array_equal(g.result().cpu().numpy(), ua)
    g.close()
    h2 = synth.disc(6)
    f2 = _obs(200, 120, h2, 64)
    jobs = [Job(to_dev(f2), h2), Job(fd, h, robust=dict(eps=0.05))]
    BatchRunner(2).iterate(jobs, [5, 9])
    assert np.array_equal(jobs[1].result().cpu().numpy(), ua)
    plain = Job(to_dev(f2), h2)
    plain.iterate(5)
    assert torch.equal(jobs[0].result(), plain.result())
    for j in jobs + [plain]:
        j.close()


def test_robust_zeros(orc):
    h = synth.box_rect(4, 6)
    f = _obs(96, 120, h, 65)
    f[20:50, 30:80] = 0.0
    ref = orc.rl_robust(f, h, 5, 0.05)
    for path in ["box_rect", "box_sat", "runs", "direct"]:
        u, _ = run_gpu(f, h, 5, path=path, robust=dict(eps=0.05))
        assert rel_err(u, ref) <= RTOL, path
        assert np.array_equal(u == 0.0, ref == 0.0), path
