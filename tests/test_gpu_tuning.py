"""GPU checks of the iteration drivers that do not change the arithmetic: captured HIP
graph replay of plain tiled jobs, and the autotuner with its tuning cache.

Graph replay must be bit-identical to direct launches (same kernels, same arguments),
over several replays interleaved with other device work; a tuned job must still match
the FP64 oracle within RTOL.
"""
import numpy as np
import pytest

import synth
from gpu_util import RTOL, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd import _abi as A  # noqa: E402
from paper_1304_7211_amd.job import Job, autotune, tune_lookup  # noqa: E402


def _obs(H, W, h, seed):
    return synth.observe(synth.latent_image(H, W, seed), h, "poisson", seed)


GRAPH_PSFS = [synth.disc(6), synth.oblique_line(31, 30.0), synth.box_h(15),
              synth.dense_random(9, 5)]


@pytest.mark.parametrize("sched", ["two_pass", "fused"])
def test_graph_replay_bit_identical(orc, sched):
    for h in GRAPH_PSFS:
        f = _obs(300, 257, h, 31)
        fd = to_dev(f)
        eager = Job(fd, h, schedule=sched)
        graph = Job(fd, h, schedule=sched, tuning=dict(graph_iters=6))
        noise = torch.zeros(1 << 20, device=fd.device)
        # uneven chunks: replays of the 6-iteration graph plus direct remainders, with
        # unrelated device work and host synchronisation between the calls
        total = 0
        for n in (13, 6, 1, 20):
            eager.iterate(n)
            graph.iterate(n)
            total += n
            noise.add_(1.0)
            torch.cuda.synchronize()
            ue = eager.result().cpu().numpy()
            ug = graph.result().cpu().numpy()
            assert np.array_equal(ue, ug), (h.shape, sched, total)
        assert graph.stats().iters_done == total
        assert rel_err(ug, orc.rl(f, h, total)) <= RTOL
        eager.close()
        graph.close()


def test_graph_ignored_for_thinned_and_resident():
    h = synth.box_h(15)
    f = _obs(200, 300, h, 5)
    fd = to_dev(f)
    for kw in (dict(thin=dict(mode="rel", tau=1e-3, hysteresis=3)), dict(schedule="resident")):
        a = Job(fd, h, **kw)
        b = Job(fd, h, tuning=dict(graph_iters=4), **kw)
        a.iterate(11)
        b.iterate(11)
        assert np.array_equal(a.result().cpu().numpy(), b.result().cpu().numpy()), kw
        a.close()
        b.close()


def test_autotune_caches_and_stays_correct(orc):
    A.rl_tune_cache_clear()
    cases = [(synth.disc(8), 512, 640), (synth.box_v(21), 384, 512),
             (synth.oblique_line(25, 60.0), 256, 256)]
    for h, H, W in cases:
        f = _obs(H, W, h, 11)
        fd = to_dev(f)
        res = autotune(fd, h, n_iter=4)
        print(h.shape, H, W, res)
        assert res["ms_per_iter"] > 0
        hit = tune_lookup(fd, h)
        assert hit == dict(schedule=res["schedule"], tuning=res["tuning"])
        # a job with default tuning now takes the cached choice
        job = Job(fd, h)
        info = job.describe()
        assert info["schedule"] == A.SCHEDS[res["schedule"]] or res["schedule"] == "auto"
        if res["tuning"]["strip"]:
            assert info["strip"] == res["tuning"]["strip"] or info["schedule"] == 3
        job.iterate(9)
        u = job.result().cpu().numpy()
        job.close()
        assert rel_err(u, orc.rl(f, h, 9)) <= RTOL, (h.shape, res)
    A.rl_tune_cache_clear()
