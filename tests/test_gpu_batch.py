"""Batched iteration of uneven jobs (one launch per phase and kernel variant covering all
jobs still running): every job's result is bit-identical to the same job run alone, and
matches the oracle."""
import numpy as np
import pytest

import synth
from gpu_util import RTOL, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd import _abi as A  # noqa: E402
from paper_1304_7211_amd.job import BatchRunner, Job, iterate_batch  # noqa: E402

THIN = dict(mode="rel", tau=1e-3, hysteresis=3, reset_period=10, compact_period=10)


def _mixed_jobs():
    spec = [
        ("disc7", 150, 231, synth.disc(7), {}, 14),
        ("disc3", 97, 64, synth.disc(3), {}, 9),
        ("obl21", 200, 180, synth.oblique_line(21, 30.0), {}, 11),
        ("obl33", 77, 300, synth.oblique_line(33, 120.0), {}, 0),
        ("dense15", 129, 130, synth.dense_random(15, 5), {}, 7),
        ("vbox9_tp", 160, 96, synth.box_v(9), dict(schedule="two_pass"), 12),
        ("hbox31_res", 64, 250, synth.box_h(31), {}, 13),
        # more resident line solvers: jobs of one line orientation share a launch, each
        # workgroup running its own job's iteration count
        ("hbox15_res", 90, 200, synth.box_h(15), {}, 9),
        ("vbox21_res", 220, 70, synth.box_v(21), {}, 17),
        ("vbox7_res", 130, 128, synth.box_v(7), {}, 6),
        ("disc5_thin", 140, 150, synth.disc(5), dict(thin=THIN), 25),
        ("obl15_thin", 120, 90, synth.oblique_line(15, 60.0), dict(thin=THIN), 16),
        ("rect9x5", 170, 140, synth.box_rect(9, 5), {}, 10),
        ("rect4x4_thin", 133, 97, synth.box_rect(4, 4), dict(thin=THIN), 15),
        ("sat7x3", 150, 120, synth.box_rect(7, 3), dict(path="box_sat"), 9),
    ]
    out = []
    for i, (name, H, W, h, kw, K) in enumerate(spec):
        f = synth.observe(synth.latent_image(H, W, 40 + i), h, "poisson", 40 + i)
        out.append((name, f, h, kw, K))
    return out


def _alone(f, h, kw, K):
    job = Job(to_dev(f), h, **kw)
    job.iterate(K)
    st = job.get_state()
    u = st["u"].cpu().numpy()
    cnt = st["cnt"].cpu().numpy() if st["cnt"] is not None else None
    job.close()
    return u, cnt


def test_batch_bit_identical_to_alone(orc):
    specs = _mixed_jobs()
    alone = [_alone(f, h, kw, K) for (_, f, h, kw, K) in specs]
    jobs = [Job(to_dev(f), h, **kw) for (_, f, h, kw, K) in specs]
    Ks = [K for (*_, K) in specs]
    # two consecutive batches: the split must not matter
    first = [k // 2 for k in Ks]
    runner = BatchRunner(len(jobs))
    runner.iterate(jobs, first)
    runner.iterate(jobs, [k - a for k, a in zip(Ks, first)])
    torch.cuda.synchronize()
    for (name, f, h, kw, K), job, (u_a, c_a) in zip(specs, jobs, alone):
        st = job.get_state()
        assert st["k"] == K
        u = st["u"].cpu().numpy()
        assert np.array_equal(u, u_a), name
        if c_a is not None:
            assert np.array_equal(st["cnt"].cpu().numpy(), c_a), name
        if not kw.get("thin"):
            assert rel_err(u, orc.rl(f, h, K)) <= RTOL, name
        job.close()


def test_batch_is_order_independent():
    specs = _mixed_jobs()[:5]
    res = []
    for order in (list(range(len(specs))), list(reversed(range(len(specs))))):
        jobs = [Job(to_dev(specs[i][1]), specs[i][2], **specs[i][3]) for i in order]
        iterate_batch(jobs, [specs[i][4] for i in order])
        torch.cuda.synchronize()
        got = {specs[i][0]: jobs[q].result().cpu().numpy() for q, i in enumerate(order)}
        for j in jobs:
            j.close()
        res.append(got)
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k


def test_batch_errors():
    h = synth.disc(3)
    f = synth.observe(synth.latent_image(40, 40, 1), h, "poisson", 1)
    job = Job(to_dev(f), h)
    runner = BatchRunner(2)
    with pytest.raises(A.RLError) as e:
        runner.iterate([job, job], [1, 1])
    assert e.value.status == A.RL_E_INVAL
    with pytest.raises(A.RLError) as e:
        A.rl_iterate_batch([job.handle], [1], runner.ws.data_ptr(), 16, 0)
    assert e.value.status == A.RL_E_NOMEM
    with pytest.raises(A.RLError) as e:
        runner.iterate([job], [-1])
    assert e.value.status == A.RL_E_INVAL
    job.close()


def test_jobs_set_up_while_a_batch_runs():
    """Jobs created while earlier batches still run (their table uploads go through pinned
    buffers that the library reuses once their copies have completed) end bit-identical to
    the same jobs run alone on an idle device, round after round."""
    specs = _mixed_jobs()
    alone = [_alone(f, h, kw, K)[0] for (_, f, h, kw, K) in specs]
    fs = [to_dev(f) for (_, f, *_r) in specs]
    runner = BatchRunner(len(specs))
    rounds = []
    for _ in range(3):
        # no synchronisation: each round's jobs are set up behind the previous round's batch
        jobs = [Job(fd, h, **kw) for fd, (_, f, h, kw, K) in zip(fs, specs)]
        runner.iterate(jobs, [K for (*_, K) in specs])
        rounds.append([j.result() for j in jobs])
        for j in jobs:
            j.close()
    torch.cuda.synchronize()
    for outs in rounds:
        for (name, *_r), o, u_a in zip(specs, outs, alone):
            assert np.array_equal(o.cpu().numpy(), u_a), name
