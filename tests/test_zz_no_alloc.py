"""The allocation-free entry point rl_solve_static (workspace in the library's static
device array) against the existing path (rl_init on a caller workspace, rl_iterate,
rl_result) through the C ABI: bit-identical outputs and statistics, on two calls in a row,
the second with a smaller input (the array keeps the first call's contents), for plain,
thinned and persistent jobs."""
import numpy as np
import pytest

import synth
from gpu_util import RTOL, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd import _abi as A  # noqa: E402
from paper_1304_7211_amd.job import Job, make_params  # noqa: E402

THIN = dict(mode="rel", tau=1e-3, hysteresis=3, reset_period=10, compact_period=10)


def _static(f_dev, h, K, **kw):
    p, keep = make_params(f_dev, h, **kw)
    out = torch.empty_like(f_dev)
    st = A.rl_solve_static(p, K, out.data_ptr(), want_stats=True)
    del keep
    return out.cpu().numpy(), st


def _existing(f_dev, h, K, **kw):
    job = Job(f_dev, h, **kw)
    job.iterate(K)
    u, st = job.result(stats=True)
    job.close()
    return u.cpu().numpy(), st


CASES = [
    ("plain disc", dict(H=512, W=480, h=lambda: synth.disc(7), K=12, kw={}),
     dict(H=131, W=97, h=lambda: synth.oblique_line(21, 30.0), K=9, kw={})),
    ("thinned", dict(H=400, W=350, h=lambda: synth.disc(5), K=23, kw=dict(thin=THIN)),
     dict(H=150, W=131, h=lambda: synth.disc(4), K=14, kw=dict(thin=THIN))),
    ("persistent and resident", dict(H=300, W=280, h=lambda: synth.disc(6), K=6,
                                     kw=dict(path="runs", schedule="persistent")),
     dict(H=120, W=200, h=lambda: synth.box_h(15), K=20, kw={})),
]


@pytest.mark.parametrize("name,first,second", CASES, ids=[c[0] for c in CASES])
def test_static_solve_equals_existing_path(orc, name, first, second):
    for i, c in enumerate((first, second)):
        h = c["h"]()
        f = synth.observe(synth.latent_image(c["H"], c["W"], 60 + i), h, "poisson", 60 + i)
        fd = to_dev(f)
        print(f"{name} call {i + 1}: {c['H']}x{c['W']} K={c['K']} {c['kw']}", flush=True)
        us, ss = _static(fd, h, c["K"], **c["kw"])
        ue, se = _existing(fd, h, c["K"], **c["kw"])
        assert np.array_equal(us, ue), (name, i)
        assert ss.iters_done == se.iters_done == c["K"]
        assert ss.flux == se.flux
        assert ss.active_now == se.active_now
        assert ss.skipped_px_iters == se.skipped_px_iters
        if not c["kw"].get("thin"):
            assert rel_err(us, orc.rl(f, h, c["K"])) <= RTOL


def test_static_solve_reports_invalid_f():
    h = synth.disc(3)
    f = synth.observe(synth.latent_image(64, 70, 3), h, "poisson", 3)
    f[10, 10] = -1.0
    fd = to_dev(f)
    p, keep = make_params(fd, h)
    with pytest.raises(A.RLError) as e:
        A.rl_solve_static(p, 3, None)
    assert e.value.status == A.RL_E_INVAL
    # the next call on the same array is unaffected
    f[10, 10] = 0.5
    us, ss = _static(to_dev(f), h, 3)
    ue, se = _existing(to_dev(f), h, 3)
    assert np.array_equal(us, ue)
