"""Parity at the benchmark's full sizes, in the launch configuration bench.py times
(configuration 2: three 1024 x 1024 jobs advanced by one rl_iterate_batch call).

* K = 5: every output against the FP64 oracle run on the whole image (RTOL).
* K = 200 (the benchmark's iteration count): properties that hold at any size -- the
  batched result is bit-identical to each job run alone, u stays finite and non-negative,
  and the FP64 flux equals the flux of f where the PSF is mirror-symmetric in both axes
  (reflecting boundary: the folded correlation is then the exact adjoint of the folded
  convolution; the oblique line is only point-symmetric, so it is exempt).
"""
import numpy as np
import pytest

import synth
from gpu_util import RTOL, rel_err, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd.job import BatchRunner, Job  # noqa: E402


def _batch(jobs_spec, K):
    jobs = [Job(to_dev(j["f"]), j["psf"], path=j["path"]) for j in jobs_spec]
    BatchRunner(len(jobs)).iterate(jobs, [K] * len(jobs))
    outs = []
    for j in jobs:
        u, st = j.result(stats=True)
        outs.append((u.cpu().numpy(), st))
        j.close()
    return outs


def test_config2_full_size_against_oracle(orc):
    spec = synth.job_for_config(2)
    outs = _batch(spec, 5)
    for j, (u, st) in zip(spec, outs):
        ref = orc.rl(j["f"], j["psf"], 5)
        err = rel_err(u, ref)
        print(f"{j['name']}: K=5 full-image err {err:.3g}")
        assert err <= RTOL, j["name"]


def test_config2_full_length_properties():
    spec = synth.job_for_config(2)
    K = spec[0]["iters"]
    outs = _batch(spec, K)
    for j, (u, st) in zip(spec, outs):
        alone = Job(to_dev(j["f"]), j["psf"], path=j["path"])
        alone.iterate(K)
        ua = alone.result().cpu().numpy()
        alone.close()
        assert np.array_equal(u, ua), j["name"]
        assert st.iters_done == K
        assert np.isfinite(u).all() and (u >= 0).all()
        h = j["psf"]
        if np.array_equal(h, h[::-1, :]) and np.array_equal(h, h[:, ::-1]):
            fsum = float(j["f"].astype(np.float64).sum())
            assert abs(st.flux - fsum) <= 1e-5 * fsum, (j["name"], st.flux, fsum)
