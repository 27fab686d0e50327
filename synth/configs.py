"""Workload descriptions of the five benchmark configurations (seeded, synthetic).

A job is a dict with keys: name, f (float32 H x W), psf (float32 kh x kw), iters,
path ("auto"/"direct"/"box_axis"/"runs"), thin (None or dict), and for reference the
latent image g (float64) when it is cheap to keep.
"""
import math

import numpy as np

from . import psf as P
from .images import latent_image, observe

CONFIGS = {
    1: dict(name="plain-128-box15", H=128, W=128, K=50, noise="poisson", peak=255.0, seed=1),
    2: dict(name="specialised-1024", H=1024, W=1024, K=200, noise="gaussian", sigma=0.01),
    3: dict(name="thinned-2048-disc16", H=2048, W=2048, K=500, noise="poisson", peak=1000.0,
            seed=3, thin=dict(mode="rel", tau=1e-4, hysteresis=5, reset_period=10,
                              compact_period=10)),
    4: dict(name="batched-256", n_jobs=256, side_lo=256, side_hi=2048, K_lo=100, K_hi=300,
            noise="poisson", peak=255.0, seed=4),
    5: dict(name="serving", side_lo=128, side_hi=4096, K_lo=50, K_hi=500, noise="poisson",
            peak=255.0, seed=5),
}


def make_job(name, H, W, h, iters, seed, noise="poisson", peak=255.0, sigma=0.01,
             path="auto", thin=None, keep_latent=False):
    g = latent_image(H, W, seed)
    f = observe(g, h, noise, seed, peak=peak, sigma=sigma)
    job = dict(name=name, f=f, psf=np.ascontiguousarray(h, dtype=np.float32),
               iters=int(iters), path=path, thin=thin)
    if keep_latent:
        job["g"] = g
    return job


def random_psf(rng):
    """One PSF drawn from the mixed family of the batched and serving workloads."""
    cls = int(rng.integers(0, 4))
    if cls == 0:
        L = int(rng.integers(5, 64))
        return ("axis", P.box_h(L) if rng.uniform() < 0.5 else P.box_v(L))
    if cls == 1:
        L = int(rng.integers(9, 48))
        return ("oblique", P.oblique_line(L, float(rng.uniform(0.0, 180.0))))
    if cls == 2:
        return ("disc", P.disc(int(rng.integers(3, 25))))
    return ("dense", P.dense_random(15, int(rng.integers(0, 2**31))))


def log_uniform_side(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def job_for_config(cfg, variant=None, scale=1, workers=1, pool="thread"):
    """Jobs of configuration ``cfg``.  ``scale`` > 1 shrinks image sides (tests only);
    ``workers`` and ``pool`` parallelise the batched workload's images (see make_jobs)."""
    c = CONFIGS[cfg]
    if cfg == 1:
        return [make_job(c["name"], c["H"] // scale, c["W"] // scale, P.box_h(15), c["K"],
                         c["seed"], noise="poisson", peak=c["peak"], path="direct")]
    if cfg == 2:
        H, W = c["H"] // scale, c["W"] // scale
        specs = {"a": ("vertical-box-41", P.box_v(41), "box_axis", 21),
                 "b": ("oblique-31-at-30deg", P.oblique_line(31, 30.0), "runs", 22),
                 "c": ("disc-r10", P.disc(10), "runs", 23)}
        keys = [variant] if variant else ["a", "b", "c"]
        return [make_job(specs[k][0], H, W, specs[k][1], c["K"], specs[k][3],
                         noise="gaussian", sigma=c["sigma"], path=specs[k][2]) for k in keys]
    if cfg == 3:
        return [make_job(c["name"], c["H"] // scale, c["W"] // scale, P.disc(16), c["K"],
                         c["seed"], noise="poisson", peak=c["peak"], path="runs",
                         thin=dict(c["thin"]))]
    if cfg == 4:
        return make_jobs(batched_specs(scale), workers=workers, pool=pool)
    raise ValueError(cfg)


def batched_specs(scale=1):
    """Parameters of the batched workload's jobs, drawn in order from one seeded stream;
    each image then comes from its own seed, so the images can be made in any order."""
    c = CONFIGS[4]
    rng = np.random.default_rng(c["seed"])
    specs = []
    for i in range(c["n_jobs"]):
        H = max(16, log_uniform_side(rng, c["side_lo"], c["side_hi"]) // scale)
        W = max(16, log_uniform_side(rng, c["side_lo"], c["side_hi"]) // scale)
        cls, h = random_psf(rng)
        K = int(rng.integers(c["K_lo"], c["K_hi"] + 1))
        specs.append(dict(name=f"b{i}-{cls}", H=H, W=W, h=h, iters=K, seed=1000 + i,
                          noise="poisson", peak=c["peak"]))
    return specs


def serving_specs(n):
    """Parameters of n distinct serving requests (sides log-uniform in 128..4096, PSFs as
    in the batched workload, 50..500 iterations), drawn in order from one seeded stream;
    each image comes from its own seed."""
    c = CONFIGS[5]
    rng = np.random.default_rng(c["seed"])
    specs = []
    for i in range(int(n)):
        H = log_uniform_side(rng, c["side_lo"], c["side_hi"])
        W = log_uniform_side(rng, c["side_lo"], c["side_hi"])
        cls, h = random_psf(rng)
        K = int(rng.integers(c["K_lo"], c["K_hi"] + 1))
        specs.append(dict(name=f"s{i}-{cls}", H=H, W=W, h=h, iters=K, seed=500 + i,
                          noise=c["noise"], peak=c["peak"]))
    return specs


def _make_from_spec(s):
    return make_job(s["name"], s["H"], s["W"], s["h"], s["iters"], s["seed"],
                    noise=s["noise"], peak=s["peak"])


def make_jobs(specs, workers=1, pool="thread"):
    """Images of every spec, in spec order.  workers > 1 spreads them over a pool of
    threads, or of forked processes (pool="fork"; only before the process has touched a
    GPU).  The result does not depend on the pool."""
    if workers <= 1:
        return [_make_from_spec(s) for s in specs]
    if pool == "fork":
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as p:
            return p.map(_make_from_spec, specs, chunksize=1)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(_make_from_spec, specs))
