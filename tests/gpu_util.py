"""Shared helpers of the GPU tests: tolerance metric, device set-up, oracle comparisons."""
import numpy as np

# Floating-point tolerance of a float32 result against the FP64 oracle: max over pixels of
# |a - b| / max(|b|, FLOOR).  RL drives a few pixels towards 0, where a relative error is
# meaningless; FLOOR = 1e-4 on images scaled to [0, 1] (1/40 of a grey level of an 8-bit
# image) is where the relative metric takes over.
RTOL = 1e-5
FLOOR = 1e-4


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), FLOOR)))


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def run_gpu(f, h, K, **kw):
    """K iterations through the C ABI; returns (u as float64 numpy, job description)."""
    import torch
    from paper_1304_7211_amd.job import Job
    job = Job(to_dev(f), h, **kw)
    job.iterate(K)
    u = job.result()
    torch.cuda.synchronize()
    info = job.describe()
    job.close()
    return u.cpu().numpy().astype(np.float64), info
