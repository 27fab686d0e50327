"""Torch-facing helpers over the C ABI: torch provides device memory and the stream.

``Job`` owns a torch uint8 workspace of exactly ``rl_workspace_bytes`` and a job handle;
every method is one C call (argument marshalling only).
"""
import numpy as np
import torch

from . import _abi as A


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_params(f, psf, boundary="reflect", path="auto", schedule="auto", kahan=True,
                thin=None, u0=None, stream=None, tuning=None, tv=None, robust=None):
    """Build an rl_params for a float32 CUDA image f (H, W) and a float32 numpy PSF."""
    if not (isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float32
            and f.dim() == 2 and f.is_contiguous()):
        raise ValueError("f must be a contiguous float32 CUDA tensor of shape (H, W)")
    psf = np.ascontiguousarray(psf, dtype=np.float32)
    p = A.rl_params()
    p.height, p.width = int(f.shape[0]), int(f.shape[1])
    p.f = f.data_ptr()
    p.psf_h, p.psf_w = int(psf.shape[0]), int(psf.shape[1])
    p.psf = psf.ctypes.data
    p.u0 = u0.data_ptr() if u0 is not None else None
    p.boundary = A.BCS[boundary]
    p.path = A.PATHS[path]
    p.schedule = A.SCHEDS[schedule]
    p.kahan = 1 if kahan else 0
    if thin:
        p.thin.mode = A.THINS[thin.get("mode", "rel")]
        p.thin.tau = float(thin["tau"])
        p.thin.hysteresis = int(thin.get("hysteresis", 1))
        p.thin.reset_period = int(thin.get("reset_period", 10))
        p.thin.compact_period = int(thin.get("compact_period", 10))
        p.thin.keep_list = 1 if thin.get("keep_list", False) else 0
        p.thin.block = int(thin.get("block", 0))
    p.stream = _stream_ptr(stream)
    if tuning:
        p.tuning.strip = int(tuning.get("strip", 0))
        p.tuning.seg = int(tuning.get("seg", 0))
        p.tuning.lines_per_wg = int(tuning.get("lines_per_wg", 0))
        p.tuning.graph_iters = int(tuning.get("graph_iters", 0))
    if tv:
        p.tv_lambda = float(tv["lam"])
        p.tv_eps = float(tv.get("eps", 1e-3))
    if robust:
        p.rob_eps = float(robust["eps"])
    return p, psf  # keep psf alive until rl_init has copied it


def workspace_bytes(f, psf, **kw):
    p, _keep = make_params(f, psf, **kw)
    return A.rl_workspace_bytes(p)


def tuning_dict(t):
    return dict(strip=t.strip, seg=t.seg, lines_per_wg=t.lines_per_wg, graph_iters=t.graph_iters)


def autotune(f, psf, n_iter=10, **kw):
    """Time the candidate kernel shapes on (f, psf) and cache the fastest for jobs of the
    same kind.  Returns dict(schedule=..., tuning=..., ms_per_iter=...)."""
    p, keep = make_params(f, psf, **kw)
    ws = torch.empty(A.rl_autotune_workspace_bytes(p), dtype=torch.uint8, device=f.device)
    sched, t, ms = A.rl_autotune(p, ws.data_ptr(), ws.numel(), n_iter)
    del keep
    return dict(schedule=A.SCHED_NAMES[sched], tuning=tuning_dict(t), ms_per_iter=ms)


def tune_lookup(f, psf, **kw):
    p, keep = make_params(f, psf, **kw)
    r = A.rl_tune_lookup(p)
    del keep
    return None if r is None else dict(schedule=A.SCHED_NAMES[r[0]], tuning=tuning_dict(r[1]))


class Job:
    def __init__(self, f, psf, boundary="reflect", path="auto", schedule="auto", kahan=True,
                 thin=None, u0=None, stream=None, workspace=None, tuning=None, tv=None,
                 robust=None):
        p, keep = make_params(f, psf, boundary, path, schedule, kahan, thin, u0, stream, tuning,
                              tv, robust)
        self.nbytes = A.rl_workspace_bytes(p)
        if workspace is None:
            workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=f.device)
        self.ws = workspace
        self.shape = (int(f.shape[0]), int(f.shape[1]))
        self.device = f.device
        self.thin = bool(thin)
        self.handle = A.rl_init(p, self.ws.data_ptr(), self.ws.numel())
        del keep

    def iterate(self, n):
        A.rl_iterate(self.handle, n)
        return self

    def result(self, out=None, stats=False):
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        st = A.rl_result(self.handle, out.data_ptr(), want_stats=stats)
        return (out, st) if stats else out

    def stats(self):
        return A.rl_result(self.handle, None, want_stats=True)

    def get_state(self):
        u = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        r = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        cnt = torch.empty(self.shape, dtype=torch.uint8, device=self.device) if self.thin else None
        k = A.rl_get_state(self.handle, u.data_ptr(), r.data_ptr(),
                           cnt.data_ptr() if cnt is not None else None)
        return dict(u=u, r=r, cnt=cnt, k=k)

    def set_state(self, u=None, r=None, cnt=None, k=0):
        A.rl_set_state(self.handle, u.data_ptr() if u is not None else None,
                       r.data_ptr() if r is not None else None,
                       cnt.data_ptr() if cnt is not None else None, k)

    def active_list(self):
        n = A.rl_active_list(self.handle)
        if n < 0:
            return None
        out = torch.empty(max(1, n), dtype=torch.int32, device=self.device)
        A.rl_active_list(self.handle, out.data_ptr(), out.numel())
        return out[:n]

    def thin_schedule(self, cap=4096):
        return A.rl_thin_schedule(self.handle, cap)

    def describe(self):
        i = A.rl_job_describe(self.handle)
        return {n: getattr(i, n) for n, _ in i._fields_}

    def close(self):
        if self.handle:
            A.rl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def deconvolve(f, psf, iters, **kw):
    """Run ``iters`` RL iterations on f (CUDA float32) and return u^K (CUDA float32)."""
    job = Job(f, psf, **kw)
    try:
        job.iterate(iters)
        return job.result()
    finally:
        job.close()


class BatchRunner:
    """Owns one batch workspace (torch uint8) sized for up to ``max_jobs`` jobs and runs
    ``rl_iterate_batch`` on it."""

    def __init__(self, max_jobs, device=None):
        self.max_jobs = int(max_jobs)
        self.nbytes = A.rl_batch_workspace_bytes(self.max_jobs)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8,
                              device=device or torch.device("cuda:0"))

    def iterate(self, jobs, n_iters, stream=None):
        if len(jobs) > self.max_jobs:
            raise ValueError("more jobs than the batch workspace was sized for")
        handles = [j.handle for j in jobs]
        A.rl_iterate_batch(handles, n_iters, self.ws.data_ptr(), self.ws.numel(),
                           _stream_ptr(stream))


def iterate_batch(jobs, n_iters, stream=None):
    """One-shot batch: every job j advances by n_iters[j] iterations."""
    BatchRunner(len(jobs), jobs[0].device).iterate(jobs, n_iters, stream)
