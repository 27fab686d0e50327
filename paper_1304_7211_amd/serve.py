"""Serving: continuous batching of deconvolution requests on one GPU.

Requests (an observed image, a PSF, an iteration budget, optional thinning) arrive over
time.  The server keeps every admitted job's state (u^k, r, counters, active lists) in
its own device workspace and advances all resident jobs together, ``chunk`` iterations
per tick, through ``rl_iterate_batch`` (one launch per phase and kernel variant covering
every job still running).  Between ticks it retires finished jobs (their result copy was
enqueued right after their last chunk) and admits waiting requests as soon as slots and
HBM budget allow -- requests that arrive while others run join the running batch.

Admission is by footprint: a request needs its workspace (rl_workspace_bytes) plus its
input and output images on the device.  A request larger than the whole budget is
rejected; otherwise it waits in arrival order (no overtaking, so a large request is not
starved by small ones).

A request can be cancelled (``Server.cancel``) or given a deadline (``Request.deadline``,
seconds after its arrival): a waiting request is dropped, a running one leaves the batch
at the next tick; either way its slot and budget are released at once, so the next
waiting request is admitted in the same tick.  A request whose result copy has already
been enqueued completes normally.

``serve_plain`` is the reference form: one request at a time, in arrival order, each
solved alone with rl_iterate.

Every job's result is bit-identical whether it runs alone or in any mix (the kernels of a
job do not depend on its neighbours in a launch).
"""
import collections
import time

import numpy as np
import torch

from . import _abi as A
from .job import BatchRunner, Job


class Request:
    def __init__(self, rid, f, psf, iters, thin=None, arrival=0.0, path="auto",
                 deadline=None):
        self.rid = rid
        self.f = f                # numpy float32 (H, W) on the host, or a CUDA tensor
        self.psf = np.ascontiguousarray(psf, dtype=np.float32)
        self.iters = int(iters)
        self.thin = thin
        self.arrival = float(arrival)
        self.path = path
        self.deadline = None if deadline is None else float(deadline)  # s after arrival
        # filled by the server
        self.admitted = None
        self.completed = None
        self.result = None
        self.footprint = None
        self.status = "new"       # pending, running, done, cancelled, timeout, rejected

    @property
    def shape(self):
        return tuple(self.f.shape)


class AdmissionController:
    """Pure bookkeeping of the HBM budget and the slot count (no device work).

    ``try_admit(nbytes)`` succeeds when the request fits next to the resident jobs;
    ``fits_ever(nbytes)`` says whether it could fit at all."""

    def __init__(self, budget_bytes, max_slots):
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.used = 0
        self.slots = 0
        self.peak_used = 0
        self.peak_slots = 0

    def fits_ever(self, nbytes):
        return nbytes <= self.budget

    def try_admit(self, nbytes):
        if self.slots >= self.max_slots or self.used + nbytes > self.budget:
            return False
        self.used += nbytes
        self.slots += 1
        self.peak_used = max(self.peak_used, self.used)
        self.peak_slots = max(self.peak_slots, self.slots)
        return True

    def release(self, nbytes):
        self.used -= nbytes
        self.slots -= 1
        assert self.used >= 0 and self.slots >= 0


def request_footprint(req, device):
    """Device bytes a request occupies while resident: workspace + f + u_out."""
    H, W = req.shape
    # rl_workspace_bytes only reads sizes and the PSF, so no image pointer is needed
    p = A.rl_params()
    p.height, p.width = H, W
    p.psf_h, p.psf_w = req.psf.shape
    p.psf = req.psf.ctypes.data
    p.path = A.PATHS[req.path]
    p.kahan = 1
    if req.thin:
        p.thin.mode = A.THINS[req.thin.get("mode", "rel")]
        p.thin.tau = float(req.thin["tau"])
        p.thin.hysteresis = int(req.thin.get("hysteresis", 1))
        p.thin.reset_period = int(req.thin.get("reset_period", 10))
        p.thin.compact_period = int(req.thin.get("compact_period", 10))
        p.thin.keep_list = 1 if req.thin.get("keep_list", False) else 0
        p.thin.block = int(req.thin.get("block", 0))
    ws = A.rl_workspace_bytes(p)
    return ws + 2 * H * W * 4


class Server:
    """Continuous-batching request loop over the C ABI."""

    def __init__(self, budget_bytes, max_slots=64, chunk=10, device=None, stream=None):
        self.device = device or torch.device("cuda:0")
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.ctl = AdmissionController(budget_bytes, max_slots)
        self.chunk = int(chunk)
        self.pending = collections.deque()
        self.active = []          # list of [req, job, f_dev, remaining]
        self.in_flight = []       # list of (event, [(req, job, f_dev, out)])
        self.done = []
        self.rejected = []
        self.cancelled = []       # cancelled and timed-out requests
        self.runner = BatchRunner(max_slots, self.device)
        self.ticks = 0

    # -- request intake ------------------------------------------------------------------
    def submit(self, req):
        req.footprint = request_footprint(req, self.device)
        if not self.ctl.fits_ever(req.footprint):
            req.completed = float("nan")
            req.status = "rejected"
            self.rejected.append(req)
            return False
        req.status = "pending"
        self.pending.append(req)
        return True

    def cancel(self, rid, status="cancelled", now=None):
        """Drop request ``rid`` if it is still waiting or running: a running job leaves the
        batch (its device state is freed on the server stream, after the work already
        enqueued for it) and its slot and budget are released.  Returns False if the
        request is unknown here or its result is already on its way."""
        now = time.perf_counter() if now is None else now
        for req in self.pending:
            if req.rid == rid:
                self.pending.remove(req)
                self._end(req, status, now)
                return True
        for a in self.active:
            if a[0].rid == rid:
                self.active.remove(a)
                req, job = a[0], a[1]
                job.close()
                self.ctl.release(req.footprint)
                self._end(req, status, now)
                return True
        return False

    def _end(self, req, status, now):
        req.status = status
        req.completed = now
        req.result = None
        self.cancelled.append(req)

    def _expire(self, now):
        late = [r.rid for r in self.pending if r.deadline is not None
                and now > r.arrival + r.deadline]
        late += [a[0].rid for a in self.active if a[0].deadline is not None
                 and now > a[0].arrival + a[0].deadline]
        for rid in late:
            self.cancel(rid, status="timeout", now=now)

    def _admit(self, now):
        while self.pending:
            req = self.pending[0]
            if not self.ctl.try_admit(req.footprint):
                break
            self.pending.popleft()
            with torch.cuda.stream(self.stream):
                f_dev = req.f if isinstance(req.f, torch.Tensor) else \
                    torch.from_numpy(np.ascontiguousarray(req.f)).to(self.device, non_blocking=False)
                job = Job(f_dev, req.psf, thin=req.thin, path=req.path, stream=self.stream)
            req.admitted = now
            req.status = "running"
            self.active.append([req, job, f_dev, req.iters])

    # -- one tick ------------------------------------------------------------------------
    def _retire_finished(self, block=False):
        keep = []
        for ev, items in self.in_flight:
            if block:
                ev.synchronize()
            if ev.query():
                t = time.perf_counter()
                for req, job, f_dev, out in items:
                    req.completed = t
                    req.result = out
                    req.status = "done"
                    job.close()
                    self.ctl.release(req.footprint)
                    self.done.append(req)
            else:
                keep.append((ev, items))
        self.in_flight = keep

    def tick(self, now=None):
        """Admit, advance every resident job by up to ``chunk`` iterations, enqueue the
        results of jobs that finished, and retire jobs whose results are complete."""
        now = time.perf_counter() if now is None else now
        self._retire_finished()
        self._expire(now)
        self._admit(now)
        if not self.active:
            return False
        jobs = [a[1] for a in self.active]
        steps = [min(self.chunk, a[3]) for a in self.active]
        self.runner.iterate(jobs, steps, stream=self.stream)
        finished, still = [], []
        for a, n in zip(self.active, steps):
            a[3] -= n
            if a[3] == 0:
                req, job, f_dev = a[0], a[1], a[2]
                out = torch.empty(req.shape, dtype=torch.float32, device=self.device)
                with torch.cuda.stream(self.stream):
                    job.result(out=out)
                finished.append((req, job, f_dev, out))
            else:
                still.append(a)
        self.active = still
        if finished:
            ev = torch.cuda.Event()
            ev.record(self.stream)
            self.in_flight.append((ev, finished))
        self.ticks += 1
        return True

    def idle(self):
        return not (self.pending or self.active or self.in_flight)

    def drain(self):
        while self.active or self.pending:
            if not self.tick():
                self._retire_finished(block=True)
        self._retire_finished(block=True)


def run_stream(requests, server, t0=None, time_scale=1.0):
    """Feed requests at their arrival times (seconds from t0, scaled) and serve until all
    are done.  Returns the wall-clock duration."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter() if t0 is None else t0
    for r in reqs:
        r.arrival = t0 + r.arrival * time_scale
    i = 0
    while i < len(reqs) or not server.idle():
        now = time.perf_counter()
        while i < len(reqs) and reqs[i].arrival <= now:
            server.submit(reqs[i])
            i += 1
        if not server.tick(now):
            if server.in_flight:
                server._retire_finished(block=False)
            elif i < len(reqs):
                time.sleep(min(1e-4, max(0.0, reqs[i].arrival - time.perf_counter())))
    server._retire_finished(block=True)
    return time.perf_counter() - t0


def serve_plain(requests, device=None, stream=None):
    """Reference form: one request at a time in arrival order, each solved alone."""
    device = device or torch.device("cuda:0")
    stream = stream or torch.cuda.current_stream(device)
    reqs = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    base = t0
    for r in reqs:
        r.arrival = base + r.arrival
    for r in reqs:
        now = time.perf_counter()
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.admitted = time.perf_counter()
        with torch.cuda.stream(stream):
            f_dev = r.f if isinstance(r.f, torch.Tensor) else torch.from_numpy(
                np.ascontiguousarray(r.f)).to(device)
            job = Job(f_dev, r.psf, thin=r.thin, path=r.path, stream=stream)
            job.iterate(r.iters)
            out = job.result()
        stream.synchronize()
        r.completed = time.perf_counter()
        r.result = out
        r.status = "done"
        job.close()
    return time.perf_counter() - t0


def latency_report(requests):
    lat = np.array([r.completed - r.arrival for r in requests
                    if r.completed == r.completed and r.status == "done"])
    if lat.size == 0:
        return dict(n=0)
    return dict(n=int(lat.size), p50_ms=float(1e3 * np.percentile(lat, 50)),
                p99_ms=float(1e3 * np.percentile(lat, 99)), mean_ms=float(1e3 * lat.mean()),
                max_ms=float(1e3 * lat.max()))
