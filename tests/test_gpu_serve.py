"""Serving with continuous batching: requests that arrive while others run join the batch;
every result is bit-identical to the same request solved alone; admission respects the
HBM budget; oversized requests are rejected."""
import numpy as np
import pytest

import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1304_7211_amd.job import Job  # noqa: E402
from paper_1304_7211_amd.serve import (Request, Server, latency_report,  # noqa: E402
                                       request_footprint, run_stream, serve_plain)

THIN = dict(mode="rel", tau=1e-4, hysteresis=5, reset_period=10, compact_period=10)


def _requests(n=12, seed=7):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        H, W = int(rng.integers(40, 180)), int(rng.integers(40, 180))
        cls = i % 4
        if cls == 0:
            h = synth.box_h(int(rng.integers(5, 20))) if i % 8 == 0 else synth.box_v(int(rng.integers(5, 20)))
        elif cls == 1:
            h = synth.oblique_line(int(rng.integers(9, 20)), float(rng.uniform(0, 180)))
        elif cls == 2:
            h = synth.disc(int(rng.integers(3, 8)))
        else:
            h = synth.dense_random(15, i)
        f = synth.observe(synth.latent_image(H, W, 100 + i), h, "poisson", 100 + i)
        thin = THIN if i % 3 == 0 else None
        reqs.append(Request(i, f, h, int(rng.integers(5, 40)), thin=thin))
    return reqs


def _alone(r):
    job = Job(to_dev(r.f), r.psf, thin=r.thin)
    job.iterate(r.iters)
    u = job.result().cpu().numpy()
    job.close()
    return u


def test_continuous_batching_same_as_alone():
    reqs = _requests()
    alone = {r.rid: _alone(r) for r in reqs}
    # a budget that holds about three requests at a time
    fp = sorted(request_footprint(r, torch.device("cuda:0")) for r in reqs)
    srv = Server(budget_bytes=fp[-1] + fp[-2] + fp[-3], max_slots=16, chunk=7)
    # requests arrive in waves while earlier ones are still running
    for k in range(0, len(reqs), 3):
        for r in reqs[k:k + 3]:
            assert srv.submit(r)
        srv.tick()
    srv.drain()
    assert len(srv.done) == len(reqs) and not srv.rejected
    assert srv.ctl.peak_slots >= 2           # work overlapped on the device
    assert srv.ctl.peak_used <= srv.ctl.budget
    assert srv.ctl.used == 0 and srv.ctl.slots == 0
    for r in reqs:
        got = r.result.cpu().numpy()
        assert np.array_equal(got, alone[r.rid]), r.rid


def test_oversized_request_is_rejected():
    reqs = _requests(2)
    srv = Server(budget_bytes=1000, max_slots=4)
    assert not srv.submit(reqs[0])
    assert srv.rejected == [reqs[0]]
    srv.drain()


def test_stream_and_plain_reference():
    reqs = _requests(10, seed=11)
    rng = np.random.default_rng(3)
    t = np.cumsum(rng.exponential(0.002, size=len(reqs)))
    for r, a in zip(reqs, t):
        r.arrival = float(a)
    srv = Server(budget_bytes=4 << 30, max_slots=32, chunk=10)
    run_stream(reqs, srv)
    rep = latency_report(reqs)
    assert rep["n"] == len(reqs)
    base = _requests(10, seed=11)
    for r, a in zip(base, t):
        r.arrival = float(a)
    serve_plain(base)
    rep0 = latency_report(base)
    assert rep0["n"] == len(base)
    for a, b in zip(sorted(reqs, key=lambda r: r.rid), sorted(base, key=lambda r: r.rid)):
        assert np.array_equal(a.result.cpu().numpy(), b.result.cpu().numpy())
    print("continuous", rep, "plain", rep0)


def test_cancel_frees_the_slot_and_admits_the_next():
    """Cancelling a running request mid-stream: it leaves the batch, its slot and budget
    are released in the same call, the next waiting request is admitted at the next tick,
    and every other result is still bit-identical to the request solved alone."""
    reqs = _requests(n=6, seed=11)
    for r in reqs:
        r.iters = max(r.iters, 30)
    alone = {r.rid: _alone(r) for r in reqs}
    srv = Server(budget_bytes=1 << 40, max_slots=2, chunk=5)
    for r in reqs:
        assert srv.submit(r)
    srv.tick()
    running = [a[0].rid for a in srv.active]
    assert len(running) == 2 and srv.ctl.slots == 2 and len(srv.pending) == 4
    victim = running[0]
    assert srv.cancel(victim)
    assert srv.ctl.slots == 1 and srv.ctl.used == reqs[running[1]].footprint
    nxt = srv.pending[0].rid
    srv.tick()
    assert nxt in [a[0].rid for a in srv.active]
    assert not srv.cancel(victim)  # already gone
    srv.drain()
    torch.cuda.synchronize()
    assert reqs[victim].status == "cancelled" and reqs[victim].result is None
    for r in reqs:
        if r.rid != victim:
            assert r.status == "done"
            assert np.array_equal(r.result.cpu().numpy(), alone[r.rid]), r.rid
    assert srv.ctl.slots == 0 and srv.ctl.used == 0


def test_deadline_times_out_waiting_and_running_requests():
    """A request past its deadline is dropped whether it waits or runs; the others finish
    unchanged."""
    reqs = _requests(n=5, seed=12)
    for r in reqs:
        r.iters = max(r.iters, 30)
    alone = {r.rid: _alone(r) for r in reqs}
    srv = Server(budget_bytes=1 << 40, max_slots=1, chunk=5)
    t0 = 1000.0
    for r in reqs:
        r.arrival = t0
    reqs[0].deadline = 0.5   # runs first, times out while running
    reqs[3].deadline = 0.5   # still waiting when it expires
    for r in reqs:
        assert srv.submit(r)
    srv.tick(now=t0)
    assert [a[0].rid for a in srv.active] == [0]
    srv.tick(now=t0 + 1.0)  # both expire; request 1 takes the freed slot
    assert reqs[0].status == "timeout" and reqs[3].status == "timeout"
    assert [a[0].rid for a in srv.active] == [1]
    srv.drain()
    torch.cuda.synchronize()
    for r in reqs:
        if r.rid not in (0, 3):
            assert r.status == "done"
            assert np.array_equal(r.result.cpu().numpy(), alone[r.rid])
    rep = latency_report(reqs)
    assert rep["n"] == 3
