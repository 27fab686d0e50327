"""Host-only checks of the C ABI (no GPU needed): the library loads and exports every
symbol include/rl.h declares; the PSF compiler's run list equals the oracle-side
definition bit for bit (P13); parameter validation returns the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    from paper_1304_7211_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1304_7211_amd import build
        build.build()
    _abi.lib()
    return _abi


def test_exports_every_declared_symbol(A):
    hdr = open(os.path.join(ROOT, "include", "rl.h")).read()
    declared = set(re.findall(r"\b(rl_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    L = ctypes.CDLL(A.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} declared in rl.h but not exported"
    assert declared == set(A.EXPORTS)


def test_status_strings(A):
    assert A.status_str(0) == "RL_OK"
    assert A.status_str(-1) == "RL_E_INVAL"
    assert A.status_str(-5) == "RL_E_UNSUPPORTED"
    assert A.status_str(42) == "RL_E_UNKNOWN"


def _psfs():
    yield synth.delta()
    for L in (2, 5, 15, 41, 63):
        yield synth.box_h(L)
        yield synth.box_v(L)
    for r in (1, 3, 4, 8, 10, 16, 24):
        yield synth.disc(r)
    for L, a in ((9, 0.0), (31, 30.0), (47, 75.0), (17, 45.0), (13, 90.0), (25, 137.0)):
        yield synth.oblique_line(L, a)
    yield synth.dense_random(15, 3)
    yield synth.box_rect(5, 7)
    yield np.array([[0, 1, 1, 2, 0, 3], [0, 0, 0, 0, 0, 0], [5, 5, 5, 5, 5, 5]], np.float32)


def test_p13_run_list_matches_oracle_definition(A):
    for h in _psfs():
        ints, ws = oracle.psf_runs(h)
        runs, w, cls = A.rl_psf_runs(np.ascontiguousarray(h))
        assert np.array_equal(runs, ints), h.shape
        assert np.array_equal(w.view(np.uint32), ws.view(np.uint32))


def test_auto_classification(A):
    assert A.rl_psf_runs(synth.delta())[2] == A.RL_PATH_DIRECT
    assert A.rl_psf_runs(synth.box_h(15))[2] == A.RL_PATH_BOX_AXIS
    assert A.rl_psf_runs(synth.box_v(41))[2] == A.RL_PATH_BOX_AXIS
    assert A.rl_psf_runs(synth.disc(10))[2] == A.RL_PATH_RUNS
    assert A.rl_psf_runs(synth.oblique_line(31, 30.0))[2] == A.RL_PATH_RUNS
    assert A.rl_psf_runs(synth.dense_random(15, 1))[2] == A.RL_PATH_RUNS
    assert A.rl_psf_runs(synth.box_rect(5, 7))[2] == A.RL_PATH_BOX_RECT
    assert A.rl_psf_runs(synth.box_rect(2, 2))[2] == A.RL_PATH_BOX_RECT
    # a rectangle with one different tap, or with a hole, is not a box
    h = np.ones((4, 6), np.float32)
    h[2, 3] = 2.0
    assert A.rl_psf_runs(h)[2] == A.RL_PATH_RUNS
    h = np.ones((4, 6), np.float32)
    h[1, 0] = 0.0
    assert A.rl_psf_runs(h)[2] == A.RL_PATH_RUNS
    # a rectangle inside zero margins is still a rectangle
    h = np.zeros((7, 9), np.float32)
    h[1:4, 2:8] = 1.0
    assert A.rl_psf_runs(h)[2] == A.RL_PATH_BOX_RECT
    # a vertical line with gaps is not a box
    h = np.zeros((5, 1), np.float32)
    h[[0, 1, 3, 4]] = 0.25
    assert A.rl_psf_runs(h)[2] == A.RL_PATH_RUNS


def _params(A, H=64, W=48, psf=None, **kw):
    psf = synth.disc(3) if psf is None else np.ascontiguousarray(psf, np.float32)
    p = A.rl_params()
    p.height, p.width = H, W
    p.f = 0
    p.psf_h, p.psf_w = psf.shape
    p.psf = psf.ctypes.data
    p.boundary = kw.get("boundary", 0)
    p.path = kw.get("path", 0)
    p.schedule = kw.get("schedule", 0)
    p.kahan = 1
    if "thin" in kw:
        p.thin.mode, p.thin.tau, p.thin.hysteresis, p.thin.reset_period, \
            p.thin.compact_period = kw["thin"]
    return p, psf


def _ws_status(A, p):
    n = ctypes.c_size_t(0)
    return A.lib().rl_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), n.value


def test_workspace_bytes_and_validation(A):
    p, keep = _params(A)
    st, n = _ws_status(A, p)
    assert st == A.RL_OK and n >= 3 * 64 * 48 * 4
    # thinning adds counters, lists and the schedule ring
    p2, keep2 = _params(A, thin=(A.RL_THIN_REL, 1e-4, 5, 10, 10))
    st2, n2 = _ws_status(A, p2)
    assert st2 == A.RL_OK and n2 > n
    bad = []
    p, k1 = _params(A, H=0)
    bad.append(p)
    p, k2 = _params(A, psf=np.array([[0.5, -0.1, 0.6]], np.float32))
    bad.append(p)
    p, k3 = _params(A, psf=np.array([[0.5, np.nan]], np.float32))
    bad.append(p)
    p, k4 = _params(A, psf=np.zeros((3, 3), np.float32))
    bad.append(p)
    p, k5 = _params(A, psf=synth.disc(3), path=A.RL_PATH_BOX_AXIS)
    bad.append(p)
    p, k6 = _params(A, boundary=7)
    bad.append(p)
    p, k7 = _params(A, thin=(A.RL_THIN_REL, 1e-4, 0, 10, 10))
    bad.append(p)
    for q in bad:
        assert _ws_status(A, q)[0] == A.RL_E_INVAL
    p, k8 = _params(A, psf=synth.box_h(9), schedule=A.RL_SCHED_RESIDENT,
                    thin=(A.RL_THIN_ABS, 0.1, 1, 10, 1))
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k9 = _params(A, psf=synth.box_h(9), schedule=A.RL_SCHED_RESIDENT)
    assert _ws_status(A, p)[0] == A.RL_OK
    # TV regularisation: lambda in [0, 0.25), eps > 0, not with thinning
    p, k12 = _params(A)
    p.tv_lambda, p.tv_eps = 0.1, 1e-3
    assert _ws_status(A, p)[0] == A.RL_OK
    p.tv_lambda = 0.25
    assert _ws_status(A, p)[0] == A.RL_E_INVAL
    p.tv_lambda, p.tv_eps = 0.1, 0.0
    assert _ws_status(A, p)[0] == A.RL_E_INVAL
    p, k13 = _params(A, thin=(A.RL_THIN_REL, 1e-4, 5, 10, 10))
    p.tv_lambda, p.tv_eps = 0.1, 1e-3
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    # robust data term: eps >= 0; not with TV, thinning, the resident or fused schedule
    p, k17 = _params(A)
    p.rob_eps = 0.05
    assert _ws_status(A, p)[0] == A.RL_OK
    p.rob_eps = -1.0
    assert _ws_status(A, p)[0] == A.RL_E_INVAL
    p, k18 = _params(A, thin=(A.RL_THIN_REL, 1e-4, 5, 10, 10))
    p.rob_eps = 0.05
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k19 = _params(A)
    p.rob_eps, p.tv_lambda, p.tv_eps = 0.05, 0.1, 1e-3
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k20 = _params(A, psf=synth.box_h(9), schedule=A.RL_SCHED_RESIDENT)
    p.rob_eps = 0.05
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k21 = _params(A, psf=synth.box_h(9))  # auto schedule: two-pass for robust jobs
    p.rob_eps = 0.05
    assert _ws_status(A, p)[0] == A.RL_OK
    # summed-area rectangles: rectangle PSFs only, tables must fit in LDS
    p, k14 = _params(A, psf=synth.box_rect(5, 7), path=A.RL_PATH_BOX_SAT)
    assert _ws_status(A, p)[0] == A.RL_OK
    p, k15 = _params(A, psf=synth.disc(3), path=A.RL_PATH_BOX_SAT)
    assert _ws_status(A, p)[0] == A.RL_E_INVAL
    p, k16 = _params(A, psf=synth.box_rect(127, 101), path=A.RL_PATH_BOX_SAT)
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    # the persistent schedule: plain RL on the span and sliding kernels only
    p, k10 = _params(A, psf=synth.disc(5), schedule=A.RL_SCHED_PERSISTENT)
    assert _ws_status(A, p)[0] == A.RL_OK
    p, k22 = _params(A, psf=synth.oblique_line(15, 30.0), schedule=A.RL_SCHED_PERSISTENT)
    assert _ws_status(A, p)[0] == A.RL_OK
    p, k23 = _params(A, psf=synth.disc(5), schedule=A.RL_SCHED_PERSISTENT,
                     thin=(A.RL_THIN_REL, 1e-4, 5, 10, 10))
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k24 = _params(A, psf=synth.disc(5), schedule=A.RL_SCHED_PERSISTENT)
    p.tv_lambda, p.tv_eps = 0.1, 1e-3
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k25 = _params(A, psf=synth.disc(5), schedule=A.RL_SCHED_PERSISTENT)
    p.rob_eps = 0.05
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k26 = _params(A, psf=synth.box_rect(5, 7), path=A.RL_PATH_BOX_RECT,
                     schedule=A.RL_SCHED_PERSISTENT)
    assert _ws_status(A, p)[0] == A.RL_E_UNSUPPORTED
    p, k11 = _params(A, schedule=9)
    assert _ws_status(A, p)[0] == A.RL_E_INVAL


def test_null_and_state_errors(A):
    L = A.lib()
    assert L.rl_iterate(None, 1) == A.RL_E_INVAL
    assert L.rl_destroy(None) == A.RL_E_INVAL
    assert L.rl_result(None, None, None) == A.RL_E_INVAL
    p, keep = _params(A)
    job = ctypes.c_void_p(0)
    # NULL workspace / NULL f are rejected before any device work
    assert L.rl_init(ctypes.byref(p), None, 0, ctypes.byref(job)) == A.RL_E_INVAL
    n = ctypes.c_int32(0)
    assert L.rl_psf_runs(np.zeros((2, 2), np.float32).ctypes.data, 2, 2, None, None, 0,
                         ctypes.byref(n), None) == A.RL_E_INVAL


def test_tune_cache_roundtrip(A, tmp_path):
    """The tuning cache (host side only): load, lookup, effect on the workspace size,
    save/reload, rejection of malformed files, clear."""
    A.rl_tune_cache_clear()
    psf = synth.disc(5)
    p, keep = _params(A, H=512, W=512, psf=psf)
    assert A.rl_tune_lookup(p) is None
    base = A.rl_workspace_bytes(p)
    runs = len(oracle.psf_runs(psf)[0])
    taps = int(np.count_nonzero(psf))
    bucket = 18  # round(log2(512 * 512))
    # key: path kh kw taps runs bucket thin schedule -> schedule strip seg lpw graph_iters
    f1 = tmp_path / "a.txt"
    f1.write_text("# comment\n"
                  f"3 11 11 {taps} {runs} {bucket} 0 0 1 16 0 0 8\n")
    A.rl_tune_cache_load(f1)
    got = A.rl_tune_lookup(p)
    assert got is not None
    sched, t = got
    assert (sched, t.strip, t.seg, t.lines_per_wg, t.graph_iters) == (1, 16, 0, 0, 8)
    # a neighbouring size bucket and a thinned job do not match the entry
    q, k2 = _params(A, H=64, W=64, psf=psf)
    assert A.rl_tune_lookup(q) is None
    q2, k3 = _params(A, H=512, W=512, psf=psf, thin=(A.RL_THIN_REL, 1e-4, 5, 10, 10))
    assert A.rl_tune_lookup(q2) is None
    # the cached strip length reaches the configuration (and so the workspace layout)
    p.tuning.strip = 16
    explicit = A.rl_workspace_bytes(p)
    p.tuning.strip = 0
    assert A.rl_workspace_bytes(p) == explicit
    # save, clear, reload
    f2 = tmp_path / "b.txt"
    A.rl_tune_cache_save(f2)
    A.rl_tune_cache_clear()
    assert A.rl_tune_lookup(p) is None
    assert A.rl_workspace_bytes(p) == base
    A.rl_tune_cache_load(f2)
    assert A.rl_tune_lookup(p)[1].strip == 16
    # malformed lines are rejected and leave the cache as it was
    for bad in ["3 11 11\n", f"3 11 11 {taps} {runs} {bucket} 0 0 9 16 0 0 8\n",
                f"3 11 11 {taps} {runs} {bucket} 0 0 1 -4 0 0 8\n"]:
        f3 = tmp_path / "bad.txt"
        f3.write_text(bad)
        with pytest.raises(A.RLError):
            A.rl_tune_cache_load(f3)
    assert A.rl_tune_lookup(p)[1].strip == 16
    with pytest.raises(A.RLError):
        A.rl_tune_cache_load(tmp_path / "missing.txt")
    A.rl_tune_cache_clear()
    assert A.rl_tune_lookup(p) is None


def test_static_solve_rejects_oversized_jobs_before_device_work(A):
    """The allocation-free entry point refuses a job whose workspace exceeds its static
    array with RL_E_NOMEM and a reason, before it touches a device (so this runs without
    a GPU); graph replay is refused the same way."""
    L = A.lib()
    p, keep = _params(A, H=4096, W=4096)
    st, need = _ws_status(A, p)
    assert st == A.RL_OK and need > A.RL_STATIC_SCRATCH_BYTES
    assert L.rl_solve_static(ctypes.byref(p), 10, None, None) == A.RL_E_NOMEM
    why = A.last_error()
    assert "rl_solve_static" in why and str(A.RL_STATIC_SCRATCH_BYTES) in why
    p2, keep2 = _params(A)
    p2.tuning.graph_iters = 4
    assert L.rl_solve_static(ctypes.byref(p2), 10, None, None) == A.RL_E_UNSUPPORTED
    assert L.rl_solve_static(ctypes.byref(p2), -1, None, None) == A.RL_E_INVAL
    assert L.rl_solve_static(None, 1, None, None) == A.RL_E_INVAL


def test_last_error_names_the_reason(A):
    L = A.lib()
    p, keep = _params(A, psf=synth.disc(3), path=A.RL_PATH_BOX_AXIS)
    job = ctypes.c_void_p(0)
    ws = ctypes.c_void_p(256)  # never dereferenced: the PSF check fails first
    p.f = 256
    assert L.rl_init(ctypes.byref(p), ws, 1 << 20, ctypes.byref(job)) == A.RL_E_INVAL
    assert "BOX_AXIS" in A.last_error()
