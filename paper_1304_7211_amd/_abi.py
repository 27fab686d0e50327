"""ctypes binding of librl.so -- argument marshalling only.

Every function here has the name and meaning of the C function declared in include/rl.h;
no Richardson-Lucy arithmetic happens in Python.  Importing this module loads the built
library and raises if it is missing: there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librl.so")

RL_OK, RL_E_INVAL, RL_E_NOMEM, RL_E_DEVICE, RL_E_STATE, RL_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
RL_BC_REFLECT, RL_BC_REPLICATE = 0, 1
RL_PATH_AUTO, RL_PATH_DIRECT, RL_PATH_BOX_AXIS, RL_PATH_RUNS, RL_PATH_BOX_RECT, RL_PATH_BOX_SAT = \
    0, 1, 2, 3, 4, 5
RL_PATH_MFMA = 6
RL_SCHED_AUTO, RL_SCHED_TWO_PASS, RL_SCHED_RESIDENT, RL_SCHED_FUSED, RL_SCHED_PERSISTENT = \
    0, 1, 2, 3, 4
RL_THIN_OFF, RL_THIN_ABS, RL_THIN_REL = 0, 1, 2

PATHS = {"auto": 0, "direct": 1, "box_axis": 2, "runs": 3, "box_rect": 4, "box_sat": 5,
         "mfma": 6}
PATH_NAMES = {v: k for k, v in PATHS.items()}
SCHEDS = {"auto": 0, "two_pass": 1, "resident": 2, "fused": 3, "persistent": 4}
SCHED_NAMES = {v: k for k, v in SCHEDS.items()}
BCS = {"reflect": 0, "replicate": 1}
THINS = {"off": 0, "abs": 1, "rel": 2}

# C symbols declared in include/rl.h (checked by the ABI test)
EXPORTS = ["rl_status_str", "rl_workspace_bytes", "rl_init", "rl_iterate", "rl_result",
           "rl_destroy", "rl_batch_workspace_bytes", "rl_iterate_batch", "rl_get_state",
           "rl_set_state", "rl_active_list", "rl_thin_schedule", "rl_psf_runs",
           "rl_timing_enable", "rl_timing_read", "rl_timing_reset", "rl_autotune_workspace_bytes",
           "rl_autotune", "rl_tune_lookup", "rl_tune_cache_save", "rl_tune_cache_load",
           "rl_tune_cache_clear", "rl_job_describe", "rl_debug_spin_limit", "rl_solve_static", "rl_last_error"]

RL_STATIC_SCRATCH_BYTES = 64 << 20


class rl_thin(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tau", ctypes.c_float),
                ("hysteresis", ctypes.c_int32), ("reset_period", ctypes.c_int32),
                ("compact_period", ctypes.c_int32), ("keep_list", ctypes.c_int32),
                ("block", ctypes.c_int32)]


class rl_tuning(ctypes.Structure):
    _fields_ = [("strip", ctypes.c_int32), ("seg", ctypes.c_int32),
                ("lines_per_wg", ctypes.c_int32), ("graph_iters", ctypes.c_int32)]


class rl_params(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("f", ctypes.c_void_p), ("psf_h", ctypes.c_int32), ("psf_w", ctypes.c_int32),
                ("psf", ctypes.c_void_p), ("u0", ctypes.c_void_p),
                ("boundary", ctypes.c_int32), ("path", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("kahan", ctypes.c_int32),
                ("thin", rl_thin), ("stream", ctypes.c_void_p), ("tuning", rl_tuning),
                ("tv_lambda", ctypes.c_float), ("tv_eps", ctypes.c_float),
                ("rob_eps", ctypes.c_float)]


class rl_stats(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int64), ("active_now", ctypes.c_int64),
                ("skipped_px_iters", ctypes.c_int64), ("flux", ctypes.c_double),
                ("path", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("f_invalid", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class rl_job_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("path", "schedule", "tile_h", "tile_w", "strip",
                                             "n_spans", "n_taps", "lmax", "halo_y0",
                                             "halo_y1", "halo_x0", "halo_x1")] + \
               [("ws_bytes", ctypes.c_int64)]


class RLError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        why = last_error()
        super().__init__(f"{fn} failed: {status_str(status)} ({status})"
                         + (f": {why}" if why else ""))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1304_7211_amd.build.build() "
                              "(there is no non-HIP fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "rl_status_str": (ctypes.c_char_p, [i32]),
            "rl_workspace_bytes": (i32, [P(rl_params), P(sz)]),
            "rl_init": (i32, [P(rl_params), vp, sz, P(vp)]),
            "rl_iterate": (i32, [vp, i32]),
            "rl_result": (i32, [vp, vp, P(rl_stats)]),
            "rl_destroy": (i32, [vp]),
            "rl_batch_workspace_bytes": (i32, [i32, P(sz)]),
            "rl_iterate_batch": (i32, [P(vp), P(i32), i32, vp, sz, vp]),
            "rl_get_state": (i32, [vp, vp, vp, vp, P(i64)]),
            "rl_set_state": (i32, [vp, vp, vp, vp, i64]),
            "rl_active_list": (i32, [vp, vp, i64, P(i64)]),
            "rl_thin_schedule": (i32, [vp, P(i64), i32, P(i32)]),
            "rl_psf_runs": (i32, [vp, i32, i32, P(i32), P(ctypes.c_float), i32, P(i32),
                                  P(i32)]),
            "rl_timing_enable": (i32, [i32]),
            "rl_timing_read": (i32, [ctypes.c_char_p, P(i64), P(ctypes.c_double)]),
            "rl_timing_reset": (i32, []),
            "rl_autotune_workspace_bytes": (i32, [P(rl_params), P(sz)]),
            "rl_autotune": (i32, [P(rl_params), vp, sz, i32, P(i32), P(rl_tuning),
                                  P(ctypes.c_double)]),
            "rl_tune_lookup": (i32, [P(rl_params), P(i32), P(rl_tuning)]),
            "rl_tune_cache_save": (i32, [ctypes.c_char_p]),
            "rl_tune_cache_load": (i32, [ctypes.c_char_p]),
            "rl_tune_cache_clear": (i32, []),
            "rl_job_describe": (i32, [vp, P(rl_job_info)]),
            "rl_debug_spin_limit": (i32, [i32, P(i32)]),
            "rl_last_error": (ctypes.c_char_p, []),
            "rl_solve_static": (i32, [P(rl_params), i32, vp, P(rl_stats)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(s):
    return lib().rl_status_str(int(s)).decode()


def last_error():
    return (lib().rl_last_error() or b"").decode()


def check(fn, status):
    if status != RL_OK:
        raise RLError(fn, status)
    return status


# ---- thin wrappers with the C names (pointers are ints; buffers belong to the caller) ----
def rl_workspace_bytes(params):
    n = ctypes.c_size_t(0)
    check("rl_workspace_bytes", lib().rl_workspace_bytes(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def rl_init(params, ws_ptr, ws_bytes):
    job = ctypes.c_void_p(0)
    check("rl_init", lib().rl_init(ctypes.byref(params), ctypes.c_void_p(ws_ptr), ws_bytes,
                                   ctypes.byref(job)))
    return job.value


def rl_iterate(job, n_iter):
    return check("rl_iterate", lib().rl_iterate(ctypes.c_void_p(job), int(n_iter)))


def rl_result(job, u_out_ptr=None, want_stats=False):
    st = rl_stats()
    s = lib().rl_result(ctypes.c_void_p(job), ctypes.c_void_p(u_out_ptr or 0),
                        ctypes.byref(st) if want_stats else None)
    check("rl_result", s)
    return st if want_stats else None


def rl_solve_static(params, n_iter, u_out_ptr=None, want_stats=False):
    st = rl_stats()
    check("rl_solve_static", lib().rl_solve_static(
        ctypes.byref(params), int(n_iter), ctypes.c_void_p(u_out_ptr or 0),
        ctypes.byref(st) if want_stats else None))
    return st if want_stats else None


def rl_debug_spin_limit(polls):
    """Set the persistent schedule's wait limit (test hook); returns the previous one."""
    prev = ctypes.c_int32(0)
    check("rl_debug_spin_limit", lib().rl_debug_spin_limit(int(polls), ctypes.byref(prev)))
    return prev.value


def rl_destroy(job):
    return check("rl_destroy", lib().rl_destroy(ctypes.c_void_p(job)))


def rl_batch_workspace_bytes(n_jobs):
    n = ctypes.c_size_t(0)
    check("rl_batch_workspace_bytes", lib().rl_batch_workspace_bytes(int(n_jobs),
                                                                      ctypes.byref(n)))
    return n.value


def rl_iterate_batch(jobs, n_iter, bws_ptr, bws_bytes, stream_ptr):
    arr = (ctypes.c_void_p * len(jobs))(*jobs)
    its = (ctypes.c_int32 * len(jobs))(*[int(v) for v in n_iter])
    return check("rl_iterate_batch", lib().rl_iterate_batch(
        arr, its, len(jobs), ctypes.c_void_p(bws_ptr), bws_bytes, ctypes.c_void_p(stream_ptr)))


def rl_get_state(job, u_ptr=None, r_ptr=None, cnt_ptr=None):
    k = ctypes.c_int64(0)
    check("rl_get_state", lib().rl_get_state(ctypes.c_void_p(job), ctypes.c_void_p(u_ptr or 0),
                                             ctypes.c_void_p(r_ptr or 0),
                                             ctypes.c_void_p(cnt_ptr or 0), ctypes.byref(k)))
    return k.value


def rl_set_state(job, u_ptr, r_ptr, cnt_ptr, k):
    return check("rl_set_state", lib().rl_set_state(
        ctypes.c_void_p(job), ctypes.c_void_p(u_ptr or 0), ctypes.c_void_p(r_ptr or 0),
        ctypes.c_void_p(cnt_ptr or 0), int(k)))


def rl_active_list(job, list_ptr=None, cap=0):
    n = ctypes.c_int64(0)
    check("rl_active_list", lib().rl_active_list(ctypes.c_void_p(job),
                                                 ctypes.c_void_p(list_ptr or 0), int(cap),
                                                 ctypes.byref(n)))
    return n.value


def rl_thin_schedule(job, cap=4096):
    out = (ctypes.c_int64 * cap)()
    n = ctypes.c_int32(0)
    check("rl_thin_schedule", lib().rl_thin_schedule(ctypes.c_void_p(job), out, cap,
                                                     ctypes.byref(n)))
    return [out[i] for i in range(n.value)]


def rl_psf_runs(psf_f32):
    """psf_f32: C-contiguous numpy float32 (kh, kw).  Returns (runs int32 (n,3), w, cls)."""
    import numpy as np
    kh, kw = psf_f32.shape
    n = ctypes.c_int32(0)
    cls = ctypes.c_int32(0)
    s = lib().rl_psf_runs(psf_f32.ctypes.data, kh, kw, None, None, 0, ctypes.byref(n),
                          ctypes.byref(cls))
    if s not in (RL_OK, RL_E_NOMEM):
        raise RLError("rl_psf_runs", s)
    runs = np.zeros((max(1, n.value), 3), dtype=np.int32)
    w = np.zeros(max(1, n.value), dtype=np.float32)
    check("rl_psf_runs", lib().rl_psf_runs(
        psf_f32.ctypes.data, kh, kw, runs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n.value, ctypes.byref(n),
        ctypes.byref(cls)))
    return runs[:n.value], w[:n.value], cls.value


def rl_timing_enable(on):
    return check("rl_timing_enable", lib().rl_timing_enable(1 if on else 0))


def rl_timing_read(name):
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0)
    check("rl_timing_read", lib().rl_timing_read(name.encode(), ctypes.byref(n),
                                                 ctypes.byref(ms)))
    return n.value, ms.value


def rl_timing_reset():
    return check("rl_timing_reset", lib().rl_timing_reset())


def rl_autotune_workspace_bytes(params):
    n = ctypes.c_size_t(0)
    check("rl_autotune_workspace_bytes",
          lib().rl_autotune_workspace_bytes(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def rl_autotune(params, ws_ptr, ws_bytes, n_iter):
    """Returns (schedule, rl_tuning, milliseconds per iteration) of the fastest candidate."""
    best = rl_tuning()
    sched = ctypes.c_int32(0)
    ms = ctypes.c_double(0)
    check("rl_autotune", lib().rl_autotune(ctypes.byref(params), ws_ptr, ws_bytes, int(n_iter),
                                           ctypes.byref(sched), ctypes.byref(best),
                                           ctypes.byref(ms)))
    return sched.value, best, ms.value


def rl_tune_lookup(params):
    """(schedule, rl_tuning) cached for these parameters, or None."""
    out = rl_tuning()
    sched = ctypes.c_int32(0)
    s = lib().rl_tune_lookup(ctypes.byref(params), ctypes.byref(sched), ctypes.byref(out))
    if s == RL_E_STATE:
        return None
    check("rl_tune_lookup", s)
    return sched.value, out


def rl_tune_cache_save(path):
    return check("rl_tune_cache_save", lib().rl_tune_cache_save(str(path).encode()))


def rl_tune_cache_load(path):
    return check("rl_tune_cache_load", lib().rl_tune_cache_load(str(path).encode()))


def rl_tune_cache_clear():
    return check("rl_tune_cache_clear", lib().rl_tune_cache_clear())


def rl_job_describe(job):
    info = rl_job_info()
    check("rl_job_describe", lib().rl_job_describe(ctypes.c_void_p(job), ctypes.byref(info)))
    return info
