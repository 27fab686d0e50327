"""FP64 CPU oracle for Richardson-Lucy deconvolution -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product path (``paper_1304_7211_amd``) never imports it, and
this package imports nothing from the product path.

The arithmetic lives in ``rl_oracle.c`` (plain C, FP64, compiled with gcc); this module
is the ctypes shim plus two pieces of pure-Python definition:
  * ``psf_runs``: the integer run list of a PSF (maximal spans of bit-identical non-zero
    weights in each PSF row), the representation behind the paper's list filter and
    generic box filter (Section 3, "Defocus blur" and "Sparse blur");
  * ``is_rebuild``: when the compacted active list of thinned RL is rebuilt.

Function index (each cites the passage it follows):
  conv, corr          Section 1 eq. 2 (u*h) and Section 2 eq. 3 (h^* * r)
  rl                  Section 2 eq. 3, u^0 = f
  thin_step, rl_thin  Section 4 eq. 4-5 and the every-ten-iterations reset; with
                      thin["block"] > 1 the block rule (freeze decisions per tile), a
                      refinement of Section 4's adaptive rule
  below               Section 4 convergence test (float32 decision)
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_SRC = os.path.join(_HERE, "rl_oracle.c")

BC = {"reflect": 0, "replicate": 1}
THIN = {"off": 0, "abs": 1, "rel": 2}

_libs = {}
_lock = threading.Lock()


def lib_path(mutant=0):
    name = "liboracle.so" if mutant == 0 else f"liboracle_m{mutant}.so"
    return os.path.join(_BUILD, name)


def build(mutant=0, force=False):
    """Compile the oracle with gcc (FP64, no FP contraction, OpenMP over rows)."""
    out = lib_path(mutant)
    if os.path.exists(out) and not force and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    os.makedirs(_BUILD, exist_ok=True)
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
           "-fPIC", f"-DORACLE_MUTANT={int(mutant)}", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def _load(mutant=0):
    with _lock:
        if mutant in _libs:
            return _libs[mutant]
        lib = ctypes.CDLL(build(mutant))
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_fold.restype = ctypes.c_long
        lib.oracle_fold.argtypes = [ctypes.c_long, ctypes.c_long, ctypes.c_int]
        for fn in (lib.oracle_conv, lib.oracle_corr):
            fn.restype = None
            fn.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                           ctypes.c_int, dp]
        lib.oracle_rl.restype = None
        lib.oracle_rl.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_thin_step.restype = ctypes.c_long
        lib.oracle_thin_step.argtypes = [dp, dp, dp, ctypes.POINTER(ctypes.c_uint8),
                                         ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                         ctypes.c_int, ctypes.c_float, ctypes.c_int,
                                         ctypes.c_int, dp]
        lib.oracle_thin_step_blocks.restype = ctypes.c_long
        lib.oracle_thin_step_blocks.argtypes = [dp, dp, dp, ctypes.POINTER(ctypes.c_uint8),
                                                ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                                ctypes.c_int, ctypes.c_float, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_below.restype = ctypes.c_int
        lib.oracle_below.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                     ctypes.c_float]
        lib.oracle_below_many.restype = None
        lib.oracle_below_many.argtypes = [ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_float), ctypes.c_long,
                                          ctypes.c_int, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_tv_div.restype = None
        lib.oracle_tv_div.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        lib.oracle_rl_tv.restype = None
        lib.oracle_rl_tv.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, dp, dp]
        lib.oracle_idiv.restype = ctypes.c_double
        lib.oracle_idiv.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_rl_robust.restype = None
        lib.oracle_rl_robust.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, dp, dp, dp, dp]
        lib.oracle_robust_terms.restype = None
        lib.oracle_robust_terms.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_double, dp, dp, dp, dp]
        lib.oracle_sum.restype = ctypes.c_double
        lib.oracle_sum.argtypes = [dp, ctypes.c_long]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        _libs[mutant] = lib
        return lib


class Oracle:
    """Bound oracle; ``Oracle(mutant=k)`` loads a variant with one planted mistake."""

    def __init__(self, mutant=0):
        self.lib = _load(mutant)

    @staticmethod
    def _d(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def fold(self, i, n, bc="reflect"):
        return int(self.lib.oracle_fold(int(i), int(n), BC[bc]))

    def conv(self, u, h, bc="reflect"):
        """(u*h)(y,x) = sum_ij h[i][j] u[fold(y-(i-oy))][fold(x-(j-ox))]  (Section 1, eq. 2)."""
        u, up = self._d(u)
        h, hp = self._d(h)
        out = np.empty_like(u)
        self.lib.oracle_conv(up, u.shape[0], u.shape[1], hp, h.shape[0], h.shape[1], BC[bc],
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def corr(self, r, h, bc="reflect"):
        """(h^* * r)(y,x) = sum_ij h[i][j] r[fold(y+(i-oy))][fold(x+(j-ox))]  (Section 2)."""
        r, rp = self._d(r)
        h, hp = self._d(h)
        out = np.empty_like(r)
        self.lib.oracle_corr(rp, r.shape[0], r.shape[1], hp, h.shape[0], h.shape[1], BC[bc],
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def rl(self, f, h, K, bc="reflect", u0=None):
        """K plain RL iterations from u^0 = f (or ``u0``)  (Section 2, eq. 3)."""
        f, fp = self._d(f)
        u, up = self._d(np.array(f if u0 is None else u0, dtype=np.float64, copy=True))
        h, hp = self._d(h)
        r = np.empty_like(f)
        self.lib.oracle_rl(fp, up, f.shape[0], f.shape[1], hp, h.shape[0], h.shape[1],
                           BC[bc], int(K), r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return u

    def tv_div(self, u, eps):
        """div(grad u / |grad u|_eps) of the TV-regularised variant (forward gradient,
        backward divergence, zero flux at the edges)."""
        u, up = self._d(u)
        out = np.empty_like(u)
        self.lib.oracle_tv_div(up, u.shape[0], u.shape[1], float(eps),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def rl_tv(self, f, h, K, lam, eps, bc="reflect", u0=None):
        """K iterations of TV-regularised RL from u^0 = f (or ``u0``)."""
        f, fp = self._d(f)
        u, up = self._d(np.array(f if u0 is None else u0, dtype=np.float64, copy=True))
        h, hp = self._d(h)
        r = np.empty_like(f)
        d = np.empty_like(f)
        dp = ctypes.POINTER(ctypes.c_double)
        self.lib.oracle_rl_tv(fp, up, f.shape[0], f.shape[1], hp, h.shape[0], h.shape[1],
                              BC[bc], int(K), float(lam), float(eps), r.ctypes.data_as(dp),
                              d.ctypes.data_as(dp))
        return u

    def idiv(self, v, f):
        """Pointwise I-divergence d(v, f) = v - f - f ln(v / f) of the robust variant."""
        return float(self.lib.oracle_idiv(float(v), float(f)))

    def rl_robust(self, f, h, K, eps, bc="reflect", u0=None):
        """K iterations of RL with the robustified data term (weights 1/sqrt(d + eps^2) of
        the I-divergence d) from u^0 = f (or ``u0``)."""
        f, fp = self._d(f)
        u, up = self._d(np.array(f if u0 is None else u0, dtype=np.float64, copy=True))
        h, hp = self._d(h)
        work = [np.empty_like(f) for _ in range(4)]
        dp = ctypes.POINTER(ctypes.c_double)
        self.lib.oracle_rl_robust(fp, up, f.shape[0], f.shape[1], hp, h.shape[0], h.shape[1],
                                  BC[bc], int(K), float(eps), *[a.ctypes.data_as(dp) for a in work])
        return u

    def robust_terms(self, f, u, h, eps, bc="reflect"):
        """(num, den) of one robust iteration at u: h^* * (w f / v) and h^* * w."""
        f, fp = self._d(f)
        u, up = self._d(u)
        h, hp = self._d(h)
        work = [np.empty_like(f) for _ in range(4)]
        dp = ctypes.POINTER(ctypes.c_double)
        self.lib.oracle_robust_terms(fp, up, f.shape[0], f.shape[1], hp, h.shape[0], h.shape[1],
                                     BC[bc], float(eps), *[a.ctypes.data_as(dp) for a in work])
        return work[2], work[3]

    def below(self, a, b, mode, tau):
        """float32 convergence decision of Section 4 (ABS or REL threshold)."""
        return bool(self.lib.oracle_below(float(np.float32(a)), float(np.float32(b)),
                                          THIN[mode], float(np.float32(tau))))

    def below_many(self, a, b, mode, tau):
        """The same decision for every pair of two float32 arrays (bool array)."""
        a = np.ascontiguousarray(a, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        assert a.shape == b.shape
        out = np.empty(a.shape, dtype=np.uint8)
        fp = ctypes.POINTER(ctypes.c_float)
        self.lib.oracle_below_many(a.ctypes.data_as(fp), b.ctypes.data_as(fp), a.size,
                                   THIN[mode], float(np.float32(tau)),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return out.astype(bool)

    def thin_step(self, f, u, r, cnt, h, k, thin, bc="reflect"):
        """One thinned iteration k, in place on u, r (float64) and cnt (uint8).

        Returns |A_k|, the number of active pixels (Section 4, eq. 4-5)."""
        H, W = f.shape
        fd, fp = self._d(f)
        hd, hp = self._d(h)
        assert u.dtype == np.float64 and r.dtype == np.float64 and cnt.dtype == np.uint8
        assert u.flags.c_contiguous and r.flags.c_contiguous and cnt.flags.c_contiguous
        work = np.empty((H, W), dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        block = int(thin.get("block", 0))
        if block > 1:  # block rule: freeze decisions per block x block tile
            return int(self.lib.oracle_thin_step_blocks(
                fp, u.ctypes.data_as(dp), r.ctypes.data_as(dp),
                cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), H, W, hp, hd.shape[0],
                hd.shape[1], BC[bc], int(k), THIN[thin["mode"]], float(np.float32(thin["tau"])),
                int(thin["hysteresis"]), int(thin["reset_period"]), block,
                work.ctypes.data_as(dp)))
        return int(self.lib.oracle_thin_step(
            fp, u.ctypes.data_as(dp), r.ctypes.data_as(dp),
            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), H, W, hp, hd.shape[0],
            hd.shape[1], BC[bc], int(k), THIN[thin["mode"]], float(np.float32(thin["tau"])),
            int(thin["hysteresis"]), int(thin["reset_period"]), work.ctypes.data_as(dp)))

    def thin_step_blocks(self, f, u, r, cnt, h, k, thin, block, bc="reflect"):
        """One thinned iteration under the block rule with the given block size (block = 1
        calls the block code with 1 x 1 blocks, for the check against the per-pixel rule)."""
        H, W = f.shape
        fd, fp = self._d(f)
        hd, hp = self._d(h)
        assert u.dtype == np.float64 and r.dtype == np.float64 and cnt.dtype == np.uint8
        work = np.empty((H, W), dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        return int(self.lib.oracle_thin_step_blocks(
            fp, u.ctypes.data_as(dp), r.ctypes.data_as(dp),
            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), H, W, hp, hd.shape[0],
            hd.shape[1], BC[bc], int(k), THIN[thin["mode"]], float(np.float32(thin["tau"])),
            int(thin["hysteresis"]), int(thin["reset_period"]), int(block),
            work.ctypes.data_as(dp)))

    def rl_thin(self, f, h, K, thin, bc="reflect", u0=None, keep_lists=False,
                callback=None):
        """K thinned RL iterations from u^0 = f (Section 4).

        Returns dict(u, r, cnt, active (per iteration |A_k|), flux (sum u^k, k = 0..K),
        lists ({k: ascending active indices} at rebuild points if ``keep_lists``))."""
        f64 = np.ascontiguousarray(f, dtype=np.float64)
        u = np.array(f64 if u0 is None else u0, dtype=np.float64, copy=True)
        r = np.zeros_like(u)
        cnt = np.zeros(u.shape, dtype=np.uint8)
        active, flux, lists = [], [self.sum(u)], {}
        for k in range(int(K)):
            if keep_lists and is_rebuild(k, thin["reset_period"], thin["compact_period"]):
                lists[k] = np.flatnonzero(cnt.reshape(-1) < thin["hysteresis"])
            active.append(self.thin_step(f64, u, r, cnt, h, k, thin, bc))
            flux.append(self.sum(u))
            if callback is not None:
                callback(k, u, r, cnt)
        return dict(u=u, r=r, cnt=cnt, active=np.array(active, dtype=np.int64),
                    flux=np.array(flux), lists=lists)

    def threads(self):
        """Threads the row loops use (OpenMP's current maximum)."""
        return int(self.lib.oracle_threads())

    def set_threads(self, n):
        """Thread count of the row loops; the results do not depend on it."""
        self.lib.oracle_set_threads(int(n))

    def sum(self, a):
        a, ap = self._d(a)
        return float(self.lib.oracle_sum(ap, a.size))


def is_full(k, reset_period):
    """Iteration k is a full step: k = 0, or every R-th iteration (Section 4)."""
    return k == 0 or (reset_period > 0 and k % reset_period == 0)


def is_rebuild(k, reset_period, compact_period):
    """The compacted active list is rebuilt at the start of non-full iteration k when the
    previous iteration was full or when (k - 1) is a multiple of the compaction period.
    The list never changes the arithmetic (pixels with cnt >= H are skipped either way);
    it only decides which pixels the work is spread over."""
    if is_full(k, reset_period):
        return False
    return is_full(k - 1, reset_period) or (compact_period > 0 and (k - 1) % compact_period == 0)


def psf_runs(h):
    """Integer run list of a float32 PSF: for each PSF row i (ascending), maximal spans of
    consecutive columns whose weights are non-zero and bit-identical.  Each run is
    (dy, x0, x1, w) with dy = i - oy, x0/x1 = first/last column offset (j - ox), and w
    the float32 weight.  Returns (int32 array (n, 3), float32 array (n,))."""
    h = np.ascontiguousarray(h, dtype=np.float32)
    kh, kw = h.shape
    oy, ox = kh // 2, kw // 2
    bits = h.view(np.uint32)
    ints, ws = [], []
    for i in range(kh):
        j = 0
        while j < kw:
            if h[i, j] == 0.0:
                j += 1
                continue
            j1 = j
            while j1 + 1 < kw and bits[i, j1 + 1] == bits[i, j] and h[i, j1 + 1] != 0.0:
                j1 += 1
            ints.append((i - oy, j - ox, j1 - ox))
            ws.append(h[i, j])
            j = j1 + 1
    return (np.array(ints, dtype=np.int32).reshape(-1, 3), np.array(ws, dtype=np.float32))
