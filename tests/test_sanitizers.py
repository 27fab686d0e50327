"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

The FP64 oracle (oracle/rl_oracle.c) and the library's PSF compiler
(paper_1304_7211_amd/csrc/psf_compile.cpp) are built with gcc / g++ and
``-fsanitize=address,undefined -fno-sanitize-recover=all`` into two small drivers
(tests/sanitize/), which run on tiny cases chosen to reach the edges: 1 x 1 and 1 x N
images, PSFs larger than the image (folds deeper than the image, both boundaries), even
PSF sizes, every thinning mode.  Any sanitizer report ends the driver with a non-zero
status.  The oracle driver's results must equal the regular oracle build's bit for bit;
the PSF compiler's run lists must equal the oracle-side definition bit for bit (P13), and
every operator table it can build must cover exactly the non-zero taps.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    ora = str(d / "oracle_driver")
    psf = str(d / "psf_driver")
    subprocess.check_call(["gcc", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-Wno-unknown-pragmas"] + SAN +
                          [os.path.join(HERE, "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "rl_oracle.c"), "-o", ora, "-lm"])
    csrc = os.path.join(ROOT, "paper_1304_7211_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17"] + SAN +
                          ["-I", csrc, "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "sanitize", "psf_driver.cpp"),
                           os.path.join(csrc, "psf_compile.cpp"), "-o", psf])
    return ora, psf


def _run(exe, text):
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=ENV, timeout=120)
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    return r.stdout


def _parse(out):
    res, lines, i = {}, out.splitlines(), 0
    while i < len(lines):
        name, n = lines[i].split()
        n = int(n)
        res[name] = np.array([float.fromhex(x) for x in lines[i + 1:i + 1 + n]])
        i += 1 + n
    return res


ORACLE_CASES = [
    (1, 1, synth.disc(2), "reflect"),
    (1, 7, synth.box_h(9), "replicate"),
    (5, 1, synth.box_v(12), "reflect"),
    (3, 4, synth.dense_random(5, 2), "reflect"),
    (6, 5, synth.oblique_line(9, 30.0), "replicate"),
    (9, 8, np.ones((2, 4), np.float32) / 8, "reflect"),
    (12, 11, synth.disc(3), "replicate"),
]


@pytest.mark.parametrize("H,W,h,bc", ORACLE_CASES,
                         ids=[f"{c[0]}x{c[1]}-{c[2].shape[0]}x{c[2].shape[1]}-{c[3]}"
                              for c in ORACLE_CASES])
@pytest.mark.parametrize("mode", ["abs", "rel"])
def test_oracle_under_sanitizers(drivers, H, W, h, bc, mode):
    rng = np.random.default_rng(H * 100 + W)
    f = (0.1 + rng.random((H, W))).astype(np.float32)
    f[rng.random((H, W)) < 0.1] = 0.0  # exact zeros: the v <= 0 ratio rule
    K = 6
    thin = dict(mode=mode, tau=0.05 if mode == "abs" else 0.05, hysteresis=2,
                reset_period=3, compact_period=3)
    hdr = (f"{H} {W} {h.shape[0]} {h.shape[1]} {oracle.BC[bc]} {K} {oracle.THIN[mode]} "
           f"{float(np.float32(thin['tau'])).hex()} {thin['hysteresis']} {thin['reset_period']}")
    vals = [float(np.float64(v)).hex() for v in f.ravel()] + \
           [float(np.float64(v)).hex() for v in h.ravel()]
    got = _parse(_run(drivers[0], hdr + "\n" + "\n".join(vals) + "\n"))
    o = oracle.Oracle()
    f64 = f.astype(np.float64)
    assert np.array_equal(got["conv"].reshape(H, W), o.conv(f64, h, bc))
    assert np.array_equal(got["corr"].reshape(H, W), o.corr(f64, h, bc))
    assert np.array_equal(got["rl"].reshape(H, W), o.rl(f, h, K, bc))
    th = o.rl_thin(f, h, K, thin, bc)
    assert np.array_equal(got["thin_u"].reshape(H, W), th["u"])
    assert np.array_equal(got["thin_r"].reshape(H, W), th["r"])
    assert np.array_equal(got["thin_cnt"].reshape(H, W), th["cnt"].astype(np.float64))
    assert np.array_equal(got["thin_active"], th["active"].astype(np.float64))
    tb = o.rl_thin(f, h, K, dict(thin, block=3), bc)
    assert np.array_equal(got["block_u"].reshape(H, W), tb["u"])
    assert np.array_equal(got["block_cnt"].reshape(H, W), tb["cnt"].astype(np.float64))
    assert np.array_equal(got["block_active"], tb["active"].astype(np.float64))
    assert np.array_equal(got["tv"].reshape(H, W), o.rl_tv(f, h, K, 0.1, 1e-3, bc))
    assert np.array_equal(got["robust"].reshape(H, W), o.rl_robust(f, h, K, 0.05, bc))
    assert got["sum"][0] == o.sum(f64)


def _psf_cases():
    yield synth.delta()
    for L in (1, 2, 5, 16, 63):
        yield synth.box_h(L)
        yield synth.box_v(L)
    for r in (1, 3, 10, 24):
        yield synth.disc(r)
    for L, a in ((9, 0.0), (31, 30.0), (47, 75.0), (17, 45.0), (25, 137.0), (13, 180.0)):
        yield synth.oblique_line(L, a)
    yield synth.dense_random(15, 3)
    yield synth.dense_random(4, 9)  # even size
    yield synth.box_rect(5, 7)
    yield synth.box_rect(127, 2)
    z = np.zeros((7, 9), np.float32)
    z[2:5, 3:8] = 1.0 / 15  # a rectangle inside zero margins
    yield z
    yield np.array([[0, 1, 1, 2, 0, 3], [0, 0, 0, 0, 0, 0], [5, 5, 5, 5, 5, 5]], np.float32)
    g = np.zeros((1, 127), np.float32)
    g[0, ::2] = 1.0  # the longest PSF line, gaps everywhere
    yield g


def test_psf_compiler_under_sanitizers(drivers):
    cases = list(_psf_cases())
    invalid = [np.array([[0.5, -0.1, 0.6]], np.float32), np.array([[0.5, np.inf]], np.float32),
               np.zeros((3, 3), np.float32)]
    text = [str(len(cases) + len(invalid))]
    for h in cases + invalid:
        text.append(f"{h.shape[0]} {h.shape[1]}")
        text.append(" ".join(float(np.float64(v)).hex() for v in h.ravel()))
    out = _run(drivers[1], "\n".join(text) + "\n")
    blocks = {}
    cur = None
    for ln in out.splitlines():
        parts = ln.split()
        if parts[0] == "psf":
            cur = int(parts[1])
            blocks[cur] = dict(valid=int(parts[2]), runs=[])
        elif parts[0] == "run":
            blocks[cur]["runs"].append((int(parts[1]), int(parts[2]), int(parts[3]),
                                        np.float32(float.fromhex(parts[4]))))
        else:
            raise AssertionError(ln)
    assert len(blocks) == len(cases) + len(invalid)
    for i, h in enumerate(cases):
        ints, ws = oracle.psf_runs(h)
        got = blocks[i]["runs"]
        assert blocks[i]["valid"] == 1
        assert [g[:3] for g in got] == [tuple(int(v) for v in row) for row in ints], i
        assert np.array_equal(np.array([g[3] for g in got], np.float32).view(np.uint32),
                              np.asarray(ws, np.float32).view(np.uint32)), i
    for j in range(len(invalid)):
        assert blocks[len(cases) + j]["valid"] == 0
