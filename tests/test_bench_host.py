"""Host-side logic of bench.py (no GPU): counter summaries, kernel-name mapping, the
algorithmic flop model and the refusal of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _pmc(dirname, counter, rows):
    os.makedirs(dirname, exist_ok=True)
    with open(os.path.join(dirname, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow(dict(Kernel_Name=name, Counter_Name=counter, Counter_Value=value))


def test_summarize_pmc_scales_by_the_calibration_copy(tmp_path):
    span = "void rlk::span_kernel<0, 8, 8, 8, true>(rlk::LaunchArgs)"
    copy = "__amd_rocclr_copyBuffer"
    # the copy of 1 MiB reads half of what it moves by this counter, writes all of it
    _pmc(tmp_path / "f", "FETCH_SIZE", [(copy, 512.0), (span, 1000.0), (span, 1200.0)])
    _pmc(tmp_path / "w", "WRITE_SIZE", [(copy, 1024.0), (span, 400.0), (span, 400.0)])
    text = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), 1, "cmd")
    data = json.loads(text[text.index("```json") + 7:text.rindex("```")])
    assert data["scale"] == {"fetch": 2.0, "write": 1.0}
    # (1100 KiB * 2 + 400 KiB * 1) per launch
    assert data["bytes_per_launch"]["span_corr_update"] == (1100 * 2 + 400) * 1024
    assert data["source_sha256"] == bench.kernel_source_hash()


def test_timing_names():
    n = bench._timing_name
    assert n("void rlk::span_kernel<0, 8, 8, 8, false>(rlk::LaunchArgs)") == "span_conv_ratio"
    assert n("void rlk::span_kernel<1, 4, 1, 8, true>(rlk::LaunchArgs)") == "direct_corr_update"
    assert n("void rlk::slide_kernel<0, 8, 8, true>(rlk::LaunchArgs)") == "slide_corr_update"
    assert n("void rlk::rect_kernel<8, 8, false>(rlk::LaunchArgs)") == "rect_conv_ratio"
    assert n("void rlk::sat_kernel<4, 8, true>(rlk::LaunchArgs)") == "sat_corr_update"
    assert n("void rlk::resident_kernel<1, 8>(rlk::ResidentArgs)") == "resident_box"
    assert n("void rlk::resident_multi_kernel<0, 16>(rlk::ResidentArgs const*, int const*, int)") \
        == "resident_box"
    assert n("void rlk::mfma_kernel<8, true>(rlk::LaunchArgs)") == "mfma_corr_update"
    assert n("void rlk::mfma_kernel<4, false>(rlk::LaunchArgs)") == "mfma_conv_ratio"
    assert n("__amd_rocclr_copyBuffer") is None


def test_flop_model():
    f = bench.algorithmic_flops_per_px
    assert f("direct", dict(n_taps=87, n_spans=17), False) == 2 * 87 + 1
    assert f("span", dict(n_taps=87, n_spans=17), True) == 2 * 87 + 1
    assert f("slide", dict(n_taps=317, n_spans=21), False) == 2 * 21 + 1
    assert f("rect", {}, True) == 5
    assert f("resident", {}, False) == 3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _stats(dirname, rows):
    os.makedirs(dirname, exist_ok=True)
    with open(os.path.join(dirname, "bench_kernel_stats.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs",
                                           "MinNs", "MaxNs", "Percentage"])
        w.writeheader()
        for name, calls, avg in rows:
            w.writerow(dict(Name=name, Calls=calls, TotalDurationNs=calls * avg, AverageNs=avg,
                            MinNs=avg, MaxNs=avg, Percentage=50.0))


def test_summaries_of_a_size_sweep_run(tmp_path):
    span = "void rlk::span_kernel<0, 8, 8, 8, false>(rlk::LaunchArgs)"
    _stats(tmp_path / "kt", [(span, 63, 90000.0)])
    log = tmp_path / "r7.log"
    log.write_text(json.dumps(dict(report="sweep", rows=[dict(
        psf="oblique", side=4096, kernels=dict(span_conv_ratio=dict(us=91.0, hbm_frac=0.28)))]))
        + "\n")
    text = bench.summarize_trace(str(tmp_path / "kt"), str(log), "cmd", 4096)
    assert "4096x4096" in text and "| 63 | 5.67 | 90.00 |" in text
    assert "oblique `span_conv_ratio`: 91.00 us per launch" in text
    copy = "__amd_rocclr_copyBuffer"
    _pmc(tmp_path / "f", "FETCH_SIZE", [(copy, 512.0), (span, 1000.0)])
    _pmc(tmp_path / "w", "WRITE_SIZE", [(copy, 1024.0), (span, 400.0)])
    text = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), 1, "cmd", 4096)
    assert "at 4096 x 4096: 6 B per pixel" in text and "= 96.0 MiB" in text


def test_pooled_traffic_over_template_instances(tmp_path):
    """Two kernel symbols with one registry name: bytes_per_launch is their scaled total
    over their dispatch count."""
    a = "void rlk::span_kernel<0, 8, 16, 8, false>(rlk::LaunchArgs)"
    b = "void rlk::span_kernel<1, 4, 8, 8, false>(rlk::LaunchArgs)"
    copy = "__amd_rocclr_copyBuffer"
    _pmc(tmp_path / "f", "FETCH_SIZE", [(copy, 512.0), (a, 100.0), (a, 300.0), (b, 50.0)])
    _pmc(tmp_path / "w", "WRITE_SIZE", [(copy, 1024.0), (a, 10.0), (a, 10.0), (b, 40.0)])
    text = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), 1, "cmd")
    data = json.loads(text[text.index("```json") + 7:text.rindex("```")])
    want = ((100 + 300 + 50) * 2 + (10 + 10 + 40)) * 1024 / 3
    assert data["bytes_per_launch"]["span_conv_ratio"] == round(want)


class _FakeAbi:
    RL_SCHED_RESIDENT, RL_PATH_BOX_RECT, RL_PATH_BOX_SAT, RL_PATH_MFMA = 2, 4, 5, 6


def test_roofline_accounting():
    """12 B per pixel-iteration: 6 B per output of each phase launch, 12 B x K per
    output of a resident launch; the bound is the resource with the longer minimum
    time."""
    import numpy as np
    jobs = [dict(name="a", f=np.zeros((100, 50), np.float32), iters=10),
            dict(name="b", f=np.zeros((20, 10), np.float32), iters=4),
            dict(name="c", f=np.zeros((30, 30), np.float32), iters=7)]
    infos = {"a": dict(schedule=1, path=3, lmax=0, n_spans=21, n_taps=317),
             "b": dict(schedule=1, path=3, lmax=0, n_spans=21, n_taps=317),
             "c": dict(schedule=2, path=2, lmax=0, n_spans=1, n_taps=41)}
    work = bench.kernel_work(_FakeAbi, jobs, infos)
    px_it = 5000 * 10 + 200 * 4
    assert work["slide_conv_ratio"]["bytes"] == 6.0 * px_it
    assert work["slide_corr_update"]["flops"] == (2 * 21 + 1) * px_it
    assert work["resident_box"]["bytes"] == 12.0 * 900 * 7
    # 10 launches of 1 us each: bytes per launch 6 B x px_it / 10
    kernels = {"slide_conv_ratio": dict(launches=10, total_ms=0.01, avg_us=1.0),
               "resident_box": dict(launches=1, total_ms=0.001, avg_us=1.0)}
    rf = bench.roofline_of(kernels, work, lambda nm: None)
    assert rf["kernel"] == "slide_conv_ratio"
    by = 6.0 * px_it / 10
    fl = (2 * 21 + 1) * px_it / 10
    assert rf["bytes_per_launch"] == round(by)
    # 43 flops per 6 B (7.2 flop/B) is below the machine balance (157.3e12 / 8e12 =
    # 19.7 flop/B): HBM binds
    assert rf["bound"] == "hbm"
    assert abs(rf["achieved"] - by / 1e-6 / 1e9) < 1e-2
    assert abs(rf["frac"] - by / 1e-6 / 1e9 / bench.PEAK_HBM_GBS) < 1e-5
    assert abs(rf["alu_frac"] - fl / 1e-6 / 1e12 / bench.PEAK_FP32_TFLOPS) < 1e-5
    # a dense 15 x 15 PSF (451 flops per output of a phase) is bound by the ALUs
    infos["a"] = dict(schedule=1, path=3, lmax=16, n_spans=15, n_taps=225)
    infos["b"] = dict(infos["a"])
    work = bench.kernel_work(_FakeAbi, jobs, infos)
    kernels = {"span_corr_update": dict(launches=10, total_ms=0.01, avg_us=1.0)}
    rf = bench.roofline_of(kernels, work, lambda nm: None)
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s"
    fl = (2 * 225 + 1) * px_it / 10
    assert abs(rf["frac"] - fl / 1e-6 / 1e12 / bench.PEAK_FP32_TFLOPS) < 1e-5


def test_roofline_of_matrix_core_kernel():
    """The matrix-core kernel's roof is the dense FP32 matrix peak (label "mfma")."""
    import numpy as np
    jobs = [dict(name="a", f=np.zeros((64, 64), np.float32), iters=10)]
    infos = {"a": dict(schedule=1, path=6, lmax=0, n_spans=15, n_taps=225)}
    work = bench.kernel_work(_FakeAbi, jobs, infos)
    kernels = {"mfma_corr_update": dict(launches=10, total_ms=0.01, avg_us=1.0)}
    rf = bench.roofline_of(kernels, work, lambda nm: None)
    assert rf["bound"] == "mfma" and rf["peak"] == bench.PEAK_FP32_TFLOPS


def test_summarize_counters_per_wavefront(tmp_path):
    """Each counter's per-dispatch total divided by the dispatch's wavefronts; SQ_WAVES
    from the pass that has it, small kernels left out."""
    d1, d2 = tmp_path / "a", tmp_path / "b"
    k = "void rlk::span_kernel<0, 8, 8, 8, false>(rlk::LaunchArgs)"
    for d, rows in ((d1, [("SQ_WAVES", 1, 1000.0), ("SQ_WAVES", 1, 1000.0), ("SQ_INSTS_VALU", 1, 5e5),
                          ("SQ_INSTS_VALU", 1, 7e5), ("SQ_WAVES", 2, 2000.0), ("SQ_INSTS_VALU", 2, 2e6)]),
                    (d2, [("SQ_INSTS_SALU", 1, 1e6), ("SQ_INSTS_SALU", 2, 3e6)])):
        os.makedirs(d)
        with open(d / "run_counter_collection.csv", "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                               "Counter_Value"])
            w.writeheader()
            for c, disp, v in rows:
                w.writerow(dict(Dispatch_Id=disp, Kernel_Name=k, Counter_Name=c, Counter_Value=v))
    text = bench.summarize_counters([str(d1), str(d2)], "cmd")
    row = [l for l in text.splitlines() if "span_kernel" in l][0]
    # 2 dispatches, 2000 wavefronts each on average (one of them summed over two engines);
    # VALU 1.2e6 + 2e6 over two dispatches / 2000 = 800; SALU 4e6 / 2 / 2000 = 1000
    assert row == "| `rlk::span_kernel<0, 8, 8, 8, false>` | 2 | 2000 | 800 | 1000 |"
