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
    assert "at 4096 x 4096: 12 B per pixel" in text and "= 192.0 MiB" in text
