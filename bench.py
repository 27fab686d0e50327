"""Benchmark: Richardson-Lucy pixel-iterations per second on one MI355X.

Default workload (one "step"): the batched configuration -- 256 float32 images from the
seeded generator, sides drawn log-uniformly in 256..2048 (non-square), each with a PSF
drawn uniformly from {axis-aligned motion box of length 5-63, antialiased oblique motion
line of length 9-47 at a uniform angle, uniform disc of radius 3-24, dense 15 x 15
random}, Poisson noise at peak 255, 100-300 RL iterations each, compensated float32 sums.
A step runs every job end to end through the C ABI: rl_init for each (copy f into its
workspace, upload the compiled PSF), ONE rl_iterate_batch call that advances all of them
by their own iteration counts, and rl_result for each (copy u^K out).  Inputs are
resident on the GPU before the timed region starts.

The line's `accuracy` compares the outputs of the last timed step of the two cheapest
jobs of each PSF class with full-length FP64 oracle runs (the same runs time the CPU
baseline).  `roofline` belongs to the kernel with the largest total time, charged
12 B per pixel-iteration (6 B per output of each of the two phase launches of an
iteration), or its algorithmic flops where those bind.

--workload specialised times the specialised-PSF configuration instead: three 1024 x 1024
images (vertical box 41 -> BOX_AXIS, oblique line 31 at 30 deg -> RUNS spans, disc r=10 ->
RUNS sliding runs), Gaussian noise sigma 0.01, 200 iterations each, all three checked
against the oracle at full length.  --mode sequential runs rl_iterate per job instead of
one batch call (the plain per-image method).

Prints ONE JSON line.  Options: --gpus (must be 1), --steps, --warmup, --workload,
--no-cpu-baseline, --no-kernel-timing, --no-kahan, --mode, --compare.

--report N prints, instead of the benchmark line, one JSON report line for another
configuration:
  1  plain RL, 128x128, horizontal box 15, Poisson 255, 50 iterations: microseconds per
     solve (init, iterations, result) for each path, and the error against the oracle;
  3  thinned RL, 2048x2048, disc r=16, Poisson 1000, 500 iterations, relative threshold
     1e-4 held 5 iterations, reset and recompaction every 10: thinning-rate schedule,
     omitted fraction, PSNR against the unthinned GPU run, both timings;
  4  256 uneven images (sides log-uniform 256..2048, mixed PSFs, 100..300 iterations) in
     one batch: throughput with compensated and plain float32 sums, and the error of both
     against the FP64 oracle on the two cheapest jobs of each PSF class;
  5  serving: Poisson arrivals of 1000 requests drawn from a pool (sides 128..4096, mixed
     PSFs, 50..500 iterations, thinning on) at 70 % of the measured batched capacity:
     p50/p99 latency and throughput of the continuous-batching server against the plain
     one-at-a-time method on the same GPU, then the server alone at 50 % and 90 % load;
  6  rectangle PSFs (5x7, 15x15, 31x31, 63x9) at 1024^2 and 2048^2, 100 iterations: the
     separable BOX_RECT kernels and the summed-area BOX_SAT kernels against the per-row
     sliding runs, px-it/s, per-launch kernel time and HBM fraction of the phase kernels;
  7  image-size sweep of the headline PSFs (oblique line 31 at 30 degrees, disc r=10) at
     512^2 .. 4096^2, 50 iterations, two-pass schedule: px-it/s, per-launch kernel time and
     HBM fraction of each phase kernel, to show how the fixed latency of a launch weighs
     at each size.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
# FP32 vector peak of MI355X: 256 CUs x 128 FP32 lanes (packed) x 2 flops (FMA) x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3
# the same without packed FP32 instructions (the library is compiled without them): 64 lanes per CU
PEAK_FP32_UNPACKED_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Algorithmic HBM bytes of one RL iteration on one pixel: u^k and f read, u^{k+1} written
# (float32 each); v and the ratio need not leave the chip.  A two-pass iteration is
# charged half of it per phase launch (BYTES_PER_PX_PHASE); halo re-reads and the ratio's
# round trip through HBM are not algorithmic.
BYTES_PER_PX_IT = 12.0
BYTES_PER_PX_PHASE = BYTES_PER_PX_IT / 2

TRAFFIC_PROFILES = {
    "batched": os.path.join(ROOT, "profiles", "batched-256_traffic.md"),
    "specialised": os.path.join(ROOT, "profiles", "phase-kernels-1024_traffic.md"),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1304_7211_amd", "csrc", n)
                  for n in ("rl_kernels.hpp", "rl_api.hip", "psf_compile.cpp", "psf_compile.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES:
        with open(fn, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name, workload="batched"):
    """HBM bytes per launch of kernel `name` (timing-registry name) from the committed
    rocprofv3 counter summary of the workload, or None if there is none or the kernel
    sources changed since the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILES[workload]).read()
    except OSError:
        return None
    a = text.find("```json")
    if a < 0:
        return None
    b = text.find("```", a + 7)
    data = json.loads(text[a + 7:b])
    if data.get("source_sha256") != kernel_source_hash():
        return None
    return data.get("bytes_per_launch", {}).get(name)


def algorithmic_flops_per_px(kind, info, phase_b):
    """Flops of the paper's algorithm for one output of one phase kernel.

    conv/corr: direct or list filter 2 per tap (multiply-add; the matrix-core kernel is
    charged the same, its split products and the zeros of its banded matrices are not
    algorithmic), generic box filter 2 per run (one add, one subtract per PSF line), 1-D box
    2 (Section 3 complexity counts); plus the ratio's division (phase A) or the update's
    multiplication (phase B)."""
    if kind == "slide":
        conv = 2.0 * info["n_spans"]
    elif kind == "rect":
        conv = 4.0  # separable 2-D box: add and subtract per pass
    elif kind == "sat":
        conv = 3.0  # summed-area table: three adds of four corners
    elif kind == "resident":
        conv = 2.0
    else:
        conv = 2.0 * info["n_taps"]
    return conv + 1.0


def job_kind(A, inf):
    """Kernel family of a job from its description (rl_job_describe)."""
    if inf["schedule"] == A.RL_SCHED_RESIDENT:
        return "resident"
    if inf["path"] == A.RL_PATH_BOX_RECT:
        return "rect"
    if inf["path"] == A.RL_PATH_BOX_SAT:
        return "sat"
    if inf["path"] == A.RL_PATH_MFMA:
        return "mfma"
    return "slide" if inf["lmax"] == 0 else ("direct" if inf["lmax"] == 1 else "span")


def kernel_work(A, jobs, infos):
    """Algorithmic bytes and flops of every timing-registry kernel over one step.

    A phase launch of a job with n pixels moves 6 B per pixel: one RL iteration moves
    12 B per pixel-iteration (u^k and f read, u^{k+1} written; the ratio needs no HBM
    round trip in principle), and the two-pass schedule splits each iteration into two
    launches, so each is charged half.  The resident solver runs all K iterations of a
    job in one launch: 12 B x n x K.  Flops: algorithmic_flops_per_px per output of
    each launch."""
    work = {}
    for j in jobs:
        inf = infos[j["name"]]
        kind = job_kind(A, inf)
        units = j["f"].size * j["iters"]
        if kind == "resident":
            names = [("resident_box", BYTES_PER_PX_IT, False)]
        else:
            names = [(f"{kind}_conv_ratio", BYTES_PER_PX_IT / 2, False),
                     (f"{kind}_corr_update", BYTES_PER_PX_IT / 2, True)]
        for nm, bpp, phase_b in names:
            w = work.setdefault(nm, dict(bytes=0.0, flops=0.0, jobs=[], px_it=0))
            w["bytes"] += bpp * units
            w["flops"] += algorithmic_flops_per_px(kind, inf, phase_b) * units
            w["px_it"] += units
            w["jobs"].append(j["name"])
    return work


def roofline_of(kernels, work, traffic_fn):
    """Roofline object of the kernel with the largest total time: the bound is the
    resource whose peak gives the longer minimum time for its algorithmic work."""
    if not kernels:
        return None
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    kinfo, w = kernels[dom], work.get(dom)
    if not w:
        return None
    t = kinfo["total_ms"] * 1e-3
    n = kinfo["launches"]
    by, fl = w["bytes"] / n, w["flops"] / n  # per launch
    dt = kinfo["avg_us"] * 1e-6
    t_alu = fl / (PEAK_FP32_TFLOPS * 1e12)
    t_hbm = by / (PEAK_HBM_GBS * 1e9)
    tr = traffic_fn(dom)
    hbm = by / dt / 1e9
    alu = fl / dt / 1e12
    if t_hbm >= t_alu:
        rf = dict(bound="hbm", achieved=round(hbm, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                  frac=round(hbm / PEAK_HBM_GBS, 5), traffic=tr)
    else:
        # the matrix-core kernel is a float32 contraction on the matrix cores (bfloat16
        # parts, float32 accumulation): its roof is the dense FP32 matrix peak, which on
        # MI355X equals the packed FP32 vector peak
        rf = dict(bound="mfma" if dom.startswith("mfma_") else "alu", achieved=round(alu, 4),
                  peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                  frac=round(alu / PEAK_FP32_TFLOPS, 5), traffic=tr)
    rf.update(kernel=dom, launches=n, avg_us=round(kinfo["avg_us"], 3),
              total_ms=round(kinfo["total_ms"], 3),
              jobs=len(w["jobs"]), bytes_per_launch=round(by), flops_per_launch=round(fl),
              hbm_frac=round(hbm / PEAK_HBM_GBS, 5),
              alu_frac=round(alu / PEAK_FP32_TFLOPS, 5),
              alu_frac_unpacked=round(alu / PEAK_FP32_UNPACKED_TFLOPS, 5),
              px_it_per_s=round(w["px_it"] / t))
    return rf


KERNEL_NAMES = ["resident_box", "mfma_conv_ratio", "mfma_corr_update", "rect_conv_ratio",
                "rect_corr_update", "sat_conv_ratio",
                "sat_corr_update", "slide_conv_ratio", "slide_corr_update", "span_conv_ratio",
                "span_corr_update", "direct_conv_ratio", "direct_corr_update"]


def read_kernel_timing(A):
    kernels = {}
    for nm in KERNEL_NAMES:
        n, ms = A.rl_timing_read(nm)
        if n:
            kernels[nm] = dict(launches=n, total_ms=ms, avg_us=1e3 * ms / n)
    return kernels


def checked_jobs(jobs, per_class=2):
    """Indices of the `per_class` cheapest jobs (pixels x iterations x taps) of each PSF
    class of the batched workload: the jobs whose full-length results the FP64 oracle
    checks."""
    cls = {}
    for i, j in enumerate(jobs):
        c = j["name"].split("-")[1]
        cost = j["f"].size * j["iters"] * np.count_nonzero(j["psf"])
        cls.setdefault(c, []).append((cost, i))
    return [i for c in sorted(cls) for _, i in sorted(cls[c])[:per_class]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["batched", "specialised"], default="batched",
                    help="batched: 256 uneven images with mixed PSFs (the default); "
                         "specialised: three 1024x1024 images with the specialised PSFs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-kahan", action="store_true",
                    help="batched workload: plain float32 sums instead of compensated ones")
    ap.add_argument("--iters", type=int, default=200, help="specialised workload: iterations")
    ap.add_argument("--mode", choices=["batch", "sequential"], default="batch")
    ap.add_argument("--compare", action="store_true",
                    help="also time the other mode (reported as 'other_mode')")
    ap.add_argument("--report", type=int, choices=[1, 3, 4, 5, 6, 7], default=None)
    ap.add_argument("--requests", type=int, default=1000, help="--report 5: requests")
    ap.add_argument("--pool-size", type=int, default=256,
                    help="--report 5: distinct requests the arrivals are drawn from")
    ap.add_argument("--sides", default="512,1024,2048,4096",
                    help="--report 7: image sides, comma-separated")
    ap.add_argument("--summary-side", type=int, default=0,
                    help="--summarize-pmc / --summarize-trace: the profiled run was "
                         "--report 7 --sides N with this N (default: the benchmark workload)")
    ap.add_argument("--summary-workload", choices=["batched", "specialised"], default="batched",
                    help="--summarize-pmc / --summarize-trace: workload of the profiled run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (the "
                         "reference dispatch for scaling HBM counters)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: turn two rocprofv3 --pmc CSV outputs (FETCH_SIZE, "
                         "WRITE_SIZE) of a run with --calibrate-copy into the traffic "
                         "summary (markdown) on stdout")
    ap.add_argument("--pmc-command", default="",
                    help="--summarize-pmc / --summarize-trace: the profiled command, quoted "
                         "in the summary")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"),
                    help="no GPU work: turn a rocprofv3 --kernel-trace --stats CSV output "
                         "and the JSON line of an unprofiled bench run into the kernel "
                         "trace summary (markdown) on stdout")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_DIR",
                    help="no GPU work: turn rocprofv3 --pmc CSV outputs of SQ counters "
                         "(SQ_WAVES among them) into per-wavefront averages per kernel "
                         "symbol (markdown) on stdout")
    args = ap.parse_args()
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.pmc_command))
        return
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1],
                            args.calibrate_copy, args.pmc_command, args.summary_side,
                            args.summary_workload))
        return
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace[0], args.summarize_trace[1],
                              args.pmc_command, args.summary_side, args.summary_workload))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the jobs are independent per GPU: N GPUs run N disjoint job sets)",
              file=sys.stderr)
        sys.exit(2)

    import synth
    jobs = None
    if args.report == 5:
        # the request pool first, in forked workers, before anything touches the GPU
        from synth.configs import make_jobs, serving_specs
        t0 = time.perf_counter()
        workers = max(1, min(16, os.cpu_count() or 1))
        args.pool = make_jobs(serving_specs(args.pool_size), workers=workers, pool="fork")
        log(f"report 5: pool of {len(args.pool)} distinct requests generated in "
            f"{time.perf_counter() - t0:.1f}s")
    if args.report is None and args.workload == "batched":
        # images first, in forked workers, before anything touches the GPU
        t0 = time.perf_counter()
        workers = max(1, min(16, os.cpu_count() or 1))
        jobs = synth.job_for_config(4, workers=workers, pool="fork")
        log(f"bench: {len(jobs)} batched jobs generated in {time.perf_counter() - t0:.1f}s "
            f"({workers} workers)")

    import torch

    from paper_1304_7211_amd import _abi as A
    from paper_1304_7211_amd.job import BatchRunner, Job

    A.lib()  # fail loudly if the HIP library is not built
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.report:
        line = {1: report_plain_small, 3: report_thinned, 4: report_batched,
                5: report_serving, 6: report_rect, 7: report_sizes}[args.report](args, dev)
        print(json.dumps(line), flush=True)
        return
    batched = args.workload == "batched"
    kahan = not args.no_kahan
    if not batched:
        jobs = synth.job_for_config(2)
        for j in jobs:
            j["iters"] = args.iters
    log(f"bench: {len(jobs)} jobs, iters {min(j['iters'] for j in jobs)}.."
        f"{max(j['iters'] for j in jobs)}, workload {args.workload}")
    f_dev = [torch.from_numpy(j["f"]).to(dev) for j in jobs]
    outs = [torch.empty_like(f) for f in f_dev]
    torch.cuda.synchronize()
    px_it_step = sum(j["f"].size * j["iters"] for j in jobs)

    infos = {}
    runner = BatchRunner(len(jobs))

    def new_job(j, f):
        return Job(f, j["psf"], path=j["path"], kahan=kahan)

    def step_sequential():
        for j, f, o in zip(jobs, f_dev, outs):
            job = new_job(j, f)
            job.iterate(j["iters"])
            job.result(out=o)
            infos[j["name"]] = job.describe()
            job.close()

    def step_batch():
        js = [new_job(j, f) for j, f in zip(jobs, f_dev)]
        runner.iterate(js, [j["iters"] for j in jobs])
        for j, jb, o in zip(jobs, js, outs):
            jb.result(out=o)
            infos[j["name"]] = jb.describe()
            jb.close()

    step = step_batch if args.mode == "batch" else step_sequential

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"bench: warmup {w + 1}/{args.warmup} done")

    # timed region (no instrumentation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = px_it_step * args.steps / elapsed
    log(f"bench: {args.steps} steps in {elapsed:.4f}s -> {value:.4g} px-it/s ({args.mode})")
    # the outputs of the last timed step, for the accuracy check against the FP64 oracle
    picked = checked_jobs(jobs) if batched else list(range(len(jobs)))
    timed_out = {i: outs[i].cpu().numpy() for i in picked}
    other = None
    if args.compare:
        ostep = step_sequential if args.mode == "batch" else step_batch
        ostep()
        torch.cuda.synchronize()
        o0 = time.perf_counter()
        for _ in range(args.steps):
            ostep()
        torch.cuda.synchronize()
        o1 = time.perf_counter()
        other = dict(mode="sequential" if args.mode == "batch" else "batch",
                     value=px_it_step * args.steps / (o1 - o0),
                     ms_per_step=1e3 * (o1 - o0) / args.steps)
        log(f"bench: other mode {other}")

    # per-kernel durations: one more step with every launch carrying HIP events in its
    # dispatch packet, on the stream it is launched on (the events add a little time per
    # launch, so the headline value above comes from the uninstrumented run)
    roofline = None
    kernels = {}
    if not args.no_kernel_timing:
        A.rl_timing_reset()
        A.rl_timing_enable(True)
        torch.cuda.synchronize()
        step()
        torch.cuda.synchronize()
        A.rl_timing_enable(False)
        kernels = read_kernel_timing(A)
        A.rl_timing_reset()
        work = kernel_work(A, jobs, infos)
        for nm, k in kernels.items():
            w = work.get(nm)
            if w:
                dt = k["total_ms"] * 1e-3
                k.update(hbm_frac=round(w["bytes"] / dt / 1e9 / PEAK_HBM_GBS, 5),
                         alu_frac=round(w["flops"] / dt / 1e12 / PEAK_FP32_TFLOPS, 5),
                         jobs=len(w["jobs"]))
        roofline = roofline_of(kernels, work,
                               lambda nm: measured_traffic(nm, args.workload))
    log(f"bench: kernels {json.dumps(kernels)}")

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        cpu, accuracy = cpu_baseline(jobs, picked, timed_out, full_length=batched)

    if batched:
        cls = {}
        for j in jobs:
            c = j["name"].split("-")[1]
            cls[c] = cls.get(c, 0) + 1
        config = {"workload": "batched: 256 images, sides log-uniform 256..2048 (seeded, "
                              "non-square), PSFs uniform over {axis box 5-63, oblique line "
                              "9-47 at a uniform angle, disc r 3-24, dense 15x15}, 100-300 "
                              "iterations, Poisson peak 255, one rl_iterate_batch call",
                  "jobs": len(jobs), "psf_classes": cls, "kahan": kahan,
                  "mode": args.mode, "px_it_per_step": px_it_step}
        data = "synthetic (seeded generator: shapes + sinusoid, reflect blur, Poisson noise)"
    else:
        config = {"workload": "specialised PSFs 1024x1024 x3 (vertical box 41, oblique "
                              f"31@30deg AA, disc r10), {args.iters} iterations each",
                  "mode": args.mode, "px_it_per_step": px_it_step}
        data = "synthetic (seeded generator: shapes + sinusoid, reflect blur, Gaussian noise)"
    paths = {}
    for v in infos.values():
        key = f"{A.PATH_NAMES[v['path']]}/{A.SCHED_NAMES[v['schedule']]}"
        paths[key] = paths.get(key, 0) + 1
    config["paths"] = paths
    line = {
        "metric": "RL pixel-iterations/s at <=1e-5 rel err vs FP64",
        "value": value,
        "unit": "px-it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": data,
        "config": config,
        "roofline": roofline,
        # the whole step's pixel-iterations at the algorithmic 12 B each, against HBM
        "method_hbm_frac": round(value * BYTES_PER_PX_IT / (PEAK_HBM_GBS * 1e9), 5),
        "accuracy": accuracy,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "other_mode": other,
    }
    print(json.dumps(line), flush=True)


def _psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def report_plain_small(args, dev):
    import torch

    import oracle
    import synth
    from paper_1304_7211_amd.job import Job
    job = synth.job_for_config(1)[0]
    f = torch.from_numpy(job["f"]).to(dev)
    K = job["iters"]
    ref = oracle.Oracle().rl(job["f"], job["psf"], K)
    out = {}
    for path, sched in (("auto", "auto"), ("box_axis", "two_pass"), ("runs", "auto"),
                        ("direct", "auto")):
        times = []
        for rep in range(20):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            j = Job(f, job["psf"], path=path, schedule=sched)
            j.iterate(K)
            u = j.result()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            info = j.describe()
            j.close()
        err = float(np.max(np.abs(u.cpu().numpy() - ref) / np.maximum(np.abs(ref), 1e-4)))
        out[f"{path}/{sched}"] = dict(us_per_solve=round(1e6 * float(np.median(times[5:])), 1),
                                      schedule=info["schedule"], max_rel_err=err)
        log(f"report 1: {path}/{sched}: {out[f'{path}/{sched}']}")
    return {"report": "plain RL, config 1", "workload": "128x128, box 1x15, Poisson 255, 50 "
            "iterations (median of 15 solves after 5 warm-ups, init to result)", "paths": out}


def report_thinned(args, dev):
    import torch

    import synth
    from paper_1304_7211_amd.job import Job
    job = synth.job_for_config(3)[0]
    f = torch.from_numpy(job["f"]).to(dev)
    K = job["iters"]
    N = job["f"].size
    log(f"report 3: {job['f'].shape} disc r=16, K={K}, thin={job['thin']}")

    def run(thin):
        j = Job(f, job["psf"], thin=thin)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        j.iterate(K)
        u, st = j.result(stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sched = j.thin_schedule() if thin else None
        j.close()
        return dict(u=u.cpu().numpy(), t=dt, st=st, sched=sched)

    run(None)  # warm-up
    plain = run(None)
    log(f"report 3: plain {plain['t'] * 1e3:.1f} ms")
    # Section 4's per-pixel rule and the block rule (freeze decisions per block), at
    # configuration 3's threshold and over a threshold sweep as in Table 2
    rules = (("pixel", 0), ("block64", 64), ("block16", 16))
    res = {}
    for tau in (1e-4, 3e-4, 1e-3, 3e-3, 1e-2):
        for rule, B in rules:
            out = run(dict(job["thin"], tau=tau, block=B))
            sc = np.array(out["sched"], dtype=np.float64) / N
            psnr = _psnr(out["u"], plain["u"])
            res[(rule, tau)] = dict(
                rule=rule, tau=tau, ms=round(out["t"] * 1e3, 2),
                speedup=round(plain["t"] / out["t"], 3),
                omitted_fraction=round(float(1.0 - sc.mean()), 4),
                # None: bit-identical to the unthinned run (nothing froze)
                psnr_vs_plain_db=None if np.isinf(psnr) else round(psnr, 2),
                flux=out["st"].flux)
            if tau == 1e-4:
                res[(rule, tau)]["active_fraction_at_k_5_15_25"] = [
                    round(float(x), 4) for x in sc[5:30:10]]
            log(f"report 3: {res[(rule, tau)]}")
    main = res[("pixel", 1e-4)]
    return {
        "report": "thinned RL, config 3",
        "workload": "2048x2048, disc r=16, Poisson peak 1000, 500 iterations, rel tau 1e-4, H=5, R=10, C=10",
        "plain_ms": plain["t"] * 1e3,
        "px_it_per_s_plain": N * K / plain["t"],
        "thinned_ms": main["ms"],
        "speedup": main["speedup"],
        "omitted_fraction": main["omitted_fraction"],
        "psnr_thinned_vs_plain_db": main["psnr_vs_plain_db"],
        "block64_ms": res[("block64", 1e-4)]["ms"],
        "block64_speedup": res[("block64", 1e-4)]["speedup"],
        "flux_plain": plain["st"].flux,
        "rules_and_taus": [res[k] for k in sorted(res, key=lambda k: (k[1], k[0]))],
    }


def report_batched(args, dev):
    import torch

    import oracle
    import synth
    from paper_1304_7211_amd.job import BatchRunner, Job
    t0 = time.perf_counter()
    jobs = synth.job_for_config(4, workers=max(1, min(16, os.cpu_count() or 1)))
    log(f"report 4: {len(jobs)} jobs generated in {time.perf_counter() - t0:.1f}s")
    fs = [torch.from_numpy(j["f"]).to(dev) for j in jobs]
    px_it = sum(j["f"].size * j["iters"] for j in jobs)
    runner = BatchRunner(len(jobs))
    out = {}
    for kahan in (True, False):
        js = [Job(f, j["psf"], kahan=kahan) for j, f in zip(jobs, fs)]
        runner.iterate(js, [2] * len(js))  # warm the kernels
        torch.cuda.synchronize()
        for jb in js:
            jb.close()
        js = [Job(f, j["psf"], kahan=kahan) for j, f in zip(jobs, fs)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        runner.iterate(js, [j["iters"] for j in jobs])
        us = [jb.result() for jb in js]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        out[kahan] = dict(t=dt, u=us, paths=[jb.describe()["path"] for jb in js])
        for jb in js:
            jb.close()
        log(f"report 4: kahan={kahan} {dt * 1e3:.1f} ms, {px_it / dt:.3g} px-it/s")
    # FP64 oracle on the two cheapest jobs of each PSF class
    picked = checked_jobs(jobs)
    o = oracle.Oracle()
    errs = []
    for i in picked:
        j = jobs[i]
        ref = o.rl(j["f"], j["psf"], j["iters"])
        e = {}
        for kahan in (True, False):
            u = out[kahan]["u"][i].cpu().numpy().astype(np.float64)
            e["compensated" if kahan else "plain"] = float(
                np.max(np.abs(u - ref) / np.maximum(np.abs(ref), 1e-4)))
        errs.append(dict(job=j["name"], shape=list(j["f"].shape), iters=j["iters"], **e))
        log(f"report 4: {errs[-1]}")
    # one lock-step iteration on every job: from the GPU's float32 state u^K, one more GPU
    # iteration in one batch call against one FP64 oracle iteration from the same state
    t2 = time.perf_counter()
    js = [Job(f, j["psf"], u0=out[True]["u"][i]) for i, (j, f) in enumerate(zip(jobs, fs))]
    runner.iterate(js, [1] * len(js))
    lock = []
    for i, (j, jb) in enumerate(zip(jobs, js)):
        u1 = jb.result().cpu().numpy().astype(np.float64)
        ref = o.rl(j["f"], j["psf"], 1, u0=out[True]["u"][i].cpu().numpy())
        lock.append(float(np.max(np.abs(u1 - ref) / np.maximum(np.abs(ref), 1e-4))))
        jb.close()
        if (i + 1) % 32 == 0:
            log(f"report 4: lock-step {i + 1}/{len(jobs)} jobs checked")
    worst = int(np.argmax(lock))
    log(f"report 4: lock-step iteration on {len(lock)} jobs in {time.perf_counter() - t2:.1f}s, "
        f"max rel err {lock[worst]:.3g} ({jobs[worst]['name']})")
    return {
        "report": "batched uneven jobs, config 4",
        "workload": "256 images, sides log-uniform 256..2048, PSFs axis/oblique/disc/dense15, "
                    "100..300 iterations, Poisson 255, one rl_iterate_batch call",
        "px_it": px_it,
        "compensated": {"ms": out[True]["t"] * 1e3, "px_it_per_s": px_it / out[True]["t"]},
        "plain_sums": {"ms": out[False]["t"] * 1e3, "px_it_per_s": px_it / out[False]["t"]},
        "max_rel_err_vs_fp64": {
            "compensated": max(e["compensated"] for e in errs),
            "plain": max(e["plain"] for e in errs)},
        "checked_jobs": errs,
        "lockstep_all_jobs": {"jobs": len(lock), "max_rel_err": max(lock),
                              "worst_job": jobs[worst]["name"]},
    }


def report_serving(args, dev):
    import torch

    import synth
    from paper_1304_7211_amd.serve import (Request, Server, latency_report, run_stream,
                                           serve_plain)
    c = synth.CONFIGS[5]
    rng = np.random.default_rng(c["seed"] + 1)
    thin = dict(synth.CONFIGS[3]["thin"])
    pool = [(j["f"], j["psf"], j["iters"]) for j in args.pool]
    pool_dev = [(torch.from_numpy(f).to(dev), h, K) for f, h, K in pool]
    budget = int(0.5 * torch.cuda.mem_get_info(dev)[0])
    # every arrival draws its request from the pool (uniformly, seeded); the first
    # len(pool) arrivals cover the pool in a shuffled order
    order = np.concatenate([rng.permutation(len(pool)),
                            rng.integers(0, len(pool), size=max(0, args.requests - len(pool)))])

    def make(n, arrivals):
        return [Request(i, pool_dev[order[i % len(order)]][0], pool_dev[order[i % len(order)]][1],
                        pool_dev[order[i % len(order)]][2], thin=thin, arrival=float(a))
                for i, a in enumerate(arrivals)]

    # capacity: the whole pool submitted at once
    warm = Server(budget, max_slots=64, chunk=10)
    run_stream(make(min(32, len(pool)), [0.0] * min(32, len(pool))), warm)
    srv = Server(budget, max_slots=64, chunk=10)
    reqs = make(len(pool), [0.0] * len(pool))
    dt = run_stream(reqs, srv)
    capacity = len(pool) / dt
    px_it_pool = sum(f.size * K for f, _, K in pool)
    log(f"report 5: batched capacity {capacity:.1f} req/s ({px_it_pool / dt:.3g} px-it/s)")
    qps = 0.7 * capacity
    n = args.requests
    arrivals = np.cumsum(rng.exponential(1.0 / qps, size=n))
    reqs = make(n, arrivals)
    srv = Server(budget, max_slots=64, chunk=10)
    dt_c = run_stream(reqs, srv)
    rep_c = latency_report(reqs)
    base = make(n, arrivals)
    dt_p = serve_plain(base)
    rep_p = latency_report(base)
    same = all(torch.equal(a.result, b.result) for a, b in zip(reqs, base))
    px_it = sum(pool[order[i % len(order)]][0].size * pool[order[i % len(order)]][2]
                for i in range(n))
    log(f"report 5: continuous {rep_c}, plain {rep_p}, identical={same}")
    del base
    # load sweep of the continuous-batching server (same request mix, other arrival rates)
    sweep = []
    for frac in (0.5, 0.9):
        arr = np.cumsum(rng.exponential(1.0 / (frac * capacity), size=n))
        rs = make(n, arr)
        sv = Server(budget, max_slots=64, chunk=10)
        dt_s = run_stream(rs, sv)
        sweep.append(dict(load=frac, qps=frac * capacity, latency=latency_report(rs),
                          px_it_per_s=px_it / dt_s))
        log(f"report 5: load {frac}: {sweep[-1]['latency']}")
        del rs
    return {
        "report": "serving, config 5",
        "workload": f"{n} requests, each drawn from {len(pool)} distinct seeded requests "
                    "(sides 128..4096, mixed PSFs, 50..500 iterations, thinning rel 1e-4 H5 "
                    "R10 C10), Poisson arrivals",
        "qps": qps,
        "batched_capacity_req_per_s": capacity,
        "continuous": dict(latency=rep_c, wall_s=dt_c, px_it_per_s=px_it / dt_c,
                           peak_slots=srv.ctl.peak_slots),
        "plain_per_image": dict(latency=rep_p, wall_s=dt_p, px_it_per_s=px_it / dt_p),
        "results_identical": bool(same),
        "load_sweep": sweep,
    }


def _timing_name(kernel):
    """Map a rocprofv3 kernel symbol to the library's timing-registry name."""
    import re
    m = re.search(r"rlk::(slide|span|resident|resident_multi|rect|sat|mixed|mfma)_kernel<([^>]*)>",
                  kernel)
    if not m:
        return None
    kind, targs = m.group(1), [t.strip() for t in m.group(2).split(",")]
    if kind in ("resident", "resident_multi"):
        return "resident_box"
    phase_b = targs[-1] == "true"
    if kind == "span" and targs[2] == "1":
        kind = "direct"
    return f"{kind}_{'corr_update' if phase_b else 'conv_ratio'}"


def _registry_totals(rows):
    """Sum (calls, total ns) per timing-registry name over the kernel symbols of a
    rocprofv3 kernel-statistics table (several template instances share one name)."""
    agg = {}
    for r in rows:
        nm = _timing_name(r["Name"])
        if not nm:
            continue
        a = agg.setdefault(nm, [0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
    return agg


def _last_dispatch_averages(trace_dir, kernels):
    """Average rocprofv3 duration (us) of the last n dispatches of each registry name,
    n = the launch count bench.py reports for it, from the per-dispatch kernel trace."""
    import csv
    import glob
    fns = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not fns or not kernels:
        return {}
    per = {}
    for r in csv.DictReader(open(fns[0])):
        nm = _timing_name(r["Kernel_Name"])
        if nm:
            per.setdefault(nm, []).append((int(r["Start_Timestamp"]),
                                           int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = {}
    for nm, k in kernels.items():
        d = sorted(per.get(nm, []))
        n = int(k["launches"])
        if len(d) >= n > 0:
            out[nm] = (n, sum(x[1] for x in d[-n:]) / n / 1e3)
    return out


def summarize_trace(trace_dir, bench_log, command, side=0, workload="batched"):
    """Per-kernel durations from rocprofv3's kernel statistics, next to bench.py's own
    dispatch-event durations of an unprofiled run of the same workload (the benchmark, or
    with side > 0 the size sweep of --report 7 at that side)."""
    import csv
    import glob
    fn = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(fn)))
    line = [ln for ln in open(bench_log).read().splitlines() if ln.startswith("{")][-1]
    bench = json.loads(line)
    if side:
        title = (f"# Kernel trace: phase kernels at {side}x{side} (oblique line 31 at 30 deg "
                 f"and disc r=10, two-pass, bench.py --report 7 --sides {side})")
        note = ("The run covers the report's warmup, timed and instrumented iterations of "
                "both PSFs.")
    elif workload == "batched":
        title = ("# Kernel trace: bench.py default workload (batched: 256 uneven images, "
                 "mixed PSFs, 100-300 iterations, one rl_iterate_batch call per step)")
        note = ("The run covers bench.py's warmup step, its timed steps and its instrumented "
                "step. rocprofv3 lengthens the uninstrumented timing, so the headline value "
                "comes from runs without the profiler.")
    else:
        title = ("# Kernel trace: bench.py --workload specialised (3 x 1024x1024, "
                 "200 iterations, batch mode)")
        note = ("The run covers bench.py's warmup step, its timed steps and its instrumented "
                "step. rocprofv3 lengthens the uninstrumented timing, so the headline value "
                "comes from runs without the profiler.")
    out = [title, "", "Command:", "", "```", command.strip(), "```", "", note, "",
           "| Kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    agg = _registry_totals(rows)
    if agg:
        out += ["", "The same, summed per timing-registry name (the names bench.py reports):",
                "", "| Registry name | calls | total ms | avg us |", "|---|---|---|---|"]
        for nm in sorted(agg, key=lambda k: -agg[k][1]):
            c, ns = agg[nm]
            out.append(f"| `{nm}` | {c} | {ns / 1e6:.2f} | {ns / c / 1e3:.2f} |")
    out += ["", f"bench.py's own per-kernel durations (dispatch-attached HIP events) from the "
            f"JSON line in `{os.path.basename(bench_log)}`:", ""]
    if side:
        for row in bench.get("rows", []):
            for k, v in row["kernels"].items():
                out.append(f"- {row['psf']} `{k}`: {v['us']:.2f} us per launch, "
                           f"HBM fraction {v['hbm_frac']}")
        return "\n".join(out)
    for k, v in bench.get("kernels", {}).items():
        out.append(f"- `{k}`: {v['avg_us']:.2f} us over {v['launches']} launches")
    last = _last_dispatch_averages(trace_dir, bench.get("kernels", {}))
    if last:
        out += ["", "rocprofv3's durations of the same dispatches bench.py timed with its "
                "events (the last `launches` dispatches of each name, i.e. bench.py's "
                "instrumented step):", "",
                "| Registry name | dispatches | rocprofv3 avg us | bench.py avg us | ratio |",
                "|---|---|---|---|---|"]
        for k, (n, us) in last.items():
            b = bench["kernels"][k]["avg_us"]
            out.append(f"| `{k}` | {n} | {us:.2f} | {b:.2f} | {us / b:.3f} |")
    rf = bench.get("roofline") or {}
    out += ["", f"Headline of that run: {bench['value']:.4g} {bench['unit']}, "
            f"{bench['ms_per_step']:.3f} ms per step; roofline of `{rf.get('kernel')}`: "
            f"{rf.get('achieved')} {rf.get('unit')} = {rf.get('frac')} of {rf.get('peak')} "
            f"(bound {rf.get('bound')})."]
    return "\n".join(out)


def summarize_counters(dirs, command, min_waves=1000):
    """Per kernel symbol, each counter's per-dispatch total (summed over the dispatch's
    shader engines) divided by the dispatch's wavefronts (SQ_WAVES), averaged over
    dispatches; SQ_WAVES itself per dispatch.  Kernels with fewer than min_waves
    wavefronts per dispatch are left out."""
    import csv
    import glob
    import re
    tot, disp = {}, {}
    for d in dirs:
        fn = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        for r in csv.DictReader(open(fn)):
            k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
            c = r["Counter_Name"]
            tot.setdefault(k, {}).setdefault(c, 0.0)
            tot[k][c] += float(r["Counter_Value"])
            disp.setdefault(k, {}).setdefault(c, set()).add(r["Dispatch_Id"])
    order = ["SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM",
             "SQ_ACTIVE_INST_VALU", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_WAIT_INST_LDS",
             "SQ_WAIT_INST_ANY", "SQ_LDS_BANK_CONFLICT", "SQ_WAVE_CYCLES"]
    present = {c for k in tot for c in tot[k]}
    counters = [c for c in order if c in present] + sorted(present - set(order) - {"SQ_WAVES"})
    lines = ["# Instruction mix per wavefront: kernels of the batched workload", "",
             "Commands (one pass per counter group; rocprofv3 does not split counters over "
             "passes):", "", "```", command, "```", "",
             "Per kernel symbol: SQ_WAVES per dispatch, and every other counter's total over a "
             "dispatch divided by that dispatch's wavefronts (averaged over dispatches).  "
             "`SQ_INSTS_*` count instructions; `SQ_WAIT_INST_*`, `SQ_LDS_BANK_CONFLICT` and "
             "`SQ_VALU_MFMA_BUSY_CYCLES` count cycles.", "",
             "| Kernel | dispatches | waves | " + " | ".join(counters) + " |",
             "|---|---|---|" + "---|" * len(counters)]
    rows = []
    for k, cs in tot.items():
        if "SQ_WAVES" not in cs:
            continue
        nd = len(disp[k]["SQ_WAVES"])
        waves = cs["SQ_WAVES"] / nd
        if waves < min_waves:
            continue
        vals = []
        for c in counters:
            if c in cs:
                vals.append(f"{cs[c] / len(disp[k][c]) / waves:.0f}")
            else:
                vals.append("")
        rows.append((-(cs.get("SQ_WAVES", 0.0)), f"| `{k}` | {nd} | {waves:.0f} | " + " | ".join(vals) + " |"))
    lines += [r for _, r in sorted(rows)]
    return "\n".join(lines)


def summarize_pmc(fetch_dir, write_dir, copy_mib, command, side=0, workload="batched"):
    """Per-kernel HBM traffic (KiB per dispatch, averaged) from two rocprofv3 --pmc runs,
    scaled by the ratio of the known size of the calibration copy to what the same
    counter reads for it.  Dispatches of kernel symbols that share a timing-registry name
    are pooled: bytes_per_launch is their scaled total over their count."""
    import csv
    import glob

    def read(d, counter):
        fn = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        per = {}
        for r in csv.DictReader(open(fn)):
            if r["Counter_Name"] != counter:
                continue
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return per

    fetch = read(fetch_dir, "FETCH_SIZE")
    write = read(write_dir, "WRITE_SIZE")
    known = copy_mib * 1024.0  # KiB read and written by the calibration copy
    # the calibration copy is the non-library dispatch that reads the most
    others = [k for k in fetch if "rlk::" not in k and k in write]
    cal = max(others, key=lambda k: max(fetch[k]))
    f_cal, w_cal = max(fetch[cal]), max(write[cal])
    sf, sw = known / f_cal, known / w_cal
    rows, pooled = [], {}
    for k in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(k, [0.0]), write.get(k, [0.0])
        fa, wa = sum(fv) / len(fv), sum(wv) / len(wv)
        name = _timing_name(k)
        rows.append((k, len(fv), fa, wa, name))
        if name:
            p = pooled.setdefault(name, [0, 0.0])
            p[0] += len(fv)
            p[1] += (sum(fv) * sf + sum(wv) * sw) * 1024.0
    per_launch = {nm: round(tot / n) for nm, (n, tot) in pooled.items()}
    src_hash = kernel_source_hash()
    if side:
        title = (f"# HBM traffic counters: phase kernels at {side}x{side} (oblique line 31 at "
                 f"30 deg and disc r=10, two-pass, bench.py --report 7 --sides {side})")
    elif workload == "batched":
        title = ("# HBM traffic counters: kernels of the batched workload (256 uneven images, "
                 "mixed PSFs, one rl_iterate_batch call)")
    else:
        title = ("# HBM traffic counters: phase kernels of the specialised-PSF workload "
                 "(3 x 1024x1024, batch mode)")
    out = [title, "",
           "Commands (one counter per run; rocprofv3 does not split counters over passes):", "",
           "```", command.strip(), "```", "",
           f"Values are KiB per dispatch, averaged over dispatches.  Calibration: a plain "
           f"device-to-device copy of {copy_mib} MiB (`{cal[:60]}`) reads FETCH_SIZE "
           f"{f_cal:.1f} KiB and WRITE_SIZE {w_cal:.1f} KiB for {known:.0f} KiB moved each "
           f"way: scale factors fetch {sf:.4f}, write {sw:.4f}.", "",
           "| Kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled total MiB | registry name |",
           "|---|---|---|---|---|---|"]
    for k, n, fa, wa, name in rows:
        out.append(f"| `{k[:90]}` | {n} | {fa:.1f} | {wa:.1f} | "
                   f"{(fa * sf + wa * sw) / 1024:.2f} | {name or ''} |")
    if side:
        n_side = side
        out += ["", f"Algorithmic traffic of one phase launch at {n_side} x {n_side}: "
                f"{BYTES_PER_PX_PHASE:g} B per pixel (half of the {BYTES_PER_PX_IT:g} B of "
                f"one iteration: u^k and f read, u^(k+1) written) = "
                f"{BYTES_PER_PX_PHASE * n_side * n_side / 2 ** 20:.1f} MiB."]
    else:
        out += ["", f"Algorithmic traffic: {BYTES_PER_PX_PHASE:g} B per output pixel of a "
                f"phase launch (half of the {BYTES_PER_PX_IT:g} B of one RL iteration)."]
    out += ["", "Machine-readable (bench.py reports `bytes_per_launch` as roofline.traffic while "
            "the kernel sources hash to `source_sha256`):", "", "```json",
            json.dumps(dict(source_sha256=src_hash, scale=dict(fetch=sf, write=sw),
                            bytes_per_launch=per_launch), indent=1), "```"]
    return "\n".join(out)


def report_rect(args, dev):
    import torch

    import synth
    from paper_1304_7211_amd import _abi as A
    from paper_1304_7211_amd.job import Job
    K = 100
    rows = []
    for my, mx in ((5, 7), (15, 15), (31, 31), (63, 9)):
        h = synth.box_rect(my, mx)
        for side in (1024, 2048):
            f = torch.from_numpy(synth.observe(synth.latent_image(side, side, 6), h,
                                               "gaussian", 6)).to(dev)
            row = dict(psf=f"{my}x{mx}", side=side)
            for path in ("runs", "box_rect", "box_sat"):
                j = Job(f, h, path=path)
                j.iterate(3)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                j.iterate(K)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                A.rl_timing_reset()
                A.rl_timing_enable(True)
                j.iterate(10)
                torch.cuda.synchronize()
                A.rl_timing_enable(False)
                us = []
                for nm in ("rect_conv_ratio", "rect_corr_update", "sat_conv_ratio",
                           "sat_corr_update", "slide_conv_ratio", "slide_corr_update",
                           "span_conv_ratio", "span_corr_update"):
                    n, ms = A.rl_timing_read(nm)
                    if n:
                        us.append(1e3 * ms / n)
                A.rl_timing_reset()
                j.close()
                avg = sum(us) / len(us)
                row[path] = dict(px_it_per_s=side * side * K / dt, us_per_it=1e6 * dt / K,
                                 kernel_us=round(avg, 2),
                                 hbm_frac=round(BYTES_PER_PX_PHASE * side * side / (avg * 1e-6)
                                                / (PEAK_HBM_GBS * 1e9), 4))
            row["speedup"] = round(row["runs"]["us_per_it"] / row["box_rect"]["us_per_it"], 3)
            row["speedup_sat"] = round(row["runs"]["us_per_it"] / row["box_sat"]["us_per_it"], 3)
            rows.append(row)
            log(f"report 6: {row}")
    return {"report": "rectangle PSFs: separable BOX_RECT and summed-area BOX_SAT vs sliding runs",
            "iterations": K, "rows": rows}


def report_sizes(args, dev):
    import torch

    import synth
    from paper_1304_7211_amd import _abi as A
    from paper_1304_7211_amd.job import Job
    K = 50
    rows = []
    for name, h in (("oblique-31-at-30deg", synth.oblique_line(31, 30.0)),
                    ("disc-r10", synth.disc(10))):
        for side in [int(x) for x in args.sides.split(",")]:
            f = torch.from_numpy(synth.observe(synth.latent_image(side, side, 7), h,
                                               "gaussian", 7)).to(dev)
            j = Job(f, h, path="runs")
            j.iterate(3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            j.iterate(K)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            A.rl_timing_reset()
            A.rl_timing_enable(True)
            j.iterate(10)
            torch.cuda.synchronize()
            A.rl_timing_enable(False)
            kernels = {}
            for nm in ("slide_conv_ratio", "slide_corr_update", "span_conv_ratio",
                       "span_corr_update"):
                n, ms = A.rl_timing_read(nm)
                if n:
                    us = 1e3 * ms / n
                    kernels[nm] = dict(us=round(us, 2), hbm_frac=round(
                        BYTES_PER_PX_PHASE * side * side / (us * 1e-6) / (PEAK_HBM_GBS * 1e9), 4))
            A.rl_timing_reset()
            strip = j.describe()["strip"]
            j.close()
            del f
            row = dict(psf=name, side=side, strip=strip, px_it_per_s=side * side * K / dt,
                       us_per_it=round(1e6 * dt / K, 2), kernels=kernels)
            rows.append(row)
            log(f"report 7: {row}")
    return {"report": "image-size sweep of the phase kernels (two-pass schedule)",
            "iterations": K, "bytes_per_px_per_phase": BYTES_PER_PX_PHASE,
            "peak_hbm_gbs": PEAK_HBM_GBS, "rows": rows}


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_err_stats(got, ref, floor=1e-4):
    """max and 99.9th percentile of |got - ref| / max(|ref|, floor) over the pixels."""
    e = np.abs(np.asarray(got, np.float64) - ref) / np.maximum(np.abs(ref), floor)
    return float(e.max()), float(np.quantile(e, 0.999))


def cpu_baseline(jobs, picked, timed_out, full_length=True):
    """The FP64 oracle on the host cores: the full-length runs of the checked jobs, timed
    (all threads), each compared with the GPU output of the last timed step; then a
    single-thread rate on a bounded sample of the cheapest checked job."""
    import oracle
    o = oracle.Oracle()
    cores = o.threads()
    total_px_it = 0
    errs = []
    t0 = time.perf_counter()
    for i in picked:
        j = jobs[i]
        ref = o.rl(j["f"], j["psf"], j["iters"])
        total_px_it += j["f"].size * j["iters"]
        mx, p999 = rel_err_stats(timed_out[i], ref)
        errs.append(dict(job=j["name"], shape=list(j["f"].shape), iters=j["iters"],
                         taps=int(np.count_nonzero(j["psf"])), max_rel_err=mx,
                         p999_rel_err=p999))
        log(f"bench: oracle {errs[-1]}")
    dt = time.perf_counter() - t0
    log(f"bench: cpu oracle {total_px_it} px-it in {dt:.2f}s on {cores} threads")
    # single thread: the cheapest checked job, iterations sized to about 3 s
    j1 = jobs[min(picked, key=lambda i: jobs[i]["f"].size * np.count_nonzero(jobs[i]["psf"]))]
    o.set_threads(1)
    try:
        p0 = time.perf_counter()
        o.rl(j1["f"], j1["psf"], 1)
        one = max(time.perf_counter() - p0, 1e-4)
        k1 = max(1, min(j1["iters"], int(3.0 / one)))
        p0 = time.perf_counter()
        o.rl(j1["f"], j1["psf"], k1)
        dt1 = time.perf_counter() - p0
    finally:
        o.set_threads(cores)
    single = j1["f"].size * k1 / dt1
    log(f"bench: cpu oracle single thread {single:.4g} px-it/s ({j1['name']} x{k1} it)")
    cpu = dict(value=total_px_it / dt, unit="px-it/s", cores=cores, kind="oracle",
               sample=f"full-length FP64 oracle runs of {len(picked)} jobs of the workload "
                      f"({', '.join(e['job'] for e in errs)}; {total_px_it:.3g} px-it in "
                      f"{dt:.1f}s)",
               single_core=dict(value=single, unit="px-it/s",
                                sample=f"{j1['name']} {j1['f'].shape[0]}x{j1['f'].shape[1]}, "
                                       f"{k1} iterations in {dt1:.1f}s"),
               cpu_model=cpu_model())
    worst = max(errs, key=lambda e: e["max_rel_err"])
    accuracy = dict(metric="max over pixels of |gpu - fp64| / max(|fp64|, 1e-4)",
                    checked_jobs=len(errs), max_rel_err=worst["max_rel_err"],
                    worst_job=worst["job"], gate=1e-5,
                    within_gate=bool(worst["max_rel_err"] <= 1e-5), per_job=errs)
    return cpu, accuracy


if __name__ == "__main__":
    main()
