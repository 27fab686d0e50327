"""Benchmark: Richardson-Lucy pixel-iterations per second on one MI355X.

Workload (one "step"): the specialised-PSF configuration -- three 1024 x 1024 float32
images from the seeded generator, Gaussian noise sigma 0.01, 200 RL iterations each:
  (a) vertical motion blur, box of length 41      -> BOX_AXIS path
  (b) oblique motion line, length 31 at 30 deg, antialiased -> RUNS path (row spans)
  (c) uniform disc of radius 10                   -> RUNS path (sliding runs)
A step runs all three jobs end to end through the C ABI: rl_init for each (copy f into
the workspace, upload the compiled PSF), one rl_iterate_batch call that advances all
three by 200 iterations (independent kernel groups on concurrent streams), and rl_result
for each (copy u^K out).  Inputs are resident on the GPU before the timed region starts.
--mode sequential runs rl_iterate per job instead (the plain per-image method).

Prints ONE JSON line.  Options: --gpus (must be 1), --steps, --warmup, --no-cpu-baseline,
--no-kernel-timing.
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_flops_per_px(kind, info, phase_b):
    """Flops of the paper's algorithm for one output of one phase kernel.

    conv/corr: direct or list filter 2 per tap (multiply-add), generic box filter 2 per
    run (one add, one subtract per PSF line), 1-D box 2 (Section 3 complexity counts);
    plus the ratio's division (phase A) or the update's multiplication (phase B)."""
    if kind == "slide":
        conv = 2.0 * info["n_spans"]
    elif kind == "resident":
        conv = 2.0
    else:
        conv = 2.0 * info["n_taps"]
    return conv + 1.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--mode", choices=["batch", "sequential"], default="batch")
    ap.add_argument("--compare", action="store_true",
                    help="also time the other mode (reported as 'other_mode')")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the jobs are independent per GPU: N GPUs run N disjoint job sets)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1304_7211_amd import _abi as A
    from paper_1304_7211_amd.job import BatchRunner, Job

    A.lib()  # fail loudly if the HIP library is not built
    dev = torch.device("cuda:0")
    jobs = synth.job_for_config(2)
    for j in jobs:
        j["iters"] = args.iters
    log(f"bench: {len(jobs)} jobs, {[j['name'] for j in jobs]}, iters={args.iters}")
    f_dev = [torch.from_numpy(j["f"]).to(dev) for j in jobs]
    outs = [torch.empty_like(f) for f in f_dev]
    torch.cuda.synchronize()
    px_it_step = sum(j["f"].size * j["iters"] for j in jobs)

    infos = {}
    runner = BatchRunner(len(jobs))

    def step_sequential():
        for j, f, o in zip(jobs, f_dev, outs):
            job = Job(f, j["psf"], path=j["path"])
            job.iterate(j["iters"])
            job.result(out=o)
            infos[j["name"]] = job.describe()
            job.close()

    def step_batch():
        js = [Job(f, j["psf"], path=j["path"]) for j, f in zip(jobs, f_dev)]
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

    # per-kernel durations: the same steps again with every launch bracketed by HIP events
    # on the stream it is launched on (events add a few microseconds per launch, so the
    # headline value above comes from the uninstrumented run)
    roofline = None
    kernels = {}
    kt = not args.no_kernel_timing
    if kt:
        A.rl_timing_reset()
        A.rl_timing_enable(True)
        torch.cuda.synchronize()
        for s in range(args.steps):
            step()
        torch.cuda.synchronize()
        A.rl_timing_enable(False)
        names = ["resident_box", "slide_conv_ratio", "slide_corr_update", "span_conv_ratio",
                 "span_corr_update", "direct_conv_ratio", "direct_corr_update"]
        for nm in names:
            n, ms = A.rl_timing_read(nm)
            if n:
                kernels[nm] = dict(launches=n, total_ms=ms, avg_us=1e3 * ms / n)
        A.rl_timing_reset()
        if kernels:
            dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
            kinfo = kernels[dom]
            kind = dom.split("_")[0]
            # which job ran the dominant kernel
            jname = None
            for j in jobs:
                inf = infos[j["name"]]
                if kind == "resident" and inf["schedule"] == A.RL_SCHED_RESIDENT:
                    jname = j["name"]
                elif kind == "slide" and inf["schedule"] != A.RL_SCHED_RESIDENT and inf["lmax"] == 0:
                    jname = j["name"]
                elif kind in ("span", "direct") and inf["lmax"] > 0:
                    jname = j["name"]
            inf = infos[jname]
            jj = [j for j in jobs if j["name"] == jname][0]
            npx = jj["f"].size
            if kind == "resident":
                units = npx * jj["iters"]
            else:
                units = npx
            fl = algorithmic_flops_per_px(kind, inf, dom.endswith("update")) * units
            achieved = fl / (kinfo["avg_us"] * 1e-6) / 1e12
            roofline = dict(bound="alu", achieved=round(achieved, 4), peak=PEAK_FP32_TFLOPS,
                            unit="TFLOP/s", frac=round(achieved / PEAK_FP32_TFLOPS, 5),
                            traffic=None, kernel=dom, job=jname,
                            avg_us=round(kinfo["avg_us"], 3),
                            flops_per_launch=fl)
    log(f"bench: kernels {json.dumps(kernels)}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(jobs)

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
        "data": "synthetic (seeded generator: shapes + sinusoid, reflect blur, Gaussian noise)",
        "config": {"workload": "specialised PSFs 1024x1024 x3 (vertical box 41, oblique 31@30deg AA, "
                               "disc r10), 200 iterations each",
                   "mode": args.mode,
                   "px_it_per_step": px_it_step,
                   "paths": {k: {"path": A.PATH_NAMES[v["path"]],
                                 "schedule": A.SCHED_NAMES[v["schedule"]]}
                             for k, v in infos.items()}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "other_mode": other,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(jobs):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload."""
    import oracle
    o = oracle.Oracle()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    total_px_it = 0
    t0 = time.perf_counter()
    sample = []
    for j in jobs:
        # about 5 s per job: iterations sized by a one-iteration probe
        p0 = time.perf_counter()
        o.rl(j["f"], j["psf"], 1)
        one = max(time.perf_counter() - p0, 1e-3)
        k = max(1, int(5.0 / one))
        o.rl(j["f"], j["psf"], k)
        total_px_it += j["f"].size * (k + 1)
        sample.append(f"{j['name']} x{k + 1} it")
    dt = time.perf_counter() - t0
    log(f"bench: cpu oracle {total_px_it} px-it in {dt:.2f}s on {cores} threads")
    return dict(value=total_px_it / dt, unit="px-it/s", cores=cores, kind="oracle",
                sample="1024x1024, " + ", ".join(sample) + f" ({dt:.1f}s)")


if __name__ == "__main__":
    main()
