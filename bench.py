"""Throughput benchmark of the AP IMEX-RK D2Q6 stepper on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision P]

Prints one JSON line.  A step is one IMEX Runge-Kutta time step of every instance of
the workload (all implicit stages: step-1 relaxation, Helmholtz right-hand side, FFT
Helmholtz solve, u/q update, stage terms).  Inputs are resident in HBM before the
timed region; the timed region is bracketed by torch.cuda.synchronize().

Default: the 8192^2 shear layer (eps = 1e-4, Ma = 0.02, ARS(4,4,3), 200 steps) in the
FP32-split form, the largest single-GPU workload, with the float64 path timed on the
same workload and steps (vs_fp64: speed ratio and relative L2 differences of u, theta
and rho = 1 + 2 eps^2 theta).  Other workloads: --workload shear512 | random2048 |
batched256 | taylor_green64, --precision fp64 | fp32split.

value = 6 * sum(nx * ny) * K / seconds   (cell-population updates/s, Q = 6)

Steps replay HIP graphs (--no-graph: launch by launch); the library's autotuner picks
the launch shapes and whether the Helmholtz solve runs on a second stream beside the
theta-free update kernel.

roofline: the launches of the kernel class with the largest share of step time are timed
during the timed region with HIP events set by the kernel launch itself
(hipExtLaunchKernelGGL: start and end of the kernel's execution), in every
TIMING_STRIDE-th step, which runs launch by launch on the library's main stream so that
each timed launch runs by itself; achieved = its algorithmic bytes per launch (every
plane it must read or write, once) / its mean duration.
roofline.traffic: HBM bytes per launch of that kernel from the rocprofv3 FETCH_SIZE and
WRITE_SIZE runs recorded under profiles/ (each scaled by what the counter reads for a
device copy of known size), reported only for the workload, precision and kernel they
were taken on and while the kernel sources still hash to the recorded value; else null.
roofline.traffic_frac: that measured traffic / the kernel's mean duration / 8 TB/s;
roofline.step_frac: algorithmic bytes of the whole step / step time / 8 TB/s.
roofline.valu_issue_frac: the time the kernel's VALU instructions alone occupy the SIMDs
(waves x instructions per wave x 4 cycles / 1024 SIMDs / 2.4 GHz, from the rocprofv3 SQ
counter run recorded under profiles/, on the same conditions as traffic) / its mean
duration: near 1 the kernel is bound by instruction issue rather than by HBM.
cpu_baseline: the FP64 NumPy oracle on a bounded sample of the same workload, on the
host (one core: NumPy's elementwise kernels and pocketfft are single-threaded).  For the
8192^2 workload one oracle step takes minutes, so the sample is whole steps of the same
flow and parameters on a 1024^2 grid (1/64 of the cells; the oracle's cost per cell is
the same up to the FFT's log factor), labelled as such.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IMEX-RK cell-pop updates/s + %HBM roofline; FP32-split/batched vs FP64"
UNIT = "cell-population updates/s"
HBM_PEAK_GBS = 8000.0
STRUCTURES = {0: "one stream", 1: "solve beside the update", 2: "one stream, theta fused into the update"}
TIMING_STRIDE = 32


def recorded_traffic(kernel_class, workload_name, precision, shape, structure):
    """HBM bytes per launch from the recorded counter runs, or None when they do not
    apply to this kernel, launch shape (tile rows, threads), stream structure (the fused
    one changes what the update and stage-terms launches move) and workload, or the
    kernel sources changed since."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_counters_*.json"))):
        with open(path) as f:
            rec = json.load(f)
        if (rec.get("kernel_class") != kernel_class or rec.get("workload") != workload_name
                or rec.get("precision") != precision
                or (rec.get("tile_rows"), rec.get("threads")) != shape
                or (rec.get("structure", 0) == 2) != (structure == 2)):
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() == rec["source_sha256"]:
            return rec["traffic_bytes_per_launch"]
    return None


def recorded_valu_issue_us(kernel_class, workload_name, precision, shape, structure):
    """VALU issue time per launch (waves x VALU instructions x 4 cycles / 1024 SIMDs /
    2.4 GHz) from the recorded SQ counter run, or None when it does not apply (other
    kernel, launch shape, stream structure or workload, or changed kernel sources)."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "sq_counters_*.json"))):
        with open(path) as f:
            rec = json.load(f)
        if (rec.get("kernel_class") != kernel_class or rec.get("workload") != workload_name
                or rec.get("precision") != precision
                or (rec.get("tile_rows"), rec.get("threads")) != shape
                or (rec.get("structure", 0) == 2) != (structure == 2)):
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() == rec["source_sha256"]:
            return rec["valu_issue_us_per_launch"]
    return None


def workload(name):
    from paper_2512_19847_amd import workloads as wl

    if name == "shear512":
        cases = [wl.shear_layer_512(e) for e in (1.0, 1e-2, 1e-6)]
        cfg = {"workload": "shear_layer_512x512_eps_1_1e-2_1e-6_ars443", "grid": [512, 512],
               "instances": 3, "eps": [1.0, 1e-2, 1e-6], "mach": 0.05,
               "tableau": "ARS(4,4,3)", "space": "WENO5 + 4th-order central",
               "cfl": wl.CFL_ARS, "steps_stated": 2000}
        return cases, "ars443", cfg
    if name == "random2048":
        cases = [wl.random_2048()]
        cfg = {"workload": "random_divfree_2048x2048_k8_rms0.1_eps1e-6_ma0.01_ars443",
               "grid": [2048, 2048], "instances": 1, "eps": 1e-6, "mach": 0.01,
               "tableau": "ARS(4,4,3)", "cfl": wl.CFL_ARS, "steps_stated": 1000}
        return cases, "ars443", cfg
    if name == "batched256":
        cases = wl.batched_256()
        cfg = {"workload": "batched_256_random_divfree_k4_sides64-512_eps1e-6-1_ma0.01-0.1_ars443",
               "instances": len(cases), "cells": int(sum(c.nx * c.ny for c in cases)),
               "tableau": "ARS(4,4,3)", "cfl": wl.CFL_ARS, "steps_stated": 500}
        return cases, "ars443", cfg
    if name == "shear8192":
        cases = [wl.shear_layer_8192()]
        cfg = {"workload": "shear_layer_8192x8192_eps1e-4_ma0.02_ars443", "grid": [8192, 8192],
               "instances": 1, "eps": 1e-4, "mach": 0.02, "tableau": "ARS(4,4,3)",
               "cfl": wl.CFL_ARS, "steps_stated": 200}
        return cases, "ars443", cfg
    if name == "taylor_green64":
        cases = [wl.taylor_green_64("paper2")]
        cfg = {"workload": "taylor_green_64x64_eps1_ma0.1_paper2", "grid": [64, 64],
               "instances": 1, "tableau": "paper second order (c = 9/4)",
               "steps_stated": 100}
        return cases, "paper2", cfg
    raise SystemExit(f"unknown workload {name}")


SAMPLE_SIDE = 1024  # oracle sample grid of workloads whose one step exceeds the budget


def cpu_baseline(cases, tab, budget_s=20.0):
    """Oracle steps on the host, as many whole instance-steps as fit the budget; an
    instance larger than SAMPLE_SIDE^2 is sampled by the same flow and parameters on a
    SAMPLE_SIDE^2 grid."""
    from oracle import scheme, tableau as otab
    from paper_2512_19847_amd import workloads as wl
    from oracle.operators import Production

    sample = []
    proxy = None
    for c in cases:
        if c.nx * c.ny > SAMPLE_SIDE * SAMPLE_SIDE:
            proxy = (c.nx, c.ny)
            st = wl.shear_layer(SAMPLE_SIDE) if c.name.startswith("shear") else \
                wl.random_divfree(SAMPLE_SIDE, kmax=8, rms=0.1, seed=3)
            c = wl.Case(c.name + "_sample", st, c.eps, c.tau, c.dt, c.tableau, c.lx, c.ly)
        sample.append(c)
    t0 = time.perf_counter()
    done_cells = 0
    k = 0
    while True:
        c = sample[k % len(sample)]
        ops = Production(c.lx / c.nx, c.ly / c.ny)
        scheme.step(c.state, scheme.Params(c.eps, c.tau, c.dt), otab.preset(tab), ops)
        done_cells += c.nx * c.ny
        k += 1
        el = time.perf_counter() - t0
        if el >= budget_s or k >= 3 * len(sample):
            break
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0))
    what = (f"{k} oracle steps of the same flow, eps, tau and dt on a {SAMPLE_SIDE}^2 grid "
            f"(sample of the {proxy[0]}x{proxy[1]} workload: 1/"
            f"{proxy[0] * proxy[1] // (SAMPLE_SIDE * SAMPLE_SIDE)} of the cells; extrapolated "
            "per cell)" if proxy else f"{k} instance-steps of the same workload")
    return {"value": 6.0 * done_cells / el, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"{what} ({el:.1f} s) on one core of {avail} available ({model})"}


def compare_fp64(apdvm, torch, stream, sim, cases, tab, args, sec):
    """Same workload and steps in float64: speed ratio and relative L2 differences of the
    final states (velocity, theta, density rho = 1 + 2 eps^2 theta), worst instance."""
    ref = apdvm.Simulation([dict(nx=c.nx, ny=c.ny, eps=c.eps, tau=c.tau, dt=c.dt, lx=c.lx,
                                 ly=c.ly) for c in cases], tableau=tab, precision=apdvm.FP64,
                           stream=stream)
    for k, c in enumerate(cases):
        ref.set_fields(k, *c.state)
    ref.set_graph(args.graph)
    ref.autotune(3)
    ref.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref.step(args.steps)
    torch.cuda.synchronize()
    sec64 = time.perf_counter() - t0
    # the split run took warmup + 36 probe + steps steps; bring the reference level
    ref.step(len(apdvm.KERNEL_CLASSES) * 4)
    worst = {"u": 0.0, "theta": 0.0, "rho": 0.0}
    for k, c in enumerate(cases):
        a, b = sim.get_fields(k), ref.get_fields(k)
        l2 = lambda x, y: float(np.sqrt(np.sum((x - y) ** 2)) / np.sqrt(np.sum(y ** 2)))
        e = {"u": l2(np.stack(a[:2]), np.stack(b[:2])), "theta": l2(a[2], b[2]),
             "rho": l2(1 + 2 * c.eps ** 2 * a[2], 1 + 2 * c.eps ** 2 * b[2])}
        for key in worst:
            worst[key] = max(worst[key], e[key])
    ref.close()
    return {"fp64_ms_per_step": sec64 / args.steps * 1e3, "speedup": sec64 / sec,
            "rel_l2": worst, "steps_compared": args.warmup + args.steps +
            len(apdvm.KERNEL_CLASSES) * 4}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="shear8192")
    ap.add_argument("--precision", default="fp32split", choices=["fp64", "fp32split"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare-fp64", dest="compare_fp64", action="store_false",
                    help="skip timing the float64 path on the same workload and steps (the "
                         "FP32-split line reports the speed ratio and the relative L2 "
                         "differences of the final states by default)")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="launch kernel by kernel instead of replaying each step as a HIP graph")
    ap.add_argument("--one-stream", action="store_true",
                    help="after autotuning, run every launch on one stream (no solve beside the "
                         "update), so that a kernel trace shows each kernel by itself, as the "
                         "sampled timed steps do")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (torch copy kernel) so that "
                         "hardware byte counters can be scaled against a known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is documented as a design and not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_19847_amd import apdvm

    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 3 copies of 268435456 bytes", file=sys.stderr)
        del src, dst

    cases, tab, cfg = workload(args.workload)
    prec = apdvm.FP32_SPLIT if args.precision == "fp32split" else apdvm.FP64
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    sim = apdvm.Simulation([dict(nx=c.nx, ny=c.ny, eps=c.eps, tau=c.tau, dt=c.dt,
                                 lx=c.lx, ly=c.ly) for c in cases],
                           tableau=tab, precision=prec, stream=stream)
    for k, c in enumerate(cases):
        sim.set_fields(k, *c.state)
    sim.set_graph(args.graph)
    cells = sum(c.nx * c.ny for c in cases)
    tiles = sim.autotune(3)
    if args.one_stream and sim.overlap() == 1:
        sim.set_overlap(0)  # the same kernels, every launch on one stream

    # warm-up, then find the kernel class with the largest share of a step (timed steps
    # run every launch by itself)
    sim.step(args.warmup)
    share = []
    for cls in range(len(apdvm.KERNEL_CLASSES)):
        sim.timing_enable(cls)
        sim.step(4)
        n, ms = sim.timing_read()
        share.append(ms)
    sim.timing_enable(-1)
    dom = int(np.argmax(share))

    # timed region: the launches of the dominant class in every TIMING_STRIDE-th step are
    # bracketed by HIP events (all of that step's launches of the class, so every stage is
    # sampled alike; the events cost a little time themselves)
    sim.timing_enable(dom)
    sim.timing_stride(TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_dom, ms_dom = sim.timing_read()
    sim.timing_stride(1)
    sim.timing_enable(-1)
    sec = t1 - t0

    dname = apdvm.KERNEL_CLASSES[dom]
    shape = (tiles.get(dname), tiles.get("threads_" + dname))
    traffic = recorded_traffic(dname, cfg["workload"], args.precision, shape, sim.overlap())
    valu_us = recorded_valu_issue_us(dname, cfg["workload"], args.precision, shape,
                                     sim.overlap())
    bytes_step, launches = sim.traffic(dom)
    per_launch = bytes_step / launches
    mean_s = ms_dom / n_dom / 1e3
    achieved = per_launch / mean_s / 1e9
    diag = [sim.diagnostics(k) for k in range(len(cases))]
    finite = all(d[7] == 1.0 for d in diag)
    total_bytes, nl = sim.traffic(-1)
    print(f"[bench] {args.workload} {args.precision}: {sec / args.steps * 1e3:.3f} ms/step, "
          f"{nl} launches/step, algorithmic {total_bytes / 1e6:.1f} MB/step "
          f"({total_bytes / (sec / args.steps) / 1e9:.0f} GB/s whole step); class shares ms "
          f"{dict(zip(apdvm.KERNEL_CLASSES, [round(x, 3) for x in share]))}; finite={finite}",
          file=sys.stderr)

    out = {
        "metric": METRIC,
        "value": 6.0 * cells * args.steps / sec,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == apdvm.FP64 else "f32+f64",
        "data": "synthetic",
        "config": dict(cfg, precision=args.precision,
                       tile_rows={k: tiles[k] for k in apdvm.TUNED_STENCIL},
                       threads={k: tiles["threads_" + k] for k in apdvm.TUNED_STENCIL},
                       graph=bool(args.graph), stream_structure=STRUCTURES[sim.overlap()]),
        "roofline": {"bound": "hbm", "kernel": apdvm.KERNEL_CLASSES[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     # measured HBM bytes (rocprofv3 counters) / mean launch time / peak
                     "traffic_frac": traffic / mean_s / 1e9 / HBM_PEAK_GBS if traffic else None,
                     "valu_issue_frac": valu_us * 1e-6 / mean_s if valu_us else None,
                     "bytes_per_launch": per_launch, "mean_launch_us": mean_s * 1e6,
                     "launches_timed": n_dom,
                     # every kernel of the step: algorithmic bytes / step time
                     "step_gbs": total_bytes / (sec / args.steps) / 1e9,
                     "step_frac": total_bytes / (sec / args.steps) / 1e9 / HBM_PEAK_GBS},
        "finite": finite,
    }
    if args.compare_fp64 and prec != apdvm.FP64:
        out["vs_fp64"] = compare_fp64(apdvm, torch, stream, sim, cases, tab, args, sec)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cases, tab)
    sim.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
