#!/usr/bin/env python3
"""Benchmark of the Schur-complement assembly on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload heat|elast]

A step is one sc_assemble over the whole batch: staircase TRSM X = L^{-1} P B^T
and staircase SYRK F = X^T X with the permutation back, for every subdomain.
Inputs (factor values, tables) are resident in HBM before the timed region:
the host factorisation and its upload happen in sc_factor, untimed.

Prints ONE JSON line on stdout (progress goes to stderr):
  value         subdomains/s over the K timed steps (wall clock, synchronised)
  useful_gflops staircase TRSM + SYRK flop count / time
  roofline      dominant kernel: its useful flops per launch / its mean launch
                duration from HIP events on the launch stream, against the
                FP64 matrix peak of the chip
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SC assembly subdomains/s and useful GFLOP/s per GPU, mixed vs FP64 at stated error"
PEAK_FP64_MATRIX_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
WORKLOADS = {"heat": 2, "elast": 3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(subs, gpu_F, seconds):
    """Times the oracle (long double, as it stands) on subdomains 0, 1, ...
    until `seconds` have elapsed; returns the baseline object and the parity
    errors of the GPU F on the same subdomains."""
    import oracle
    nthreads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    done = 0
    errs = []
    while done < len(subs):
        F = oracle.schur(subs[done], prec="ld", nthreads=nthreads)
        errs.append(oracle.relF(gpu_F(done), F))
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "subdomains/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first {done} subdomains of the batch, long-double oracle (Cholesky in natural "
                      f"order, full forward substitution, Y^T Y), {el:.1f} s"}, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="heat")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-orig", action="store_true", help="also time the assembly without the staircase")
    ap.add_argument("--panel-width", type=int, default=0, help="GPU factor block width (0 = library default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 2 GiB first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); every box here has one MI355X",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import scgen
    import paper_2509_21037_amd as P

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    cfg = WORKLOADS[args.workload]
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("bench: copy calibration: 2 GiB read + 2 GiB written")
        del a, b
    t0 = time.perf_counter()
    subs = scgen.config_subdomains(cfg)
    log(f"bench: generated {len(subs)} subdomains in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    plan = P.Plan(subs, panel_width=args.panel_width)
    log(f"bench: plan created in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    plan.factor()
    torch.cuda.synchronize()
    log(f"bench: host factorisation + upload in {time.perf_counter() - t0:.1f}s")
    st = plan.stats()

    for _ in range(args.warmup):
        plan.assemble()
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.kernel_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.assemble()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = plan.kernel_times(reset=True)
    plan.set_timing(False)
    ms_per_step = 1e3 * elapsed / args.steps
    nsub = st["nsub"]
    useful = st["trsm_useful"] + st["syrk_useful"]
    log(f"bench: {ms_per_step:.3f} ms/step, kernels {kt}")

    flops_per_launch = {"trsm": st["trsm_useful"], "syrk": st["syrk_useful"]}
    avg_ms = {k: kt[k][0] / max(1, kt[k][1]) for k in ("trsm", "syrk")}
    dom = max(avg_ms, key=avg_ms.get)
    achieved = flops_per_launch[dom] / (avg_ms[dom] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_MATRIX_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MATRIX_TFLOPS, "traffic": None,
                "kernel_ms": {k: avg_ms[k] for k in avg_ms},
                "kernel_tflops": {k: flops_per_launch[k] / (avg_ms[k] * 1e-3) / 1e12 for k in avg_ms}}

    orig = None
    if args.compare_orig:
        plan_o = P.Plan(subs, staircase=False, panel_width=args.panel_width)
        plan_o.factor()
        plan_o.assemble()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(max(1, args.steps // 2)):
            plan_o.assemble()
        torch.cuda.synchronize()
        orig = 1e3 * (time.perf_counter() - t1) / max(1, args.steps // 2)
        plan_o.destroy()

    cpu = None
    errs = []
    if not args.no_cpu_baseline:
        cpu, errs = cpu_baseline(subs, plan.get_F, args.cpu_seconds)
        log(f"bench: cpu baseline {cpu}")
    s0 = subs[0]
    out = {
        "metric": METRIC,
        "value": nsub / (ms_per_step * 1e-3),
        "unit": "subdomains/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": scgen.CONFIG_NAMES[cfg], "subdomains": nsub,
                   "n": s0.n if cfg == 2 else "6..16 elements per axis",
                   "m": s0.m if cfg == 2 else "surface DOFs", "precision": "fp64", "staircase": True},
        "useful_gflops": useful / (ms_per_step * 1e-3) / 1e9,
        "useful_gflop_per_step": useful / 1e9,
        "relF_max_sampled": max(errs) if errs else None,
        "relF_samples": len(errs),
        "orig_ms_per_step": orig,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.destroy()


if __name__ == "__main__":
    main()
