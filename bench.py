#!/usr/bin/env python3
"""Benchmark of the Schur-complement assembly on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload heat|elast|large]
                    [--pcpg ITERS] [--no-mixed] [--no-cpu-baseline] [--compare-orig] [--compare-reach]

A step is one sc_assemble over the whole batch: staircase TRSM X = L^{-1} P B^T
and staircase SYRK F = X^T X with the permutation back, for every subdomain.
Inputs (factor values, tables) are resident in HBM before the timed region:
the host factorisation and its upload happen in sc_factor, untimed.

Workloads: large = 64 x 20^3 hex8 elasticity subdomains (27783 DOFs, 7938
                   per-face multipliers each; the default and the headline:
                   the largest single-GPU configuration), with the
                   explicit-vs-implicit apply and the amortisation point,
           heat  = 1024 x 12^3 hex8 heat subdomains,
           elast = 512 uneven hex8 elasticity boxes (6..16 elements per axis);
                   with --pcpg both assemblies run that many PCPG iterations.

Prints ONE JSON line on stdout (progress goes to stderr):
  value         subdomains/s of the FP64 assembly over the K timed steps
                (wall clock, synchronised)
  useful_gflops structural TRSM + SYRK flop count / time: the flops on the
                structurally nonzero rows of X only (sum_i r(i)(2 c_i - 1) +
                r(i)(r(i) + 1), r(i) = columns of X nonzero in row i); the
                staircase count (a(i) = columns with pivot <= i) is reported
                beside it as staircase_gflop_per_step
  mixed         the same assembly in mixed precision (its difference to the
                FP64 GPU result on kept subdomains)
  relF_*        errors against the oracle, computed inside the cpu_baseline
                leg on the subdomains it runs (GPU F kept from both plans)
  roofline      dominant kernel of the FP64 assembly: structural flops per launch /
                mean launch duration (HIP events on the launch stream), against
                the chip's published FP64 matrix peak
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
                (large subdomains: 256-column subsets of two subdomains, the
                whole-F time extrapolated from its timed steps)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SC assembly subdomains/s and useful GFLOP/s per GPU, mixed vs FP64 at stated error"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
PEAK_HBM_GBS = 8000.0
WORKLOADS = {"heat": 2, "elast": 3, "large": 5}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that fix what an assembly launch reads and writes: the kernels and
# the planner that lays out their blocks, tiles and merged pairs.
PROFILED_SOURCES = ("kernels.hip", "planner.cpp")


def kernels_digest():
    import hashlib
    h = hashlib.sha256()
    for name in PROFILED_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_21037_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it was taken on other kernel or planner sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_sha256") != kernels_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def blended_peak(workload):
    """Peak of the mixed-precision assembly weighted by its own flop split
    (FP64 MFMA for the diagonal blocks at 78.6 TFLOP/s, FP32 MFMA for the rest
    at 157.3): total / (f64 / peak64 + f32 / peak32), with the MFMA flops the
    counter summary of the mixed TRSM and SYRK launches recorded, or None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_mixed.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    ks = t.get("kernels", {})
    f64 = sum(k.get("mfma_f64_flops", 0.0) for k in ks.values())
    f32 = sum(k.get("mfma_f32_flops", 0.0) for k in ks.values())
    if f64 + f32 <= 0:
        return None
    return {"tflops": (f64 + f32) / (f64 / PEAK_TFLOPS["fp64"] + f32 / PEAK_TFLOPS["fp32"]),
            "fp64_share": f64 / (f64 + f32)}


def time_assembly(torch, plan, steps, warmup, graph=False):
    """Wall-clock ms per sc_assemble over `steps` synchronised steps, and the
    mean per-kernel ms from HIP events (an extra eager pass when the plan
    replays a captured graph)."""
    for _ in range(warmup):
        plan.assemble()
    torch.cuda.synchronize()
    if not graph:
        plan.set_timing(True)
        plan.kernel_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.assemble()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if graph:
        plan.set_timing(True)
        plan.kernel_times(reset=True)
        for _ in range(max(1, min(steps, 3))):
            plan.assemble()
        torch.cuda.synchronize()
    kt = plan.kernel_times(reset=True)
    plan.set_timing(False)
    return 1e3 * elapsed / steps, {k: kt[k][0] / kt[k][1] for k in ("trsm", "syrk", "assemble_overlap")
                                   if kt[k][1] > 0}


def time_apply(torch, plan, which, iters=20):
    """(wall-clock ms per apply, HIP-event ms per apply); the wall clock
    covers graph replays where the plan uses them, the events an eager pass."""
    st = plan.stats()
    p = torch.rand(st["dual_total"], dtype=torch.float64, device="cuda")
    q = torch.zeros_like(p)
    f = plan.apply if which == "explicit" else plan.apply_implicit
    f(p, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        f(p, q)
    torch.cuda.synchronize()
    wall = 1e3 * (time.perf_counter() - t0) / iters
    plan.set_timing(True)
    plan.kernel_times(reset=True)
    for _ in range(iters):
        f(p, q)
    torch.cuda.synchronize()
    kt = plan.kernel_times(reset=True)
    plan.set_timing(False)
    key = "apply" if which == "explicit" else "apply_implicit"
    return wall, kt[key][0] / max(1, kt[key][1])


def preprocessing_times(torch, plan, factor_s, asm_ms, reps=2):
    """The whole preprocessing stage (Sec. 4.4): host factorisation and
    extraction of the factors, upload, GPU assembly.  sep = sc_factor (timed
    once, synchronised) + the timed assembly step; mix = sc_preprocess (host
    factorisation of later subdomain groups overlapped with the GPU assembly
    of earlier ones), wall clock to the end of the stream, best of `reps`."""
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.preprocess()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        best = el if best is None else min(best, el)
    sep = factor_s + asm_ms * 1e-3
    return {"factor_upload_s": factor_s, "assembly_s": asm_ms * 1e-3, "sep_s": sep, "mix_s": best,
            "mix_gain": sep / best, "host_threads": min(16, os.cpu_count() or 1)}


def time_selection(torch, subs, iters, panel_width, use_graph):
    """Per-subdomain explicit / implicit choice for `iters` applications
    (Sec. 5): the whole cost (assembly + iters applications, FP64) with the
    plan's choice, all explicit, and all implicit (the implicit apply needs no
    assembly)."""
    out = {"iterations": iters}
    for name, kw in (("hybrid", {"select_iters": iters}), ("explicit", {}),
                     ("implicit", {"select_iters": iters, "select_model": (1.0, 1.0, 1e9)})):
        plan = P_mod().Plan(subs, panel_width=panel_width, use_graph=use_graph, block_split="etree", **kw)
        plan.factor()
        ms_asm, _ = time_assembly(torch, plan, 3, 1, use_graph)
        st = plan.stats()
        p = torch.rand(st["dual_total"], dtype=torch.float64, device="cuda")
        q = torch.zeros_like(p)
        plan.apply(p, q)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            plan.apply(p, q)
        torch.cuda.synchronize()
        ms_apply = 1e3 * (time.perf_counter() - t0) / iters
        nimp = sum(plan.selection(i)["implicit"] for i in range(len(subs)))
        out[name] = {"implicit_subdomains": nimp, "assembly_ms": ms_asm, "apply_ms": ms_apply,
                     "total_ms": ms_asm + iters * ms_apply}
        plan.destroy()
    return out


def paper_curves(torch, cap_gb=32.0, dims=(2, 3)):
    """The paper's own workloads (Sec. 4: heat transfer on P1 triangles and
    tetrahedra, the subdomain sizes of its figures, batches of about 8.4 M (2D)
    / 1.1 M (3D) unknowns): FP64 assembly time per subdomain without the
    staircase ("orig", Sec. 3.1), with the staircase alone (Sec. 3.2-3.3) and
    with the staircase restricted to the elimination-tree reach, one plan at a
    time, the X temporary capped at cap_gb (waves) so that every size fits."""
    import scgen
    out = []
    for dim in dims:
        for nodes in scgen.PAPER_NODES[dim]:
            subs = scgen.paper_subdomains(dim, nodes)
            row = {"dim": dim, "nodes_per_side": nodes, "n": subs[0].n, "m": subs[0].m, "subdomains": len(subs)}
            for name, kw in (("orig", {"staircase": False}), ("staircase", {"reach": False}), ("reach", {})):
                plan = P_mod().Plan(subs, arena_cap_bytes=int(cap_gb * 2 ** 30), **kw)
                plan.factor()
                ms, _ = time_assembly(torch, plan, 2, 1)
                row[f"{name}_ms_per_subdomain"] = ms / len(subs)
                plan.destroy()
            row["speedup_staircase"] = row["orig_ms_per_subdomain"] / row["staircase_ms_per_subdomain"]
            row["speedup_reach"] = row["orig_ms_per_subdomain"] / row["reach_ms_per_subdomain"]
            log(f"bench: paper workload {row}")
            out.append(row)
    return out


def P_mod():
    import paper_2509_21037_amd as P
    return P


def sample_ids(subs, big):
    """Subdomains whose GPU F is kept for the error check of the cpu_baseline
    leg (the leg runs the oracle on subdomains 0, 1, ... in order): the first
    two of the large-subdomain batch, the first eight otherwise."""
    return list(range(min(2 if big else 8, len(subs))))


SAMPLE_COLS = 256


def sample_cols(s, i):
    """Seeded column subset (256 columns, sorted) the cpu_baseline leg uses
    for subdomain i when its n exceeds 3000."""
    import numpy as np
    rng = np.random.default_rng(1000 + i)
    return np.sort(rng.choice(s.m, size=min(SAMPLE_COLS, s.m), replace=False))


def keep_F(plan, subs, ids):
    """Host copies of F (or F[S, S] for the large subdomains) for `ids`."""
    import numpy as np
    out = {}
    for i in ids:
        F = plan.get_F(i)
        if subs[i].n > 3000:
            sel = sample_cols(subs[i], i)
            F = F[np.ix_(sel, sel)]
        out[i] = F
    return out


def rel_diff(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cpu_baseline(subs, seconds, kept=None, big=False):
    """The FP64 oracle (as it stands: natural-order Cholesky, forward
    substitution of every column over all rows, Y^T Y) on the host cores.
    Small subdomains (n <= 3000): whole F of subdomains 0, 1, ... until
    `seconds` have elapsed; value = subdomains per second.  Large ones: F[S, S]
    for a seeded 256-column subset S of the first two subdomains, each step
    timed; the time of the whole F of one subdomain is extrapolated as
    t_chol + t_fwd * m / |S| + t_syrk * m (m + 1) / (|S| (|S| + 1)) (the
    Cholesky is independent of the columns, the substitution linear in them,
    Y^T Y quadratic); value = 1 / that time.  Where a GPU result was kept
    (`kept`: precision -> {subdomain: F}), its relative Frobenius error
    against the oracle's F."""
    import numpy as np
    import oracle
    kept = kept or {}
    nthreads = max(1, min(16, os.cpu_count() or 1))
    errs = {k: [] for k in kept}
    t0 = time.perf_counter()
    done = 0
    full_times = []
    phases = []
    while done < len(subs):
        s = subs[done]
        if big:
            sel = sample_cols(s, done)
            F = oracle.schur(s, sel=sel, prec="d", nthreads=nthreads)
            tc, tf, ts = oracle.last_phase_seconds()
            k = len(sel)
            full_times.append(tc + tf * s.m / k + ts * s.m * (s.m + 1) / (k * (k + 1)))
            phases.append((tc, tf, ts))
        else:
            F = oracle.schur(s, prec="d", nthreads=nthreads)
        for key, fk in kept.items():
            if done in fk:
                errs[key].append(oracle.relF(fk[done], F))
        done += 1
        if big and done >= 2:
            break
        if not big and time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    if big:
        tfull = float(np.mean(full_times))
        ph = np.mean(np.array(phases), axis=0)
        out = {"value": 1.0 / tfull, "unit": "subdomains/s", "cores": nthreads, "kind": "oracle",
               "sample": f"FP64 oracle on F[S, S] of subdomains 0..{done - 1}, |S| = {SAMPLE_COLS} seeded "
                         f"columns, {el:.1f} s measured (Cholesky {ph[0]:.1f} s on one thread, substitution "
                         f"{ph[1]:.2f} s, Y^T Y {ph[2]:.3f} s per subdomain); whole-F time per subdomain "
                         f"extrapolated as t_chol + t_fwd m/|S| + t_syrk m(m+1)/(|S|(|S|+1)) = {tfull:.0f} s",
               "measured_s": el, "extrapolated_s_per_subdomain": tfull}
    else:
        out = {"value": done / el, "unit": "subdomains/s", "cores": nthreads, "kind": "oracle",
               "sample": f"first {done} subdomains of the batch, whole F by the FP64 oracle (Cholesky in "
                         f"natural order, full forward substitution, Y^T Y), {el:.1f} s",
               "measured_s": el}
    return out, errs


def ld_errors(subs, kept, big):
    """relF of the kept GPU F against the long-double oracle (the parity
    reference: on the 20^3 elasticity subdomains the FP64 oracle itself is
    ~7e-12 away from it): every kept subdomain when they are small, the first
    one (its seeded 256-column subset) when they are large."""
    import oracle
    nthreads = max(1, min(16, os.cpu_count() or 1))
    ids = sorted(next(iter(kept.values())).keys()) if kept else []
    if big:
        ids = ids[:1]
    errs = {k: [] for k in kept}
    for i in ids:
        s = subs[i]
        sel = sample_cols(s, i) if big else None
        ref = oracle.schur(s, sel=sel, prec="ld", nthreads=nthreads)
        for key, fk in kept.items():
            errs[key].append(oracle.relF(fk[i], ref))
    return errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="large")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--pcpg", type=int, default=0, help="PCPG iterations on the FP64 and the mixed F")
    ap.add_argument("--compare-orig", action="store_true", help="also time the assembly without the staircase")
    ap.add_argument("--compare-reach", action="store_true",
                    help="also time the FP64 assembly with the TRSM sweeping every block after the first pivot")
    ap.add_argument("--panel-width", type=int, default=0, help="GPU factor block width (0 = library default)")
    ap.add_argument("--autotune", choices=("auto", "on", "off"), default="auto",
                    help="per-size-class autotuner (block split, width, SYRK kind; auto: on unless "
                         "--panel-width is given)")
    ap.add_argument("--graph", choices=("auto", "on", "off"), default="auto",
                    help="replay the assembly as a captured HIP graph (auto: on for the elasticity batches)")
    ap.add_argument("--assembly", choices=("overlap", "separate"), default="separate",
                    help="TRSM and SYRK of successive subdomain groups overlapped on two streams, or two launches")
    ap.add_argument("--compare-assembly", action="store_true",
                    help="also time the FP64 assembly in the other mode (overlap / separate)")
    ap.add_argument("--tune-cache", default=None, help="autotune cache file (read, and appended to)")
    ap.add_argument("--tune-sample", type=int, default=0,
                    help="autotune subdomains per size class (default: 128 heat, 8 uneven elasticity, 16 20^3)")
    ap.add_argument("--paper-curves", action="store_true",
                    help="also time the paper's P1 triangle / tetrahedron heat workloads at its figure sizes, "
                         "without the staircase, with it, and with the reach (FP64, ms per subdomain)")
    ap.add_argument("--select", type=int, default=0,
                    help="also time K applications with per-subdomain explicit / implicit selection for K "
                         "iterations, against all-explicit and all-implicit (FP64)")
    ap.add_argument("--block-split", choices=("uniform", "etree"), default="uniform",
                    help="GPU factor blocks: uniform column ranges, or ranges that follow the elimination tree")
    ap.add_argument("--no-prep", dest="prep", action="store_false",
                    help="skip the whole-preprocessing timing (factorisation + assembly, separate and pipelined)")
    ap.add_argument("--latency", action="store_true",
                    help="also time one 16 x 16 Q1 single-subdomain assembly (median of 1000 calls)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 2 GiB first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); every box here has one MI355X",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    big = subs[0].n > 3000
    ids = sample_ids(subs, big)
    use_graph = args.graph == "on" or (args.graph == "auto" and cfg != 2)
    tune, classes64, classes32 = None, None, None
    if args.autotune == "on" or (args.autotune == "auto" and not args.panel_width):
        # per size class: block split, block width, SYRK work items (FP64 and
        # mixed tuned separately), on samples of each class; not timed
        t0 = time.perf_counter()
        # the sample of a class must fill the chip the way the batch does
        # (12^3 heat: 14 column tiles per subdomain, 128 of them ~1800
        # workgroups); 8 per class of the uneven batch, 16 of the 20^3 ones
        smp = args.tune_sample or {2: 128, 3: 8}.get(cfg, 16)
        classes64 = P.autotune_classes(subs, sample=smp, reps=2, cache_path=args.tune_cache)
        classes32 = None if args.no_mixed else \
            P.autotune_classes(subs, sample=smp, reps=2, cache_path=args.tune_cache, precision="mixed")
        tune = {"fp64": classes64, "mixed": classes32, "sample_per_class": smp,
                "seconds": time.perf_counter() - t0}
        log(f"bench: autotune {tune}")

    # ---------------------------------------------------------------- FP64
    t0 = time.perf_counter()
    plan = P.Plan(subs, panel_width=args.panel_width, use_graph=use_graph, assembly=args.assembly,
                  block_split=args.block_split, tune_classes=classes64)
    t1 = time.perf_counter()
    plan.factor()
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    prep_factor_s = time.perf_counter() - t1
    log(f"bench: FP64 plan + host factorisation + upload in {prep_s:.1f}s (not in the timed region)")
    st = plan.stats()
    plan_nnzl = [plan.query(i)["nnzL"] for i in range(len(subs))]
    ms_per_step, kms = time_assembly(torch, plan, args.steps, args.warmup, use_graph)
    log(f"bench: FP64 {ms_per_step:.3f} ms/step, kernels {kms}")
    useful = st["trsm_reach"] + st["syrk_reach"]
    flops = {"trsm": st["trsm_reach"], "syrk": st["syrk_reach"], "assemble_overlap": useful}
    dom = max(kms, key=kms.get)
    achieved = flops[dom] / (kms[dom] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_TFLOPS["fp64"],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["fp64"],
                "traffic": measured_traffic(args.workload, "fp64", dom),
                "kernel_ms": kms,
                "kernel_tflops": {k: flops[k] / (kms[k] * 1e-3) / 1e12 for k in kms}}
    kept = {"fp64": keep_F(plan, subs, ids)}
    prep = preprocessing_times(torch, plan, prep_factor_s, ms_per_step) if args.prep else None
    if prep:
        log(f"bench: FP64 preprocessing {prep}")
    _, apply64 = time_apply(torch, plan, "explicit")
    # the apply reads the stored F: lower 128 x 128 tiles in sorted column order
    f_bytes64 = sum((t := (s.m + 127) // 128) * (t + 1) // 2 * 128 * 128 for s in subs) * 8
    extra = {"explicit_fp64F_ms": apply64, "explicit_fp64F_GBps": f_bytes64 / (apply64 * 1e-3) / 1e9}
    pcpg = {}
    d = None
    if args.pcpg:
        d = torch.from_numpy(scgen.splitmix64_uniform(scgen.BASE_SEED + 4, st["dual_total"])).cuda()
        lam64 = torch.zeros_like(d)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h64 = plan.pcpg(d, lam64, args.pcpg, history=True)
        pcpg["iterations"] = args.pcpg
        pcpg["fp64_s"] = time.perf_counter() - t1
        pcpg["fp64_w_reduction_worst"] = float(np.max(h64[-1] / np.maximum(h64[0], 1e-300)))
    if cfg == 5:
        # graph replays (the triangular sweeps) where the plan uses them; the
        # HIP-event time of the eager launches beside it
        wall_i, extra["implicit_eager_ms"] = time_apply(torch, plan, "implicit", iters=5)
        extra["implicit_ms"] = wall_i if use_graph else extra["implicit_eager_ms"]
        extra["implicit_split"] = args.block_split
        log(f"bench: apply {extra}")
    orig, kms_o, prep_orig = None, None, None
    if args.compare_orig:
        plan_o = P.Plan(subs, staircase=False, panel_width=args.panel_width)
        t1 = time.perf_counter()
        plan_o.factor()
        torch.cuda.synchronize()
        fo_s = time.perf_counter() - t1
        orig, kms_o = time_assembly(torch, plan_o, max(1, args.steps // 2), 1)
        if args.prep:
            prep_orig = preprocessing_times(torch, plan_o, fo_s, orig, reps=1)
            log(f"bench: FP64 preprocessing without the staircase {prep_orig}")
        plan_o.destroy()
        log(f"bench: FP64 without the staircase {orig:.3f} ms/step, kernels {kms_o}")
    noreach = None
    if args.compare_reach:
        plan_r = P.Plan(subs, reach=False, panel_width=args.panel_width)
        plan_r.factor()
        noreach, kms_r = time_assembly(torch, plan_r, max(1, args.steps // 2), 1)
        plan_r.destroy()
        log(f"bench: FP64 without the reach {noreach:.3f} ms/step, kernels {kms_r}")
    # latency of one small assembly (16 x 16 Q1 square, m = 64): median of 1000
    lat1 = None
    if args.latency:
        sub1 = scgen.config_subdomains(1)
        plan1 = P.Plan(sub1)
        plan1.factor()
        for _ in range(20):
            plan1.assemble()
        torch.cuda.synchronize()
        lt = []
        for _ in range(1000):
            t1 = time.perf_counter()
            plan1.assemble()
            torch.cuda.synchronize()
            lt.append(time.perf_counter() - t1)
        lat1 = 1e6 * float(np.median(lt))
        plan1.destroy()
        log(f"bench: 16x16 Q1 single-subdomain assembly latency {lat1:.1f} us (median of 1000)")
    other = None
    if args.compare_assembly:
        alt = "separate" if args.assembly == "overlap" else "overlap"
        plan_s = P.Plan(subs, panel_width=args.panel_width, use_graph=use_graph, assembly=alt)
        plan_s.factor()
        ms_s, kms_s = time_assembly(torch, plan_s, args.steps, args.warmup, use_graph)
        other = {"assembly": alt, "ms_per_step": ms_s, "kernel_ms": kms_s,
                 "kernel_tflops": {k: flops[k] / (kms_s[k] * 1e-3) / 1e12 for k in kms_s}}
        log(f"bench: FP64 {alt} assembly {ms_s:.3f} ms/step, kernels {kms_s}")
        plan_s.destroy()
    plan.destroy()
    if cfg == 5 and args.block_split != "etree":
        # the implicit apply on factor blocks that follow the elimination tree
        # (independent subtrees solved in parallel): a plan of its own, factor
        # only; the amortisation point uses the faster of the two
        plan_i = P.Plan(subs, panel_width=args.panel_width, use_graph=use_graph, block_split="etree")
        plan_i.factor()
        wall_e, eager_e = time_apply(torch, plan_i, "implicit", iters=5)
        plan_i.destroy()
        t_e = wall_e if use_graph else eager_e
        extra["implicit_etree_ms"] = t_e
        extra["implicit_etree_eager_ms"] = eager_e
        if t_e < extra["implicit_ms"]:
            extra["implicit_uniform_ms"] = extra["implicit_ms"]
            extra["implicit_ms"], extra["implicit_split"] = t_e, "etree"
        log(f"bench: implicit apply, etree blocks: {t_e:.3f} ms")
    if cfg == 5:
        # HBM floor of the implicit apply: the factor read twice (FP64)
        nnzl = sum(plan_nnzl)
        extra["implicit_hbm_floor_ms"] = 2 * 8 * nnzl / (PEAK_HBM_GBS * 1e9) * 1e3
        extra["implicit_frac_of_floor"] = extra["implicit_hbm_floor_ms"] / extra["implicit_ms"]

    curves = paper_curves(torch) if args.paper_curves else None
    selection = None
    if args.select:
        selection = time_selection(torch, subs, args.select, args.panel_width, use_graph)
        log(f"bench: selection for {args.select} iterations {selection}")

    # ---------------------------------------------------------------- mixed
    mixed = None
    if not args.no_mixed:
        plan_m = P.Plan(subs, precision="mixed", panel_width=args.panel_width, use_graph=use_graph,
                        assembly=args.assembly, block_split=args.block_split, tune_classes=classes32)
        plan_m.factor()
        ms_m, kms_m = time_assembly(torch, plan_m, args.steps, args.warmup, use_graph)
        log(f"bench: mixed {ms_m:.3f} ms/step, kernels {kms_m}")
        kept["mixed"] = keep_F(plan_m, subs, ids)
        _, apply32 = time_apply(torch, plan_m, "explicit")
        mixed = {"ms_per_step": ms_m, "subdomains_per_s": len(subs) / (ms_m * 1e-3),
                 "useful_gflops": useful / (ms_m * 1e-3) / 1e9, "kernel_ms": kms_m,
                 "kernel_tflops": {k: flops[k] / (kms_m[k] * 1e-3) / 1e12 for k in kms_m},
                 "frac_of_fp32_mfma_peak": useful / (ms_m * 1e-3) / 1e12 / PEAK_TFLOPS["fp32"],
                 "blended_peak": blended_peak(args.workload),
                 "relF_vs_fp64_gpu_max": max(rel_diff(kept["mixed"][i], kept["fp64"][i]) for i in ids)}
        if mixed["blended_peak"]:
            mixed["frac_of_blended_peak"] = useful / (ms_m * 1e-3) / 1e12 / mixed["blended_peak"]["tflops"]
        extra["explicit_fp32F_ms"] = apply32
        extra["explicit_fp32F_GBps"] = f_bytes64 / 2 / (apply32 * 1e-3) / 1e9
        if args.pcpg:
            lam32 = torch.zeros_like(d)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            plan_m.pcpg(d, lam32, args.pcpg, history=False)
            pcpg["mixed_s"] = time.perf_counter() - t1
            pcpg["lambda_rel_err_mixed_vs_fp64"] = float(torch.linalg.norm(lam32 - lam64) / torch.linalg.norm(lam64))
        if cfg == 5:
            t_impl = extra["implicit_ms"]
            for name, t_asm, t_expl in (("fp64", ms_per_step, extra["explicit_fp64F_ms"]),
                                        ("mixed", ms_m, apply32)):
                gain = t_impl - t_expl
                extra[f"amortization_iters_{name}"] = (t_asm / gain) if gain > 0 else None
        plan_m.destroy()

    cpu, errs64 = (None, {}) if args.no_cpu_baseline else cpu_baseline(subs, args.cpu_seconds, kept, big)
    if cpu:
        log(f"bench: cpu baseline {cpu}")
        log(f"bench: relF against the FP64 oracle {errs64}")
    errs = {} if args.no_cpu_baseline else ld_errors(subs, kept, big)
    import numpy as np

    def err_stats(e):
        return {"relF_max_sampled": max(e) if e else None,
                "relF_median_sampled": float(np.median(e)) if e else None, "relF_samples": len(e)}
    if mixed is not None:
        mixed.update(err_stats(errs.get("mixed", [])))
        log(f"bench: mixed relF vs oracle {errs.get('mixed')}")
    log(f"bench: FP64 relF vs oracle {errs.get('fp64')}")
    s0 = subs[0]
    out = {
        "metric": METRIC,
        "value": len(subs) / (ms_per_step * 1e-3),
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
        "config": {"workload": scgen.CONFIG_NAMES[cfg], "subdomains": len(subs),
                   "n": s0.n if cfg != 3 else "1029..14739", "m": s0.m if cfg != 3 else "654..4614",
                   "precision": "fp64", "staircase": True, "reach": True,
                   "panel_width": "per size class (autotune)" if classes64 else (args.panel_width or 64),
                   "graph": use_graph, "assembly": args.assembly, "block_split": args.block_split},
        "autotune": tune,
        "useful_gflops": useful / (ms_per_step * 1e-3) / 1e9,
        "useful_gflop_per_step": useful / 1e9,
        "staircase_gflop_per_step": (st["trsm_useful"] + st["syrk_useful"]) / 1e9,
        **err_stats(errs.get("fp64", [])),
        "relF_source": "long-double oracle against the kept GPU F: the first 8 subdomains whole (small "
                       "subdomains), the seeded 256-column subset F[S, S] of subdomain 0 (n > 3000)",
        "relF_vs_fp64_oracle": errs64.get("fp64"),
        "prep_s": prep_s,
        "preprocessing": prep,
        "preprocessing_orig": prep_orig,
        "speedup_orig_over_opt": None if not (orig and prep and prep_orig) else {
            "gpu_section_sep": orig / ms_per_step, "whole_sep": prep_orig["sep_s"] / prep["sep_s"],
            "whole_mix": prep_orig["mix_s"] / prep["mix_s"]},
        "latency_config1_us": lat1,
        "orig_ms_per_step": orig,
        "orig_kernel_ms": kms_o,
        "no_reach_ms_per_step": noreach,
        "other_assembly": other,
        "mixed": mixed,
        "pcpg": pcpg or None,
        "apply": extra,
        "selection": selection,
        "paper_curves": curves,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
