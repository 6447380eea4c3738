"""Benchmark: directional H2 compression on one MI355X.

A step is one full compression (both bases, transfer matrices, projection of
every admissible block, near field) of a synthetic workload whose points are
already on the device side of the call.  The default workload is the
131072-point golden-spiral sphere, kappa = 64, leaf size 64, eps = 1e-4,
eta1 = 20, eta2 = 5, entries generated on the fly.

Prints ONE JSON line (the contract in the repository's README of the driver):
metric/value/unit, roofline of the dominant kernel (the Gram kernel), and the
CPU baseline (the FP64 oracle on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compression s & GFLOP/s, mixed vs FP64 form at equal eps, n=131072 kappa=64"
PEAK_FP64_MFMA = 78.6e12   # MI355X dense matrix peaks (published)
PEAK_FP32_MFMA = 157.3e12
PEAK_INT8_MFMA = 5.0e15
# HBM bytes per launch of k_gram_i8<0> on the default workload: FETCH_SIZE x 2 +
# WRITE_SIZE x 1 (1 GiB copy calibration), profiles/compress_sphere131072_mixed.md
TRAFFIC_GRAM_I8_LEAF = (2 * 1274155.3 + 305164.0) * 1024
# HBM bytes of all k_project_stacked launches of one compression on the default
# workload (same counters and calibration, same profile)
TRAFFIC_PROJECTION_STACKED = (2 * 9312310.5 + 5717289.25) * 1024


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(dh2, torch, blocks, w, eps, leaf, form, steps, warmup, groups):
    prec = dh2.FP64 if form == "fp64" else dh2.MIXED
    o = dh2.opts(leaf_size=leaf, precision=prec, groups=groups)
    times, st, m = [], None, None
    for it in range(warmup + steps):
        m = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = dh2.compress_helmholtz(blocks, w, eps, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = dh2.stats(m)
        log(f"[bench] {form} step {it} {'warmup' if it < warmup else 'timed'}: {dt:.3f} s "
            f"(device {st['t_total']:.3f} s, gram {st['t_gram_kernel']:.3f} s, "
            f"k_max {st['k_max']}, groups {st['groups']})")
        if it >= warmup:
            times.append(dt)
    return m, st, times


def cpu_baseline(points, w, kappa, leaf, eps, budget_s):
    """The oracle on a bounded sample: leaf block rows of the row basis, in a
    seeded random order, each with its block weights, weighted block row,
    SVD and R product, until the time budget is used."""
    from threadpoolctl import threadpool_info

    from oracle import compress as OC
    from oracle import matrix as OM
    from oracle import plan as OP

    t_plan = time.perf_counter()
    plan = OP.build_plan(points, kappa, leaf)
    t_plan = time.perf_counter() - t_plan
    M = OM.HelmholtzMatrix(points, w, kappa, plan.tree.perm)
    tr, bt = plan.tree, plan.blocks
    items = [(t, c) for t in range(tr.nc) if tr.son1[t] < 0 for c in plan.rowsets.used(t)]
    order = np.random.default_rng(0).permutation(len(items))
    omega = {}
    flops, done = 0.0, 0
    t0 = time.perf_counter()
    for idx in order:
        t, c = items[idx]
        for (b, s, d) in plan.rowsets.F[t][c]:
            if b not in omega:
                omega[b] = np.linalg.norm(M.block(tr.rows(bt.adm_t[b]), tr.rows(bt.adm_s[b])))
        A = OC.weighted_block_row(M, plan, plan.rowsets, t, c, omega, 2.0 / 3.0)
        Q, sig, k = OC.truncated_left_singular(A, eps)
        _ = Q.conj().T @ A
        r, N = A.shape
        flops += 4.0 * r * r * N + 8.0 * k * r * N
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": flops / el / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} of {len(items)} leaf block rows of the row basis "
                      f"(weights, weighted block row, SVD, R product) in {el:.1f} s; "
                      f"oracle plan {t_plan:.1f} s not timed",
            "host_cpus": len(os.sched_getaffinity(0))}


def run_batch(args, dh2, torch, synth):
    """Independent instances (sphere, ellipsoid, cube surface) in one call,
    mixed form, eps 1e-4, leaf 64; also timed one instance after the other."""
    count = int(args.workload[len("batch"):] or 48)
    eps = 1e-4
    inst = synth.batch_instances(count=count, seed=4)
    forms = [f for f in args.forms.split(",") if f]
    form = "mixed" if "mixed" in forms else forms[0]
    o = dh2.opts(leaf_size=64, precision=dh2.MIXED if form == "mixed" else dh2.FP64)
    t0 = time.perf_counter()
    blocks = [dh2.blocks_build(dh2.tree_build(i.points, i.kappa, o), o) for i in inst]
    t_plan = time.perf_counter() - t0
    ws = [i.weights for i in inst]
    log(f"[bench] {count} instances, n from {min(len(i.points) for i in inst)} to "
        f"{max(len(i.points) for i in inst)}, host plans {t_plan:.2f} s")
    times, seq, flops = [], [], 0.0
    for it in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = dh2.compress_batch(blocks, ws, eps, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = [dh2.stats(m) for m in ms]
        flops = sum(x["flops_row"] + x["flops_col"] + x["flops_prj"] for x in st)
        log(f"[bench] batch step {it} {'warmup' if it < args.warmup else 'timed'}: {dt:.3f} s")
        if it >= args.warmup:
            times.append(dt)
        del ms
    # the same instances one after the other (reference for the batching gain)
    for it in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b, w in zip(blocks, ws):
            m = dh2.compress_helmholtz(b, w, eps, o)
            del m
        torch.cuda.synchronize()
        if it == 1:
            seq.append(time.perf_counter() - t0)
    s_b = float(np.median(times))
    out = {
        "metric": METRIC, "value": flops / s_b / 1e9, "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": s_b * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8+f32+f64" if form == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "instances": count, "eps": eps, "leaf_size": 64,
                   "form": form, "surfaces": "sphere / rotated ellipsoid / cube surface",
                   "kappa": "sqrt(n)/5.66"},
        "batch_s": s_b, "sequential_s": seq[0], "batch_speedup": seq[0] / s_b,
        "host_plan_s": t_plan,
    }
    print(json.dumps(out), flush=True)


def run_matvec(args, dh2, torch, synth, blocks, w, eps, leaf, kappa, n, form):
    """Matvec timing: one compression (untimed), then y = G~x and y = G~^*x on
    one right-hand side, each timed over `steps` products after `warmup`.  The
    representation (bases, transfer matrices, coupling matrices, near field)
    is read once per product: its size over the product time is the HBM rate."""
    prec = dh2.FP64 if form == "fp64" else dh2.MIXED
    o = dh2.opts(leaf_size=leaf, precision=prec, groups=args.groups)
    m = dh2.compress_helmholtz(blocks, w, eps, o)
    torch.cuda.synchronize()
    st = dh2.stats(m)
    rep_bytes = st["mem_bytes"]
    x = torch.from_numpy(synth.complex_gaussian(n, 6)).to("cuda")
    y = torch.empty_like(x)
    ms = {}
    for op in ("N", "C"):
        for _ in range(args.warmup):
            dh2.matvec(m, op, x, y)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(args.steps):
            dh2.matvec(m, op, x, y)
        ev1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps * 1e3
        ms[op] = ev0.elapsed_time(ev1) / args.steps
        log(f"[bench] matvec {op}: {ms[op]:.3f} ms per product (wall {wall:.3f} ms), "
            f"representation {rep_bytes / 1e9:.2f} GB")
    ach = rep_bytes / (ms["N"] * 1e-3) / 1e9
    out = {
        "metric": "matvec ms, y = G~x with the compressed representation, n=%d kappa=%g" % (n, kappa),
        "value": ms["N"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms["N"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "kappa": kappa, "leaf_size": leaf,
                   "eps": eps, "form": form, "nrhs": 1},
        "roofline": {"bound": "hbm", "kernel": "matvec (representation read once per product)",
                     "achieved": ach, "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                     "traffic": None},
        "adjoint_ms": ms["C"],
        "representation_bytes": rep_bytes,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere131072")
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--groups", type=int, default=0)
    ap.add_argument("--err-iters", type=int, default=8)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", type=float, default=None,
                    help="HBM bytes per launch of the roofline kernel from the counter runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy first (counter scale calibration)")
    ap.add_argument("--mode", choices=("compress", "matvec"), default="compress",
                    help="compress (default): the compression step; matvec: y = G~x and "
                         "y = G~^*x with the compressed representation of the first form")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1510_07087_amd import dh2

    dh2.lib()
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
        del src, dst
    if args.workload.startswith("batch"):
        run_batch(args, dh2, torch, synth)
        return
    p, w, kappa, leaf, eps = synth.workload(args.workload)
    n = len(p)
    log(f"[bench] workload {args.workload}: n={n} kappa={kappa} leaf={leaf} eps={eps}")
    o = dh2.opts(leaf_size=leaf)
    t0 = time.perf_counter()
    tree = dh2.tree_build(p, kappa, o)
    blocks = dh2.blocks_build(tree, o)
    t_plan = time.perf_counter() - t0
    binfo = dh2.blocks_info(blocks)
    log(f"[bench] host plan {t_plan:.2f} s: {binfo}")

    forms = [f for f in args.forms.split(",") if f]
    if args.mode == "matvec":
        run_matvec(args, dh2, torch, synth, blocks, w, eps, leaf, kappa, n, forms[0])
        return
    res = {}
    for form in forms:
        m, st, times = run_form(dh2, torch, blocks, w, eps, leaf, form, args.steps, args.warmup,
                                args.groups)
        rows = np.random.default_rng(5).choice(n, 16, replace=False)
        x = torch.from_numpy(synth.complex_gaussian(n, 6)).to("cuda")
        _, _, rows_rel = dh2.rows_check(m, rows, x)
        err = dh2.error_estimate(m, None, iters=args.err_iters, seed=1) if args.err_iters > 0 \
            else None
        s = float(np.median(times))
        flops = st["flops_row"] + st["flops_col"] + st["flops_prj"]
        res[form] = dict(s=s, gflops=flops / s / 1e9, stats=st, rows_rel=rows_rel, rel_err=err)
        log(f"[bench] {form}: {s:.3f} s, {flops / s / 1e9:.1f} GFLOP/s, rows {rows_rel:.2e}, "
            f"err {err}")
        log(f"[bench] {form} flops: gram leaf {st['flops_gram_leaf']:.4e} "
            f"inner {st['flops_gram'] - st['flops_gram_leaf']:.4e}; rprod leaf "
            f"{st['flops_rprod_leaf']:.4e} inner {st['flops_rprod'] - st['flops_rprod_leaf']:.4e}; "
            f"projection {st['flops_prj']:.4e}")
        del m
    head = "mixed" if "mixed" in res else forms[0]
    r = res[head]
    st = r["stats"]
    nl = max(1, st["n_gram_leaf"])
    traffic = args.traffic
    if head == "mixed":
        # dominant kernel: the int8-sliced leaf Gram (k_gram_i8<0>)
        kern = "k_gram_i8<0> (leaf Gram matrices, exact int8 slices on int8 MFMA)"
        work, peak, unit = st["ops_gram_leaf_i8"], PEAK_INT8_MFMA, "TOP/s"
        if traffic is None and args.workload == "sphere131072":
            traffic = TRAFFIC_GRAM_I8_LEAF
    else:
        kern = "k_gram_leaf_w (leaf Gram matrices on FP64 MFMA)"
        work, peak, unit = st["flops_gram_leaf"], PEAK_FP64_MFMA, "TFLOP/s"
    achieved = work / st["t_gram_leaf"] if st["t_gram_leaf"] > 0 else 0.0
    pk_prj = PEAK_FP32_MFMA if head == "mixed" else PEAK_FP64_MFMA
    # the stacked projection also against HBM: counter bytes per compression
    prj_hbm = {}
    if head == "mixed" and args.workload == "sphere131072" and st["t_prj"] > 0:
        gbs = TRAFFIC_PROJECTION_STACKED / st["t_prj"] / 1e9
        prj_hbm = {"traffic": TRAFFIC_PROJECTION_STACKED, "hbm_achieved_GBps": gbs,
                   "hbm_frac": gbs / 8000.0}
    ach_prj = st["flops_prj"] / st["t_prj"] if st["t_prj"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": r["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "i8+f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "kappa": kappa, "leaf_size": leaf,
                   "eps": eps, "eta1": 20.0, "eta2": 5.0, "zeta": 2.0 / 3.0, "form": head,
                   "entries": "generated on the fly"},
        "roofline": {"bound": "mfma", "kernel": kern,
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic,
                     "launches": st["n_gram_leaf"],
                     "avg_launch_ms": st["t_gram_leaf"] / nl * 1e3,
                     "work_per_launch": work / nl},
        "roofline_projection": {"bound": "mfma",
                                "kernel": ("k_project_stacked (S_b = omega_b R|s W, stacked "
                                           "by W, FP32 4x4x1 MFMA)" if head == "mixed" else
                                           "k_project_tiled (S_b = omega_b R|s W, FP64 MFMA)"),
                                "achieved": ach_prj / 1e12, "peak": pk_prj / 1e12,
                                "unit": "TFLOP/s", "frac": ach_prj / pk_prj,
                                **prj_hbm},
        "compression_s": {f: res[f]["s"] for f in res},
        "gflops": {f: res[f]["gflops"] for f in res},
        "rel_err_2": {f: res[f]["rel_err"] for f in res},
        "rows_check_max_rel": {f: res[f]["rows_rel"] for f in res},
        "phases_s": {f: {k: res[f]["stats"][k] for k in ("t_row", "t_col", "t_prj", "t_near")}
                     for f in res},
        "k_max": st["k_max"],
        "mem_per_n_kib": st["mem_per_n_kib"],
        "host_plan_s": t_plan,
    }
    if "mixed" in res and "fp64" in res:
        out["speedup_mixed_vs_fp64"] = res["fp64"]["s"] / res["mixed"]["s"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, w, kappa, leaf, eps, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
