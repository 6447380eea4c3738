"""Benchmark: directional H2 compression on one MI355X.

A step is one full compression (both bases, transfer matrices, projection of
every admissible block, near field) of a synthetic workload whose points are
already on the device side of the call.  The default workload is the
131072-point golden-spiral sphere, kappa = 64, leaf size 64, eps = 1e-4,
eta1 = 20, eta2 = 5, entries generated on the fly.

Prints ONE JSON line: metric/value/unit (GFLOP/s = algorithmic flops of the
compression -- 8 r^2 N per block row for the reduction, 8 k r N for the
R-products, 8 k_t k_s #s per block for the projection -- over its seconds),
the roofline of the dominant kernel (the leaf Gram kernel) and of the
projection, with the counter figures of the committed profile when the
kernels are the ones it was taken on, and the CPU baseline (the FP64 oracle
timed per phase on smaller spheres, with the benchmark size extrapolated).
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
PEAK_HBM = 8.0e12
# VALU issue ceiling: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every
# 4 cycles at 2.4 GHz (16 lanes per SIMD and cycle)
PEAK_VALU_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1510_07087_amd", "csrc", f)
                  for f in ("kernels.hip", "common.hpp")]


def sources_sha():
    """First 16 hex digits of the SHA-256 of the kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def profile_figures(name):
    """Counter figures of a committed profile summary (profiles/<name>.md):
    its 'figures' block holds one 'key value' per line, e.g. the HBM bytes
    per dispatch of a kernel.  Returns {} when the file is missing or when the
    kernel sources changed since the counters were taken (the block records
    their hash), since the figures then describe other code."""
    path = os.path.join(PROFILES, name + ".md")
    if not os.path.exists(path):
        return {}
    txt = open(path).read()
    if "```figures" not in txt:
        return {}
    block = txt.split("```figures", 1)[1].split("```", 1)[0]
    fig = {}
    for line in block.strip().splitlines():
        k, v = line.split(None, 1)
        fig[k] = v.strip()
    if fig.get("sources_sha256_16") != sources_sha():
        return {}
    return fig


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(dh2, torch, blocks, w, eps, leaf, form, steps, warmup, groups, normals=None,
             cap=0):
    prec = dh2.FP64 if form == "fp64" else dh2.MIXED
    o = dh2.opts(leaf_size=leaf, precision=prec, groups=groups, max_device_bytes=cap)
    times, st, m = [], None, None
    for it in range(warmup + steps):
        m = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if normals is None:
            m = dh2.compress_helmholtz(blocks, w, eps, o)
        else:
            m = dh2.compress_helmholtz_dlp(blocks, w, normals, eps, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = dh2.stats(m)
        log(f"[bench] {form} step {it} {'warmup' if it < warmup else 'timed'}: {dt:.3f} s "
            f"(device {st['t_total']:.3f} s, gram {st['t_gram_kernel']:.3f} s, "
            f"k_max {st['k_max']}, groups {st['groups']})")
        if it >= warmup:
            times.append(dt)
    return m, st, times


def _oracle_flops(plan, cp):
    """Algorithmic real flops of a compression from the oracle's ranks, with
    the counts of the hot-path table: per (t,c) of both bases 8 r^2 N for the
    reduction and 8 k r N for R = Q^* A (r = #t for leaves, k1 + k2 above;
    N = #F_tc), per admissible block 8 k_t k_s #s for the projection."""
    tr, dr, bt = plan.tree, plan.dirs, plan.blocks
    fl = 0.0
    for basis, sets in ((cp.V, plan.rowsets), (cp.W, plan.colsets)):
        for (t, c), k in basis.k.items():
            N = float(sum(int(tr.size[s]) for (_, s, _) in sets.F[t][c]))
            if tr.son1[t] < 0:
                r = int(tr.size[t])
            else:
                cp_ = int(dr.sd[tr.level[t]][c])
                r = sum(basis.k[(ts, cp_)] for ts in tr.sons(t))
            fl += 8.0 * r * r * N + 8.0 * k * r * N
    for b in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        fl += 8.0 * cp.V.k[(t, c)] * cp.W.k[(s, c)] * int(tr.size[s])
    return fl


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s, k_target, n_target):
    """The FP64 oracle (NumPy/LAPACK, plan + weights + row basis + column basis
    + projection + near field, exactly as the parity tests run it) timed per
    phase on this host's cores: the 2048-point sphere (kappa 8, leaf 32, the
    smallest workload) and, within the time budget, the 4608-point
    and 8192-point spheres (kappa sqrt(n)/5.66, leaf 64, the leaf size of the
    benchmark workload).
    The benchmark workload itself would take hours; its oracle time is
    extrapolated from the larger timed run by keeping time / (n^2 k_max)
    constant, as the paper observes for its own timings."""
    from threadpoolctl import threadpool_info

    import synth
    from oracle import compress as OC
    from oracle import dh2 as OD
    from oracle import matrix as OM
    from oracle import plan as OP

    runs, last = {}, None
    spent = 0.0
    for name in ("sphere2048", "sphere4608", "sphere8192"):
        # the next sphere takes about four times the last one
        if runs and spent + 4.0 * runs[last]["t_total"] > budget_s:
            break
        p, w, kappa, leaf, eps = synth.workload(name)
        t0 = time.perf_counter()
        plan = OP.build_plan(p, kappa, leaf)
        t1 = time.perf_counter()
        M = OM.HelmholtzMatrix(p, w, kappa, plan.tree.perm)
        omega = OC.block_weights(M, plan)
        t2 = time.perf_counter()
        V = OC.build_basis(M, plan, plan.rowsets, omega, eps, 2.0 / 3.0)
        t3 = time.perf_counter()
        W = OC.build_basis(OM.AdjointMatrix(M), plan, plan.colsets, omega, eps, 2.0 / 3.0)
        t4 = time.perf_counter()
        tr, bt = plan.tree, plan.blocks
        S = [V.Qexp[(int(t), int(c))].conj().T @ M.block(tr.rows(t), tr.rows(s_))
             @ W.Qexp[(int(s_), int(c))] for t, s_, c in zip(bt.adm_t, bt.adm_s, bt.adm_c)]
        near = [M.block(tr.rows(t), tr.rows(s_)) for t, s_ in zip(bt.near_t, bt.near_s)]
        t5 = time.perf_counter()
        cp = OC.Compressed(plan, eps, 2.0 / 3.0, omega, V, W, S, near)
        fl = _oracle_flops(plan, cp)
        sto = OD.storage_stats(cp)
        tot = t5 - t1
        spent += t5 - t0
        runs[name] = dict(n=len(p), kappa=kappa, leaf=leaf, eps=eps, t_plan=t1 - t0,
                          t_weights=t2 - t1, t_row=t3 - t2, t_col=t4 - t3, t_prj=t5 - t4,
                          t_total=tot, flops=fl, gflops=fl / tot / 1e9, k_max=sto["k_max"],
                          mem_per_n_kib=sto["mem_per_n_kib"])
        last = name
        log(f"[bench] oracle {name}: {runs[name]}")
    threads = max([q.get("num_threads", 1) for q in threadpool_info()] + [1])
    L = runs[last]
    t_extra = L["t_total"] * (n_target / L["n"]) ** 2 * (k_target / max(1, L["k_max"]))
    return {"value": L["gflops"], "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"whole oracle compressions of {', '.join(runs)} (per-phase times below); "
                      f"value = algorithmic flops / oracle seconds of {last}",
            "host_cpus": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model(),
            "blas_threads": int(threads), "runs": runs,
            "extrapolated_s_benchmark_workload": t_extra,
            "extrapolation": f"oracle seconds at n={n_target}, k_max={k_target} from {last} "
                             f"with time / (n^2 k_max) held constant (not measured)"}


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
        gl_flops = sum(x["flops_gram_leaf"] for x in st)
        gl_time = sum(x["t_gram_leaf"] for x in st)
        gl_n = sum(x["n_gram_leaf"] for x in st)
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
        # leaf Gram kernels of all instances (the largest kernel of each):
        # algorithmic 8 r^2 N flops over their event-timed launch durations on
        # the instances' streams; launches of concurrent instances share the
        # device, so this is a lower bound of the kernel's own rate
        "roofline": {"bound": "mfma",
                     "kernel": ("k_gram_i8<0> (leaf Gram matrices, exact int8 slices on int8 "
                                "MFMA), all instances" if form == "mixed" else
                                "k_gram_leaf_w (leaf Gram matrices on FP64 MFMA), all instances"),
                     "achieved": gl_flops / gl_time / 1e12 if gl_time > 0 else 0.0,
                     "peak": (PEAK_INT8_MFMA if form == "mixed" else PEAK_FP64_MFMA) / 1e12,
                     "unit": "TOP/s" if form == "mixed" else "TFLOP/s",
                     "frac": (gl_flops / gl_time / (PEAK_INT8_MFMA if form == "mixed"
                                                     else PEAK_FP64_MFMA)) if gl_time > 0 else 0.0,
                     "traffic": None, "launches": gl_n,
                     "avg_launch_ms": gl_time / max(1, gl_n) * 1e3,
                     "work_per_launch": gl_flops / max(1, gl_n),
                     "work": "8 r^2 N real flops per leaf block row (r = #t, N = #F_tc)"},
    }
    print(json.dumps(out), flush=True)


def run_matvec(args, dh2, torch, synth, blocks, w, eps, leaf, kappa, n, form):
    """Matvec timing: one compression (untimed), then y = G~x and y = G~^*x,
    each timed over `steps` calls after `warmup`, with one right-hand side
    and with eight (one pass of the kernels, which read the representation
    once for all eight).  The representation (bases, transfer matrices,
    coupling matrices, near field) is read once per pass: its size over the
    pass time is the HBM rate."""
    prec = dh2.FP64 if form == "fp64" else dh2.MIXED
    o = dh2.opts(leaf_size=leaf, precision=prec, groups=args.groups)
    m = dh2.compress_helmholtz(blocks, w, eps, o)
    torch.cuda.synchronize()
    st = dh2.stats(m)
    rep_bytes = st["repr_bytes"]   # as stored: S_b and near field in FP32 in the mixed form
    ms = {}
    for nrhs in (1, 8):
        xn = synth.complex_gaussian(n, 6, nrhs if nrhs > 1 else None)
        x = (torch.from_numpy(xn).to("cuda") if nrhs == 1 else
             torch.from_numpy(np.ascontiguousarray(xn.T)).to("cuda").T)
        y = torch.empty_like(x)
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
            ms[(op, nrhs)] = ev0.elapsed_time(ev1) / args.steps
            log(f"[bench] matvec {op} nrhs {nrhs}: {ms[(op, nrhs)]:.3f} ms per call "
                f"({ms[(op, nrhs)] / nrhs:.3f} ms per right-hand side, wall {wall:.3f} ms), "
                f"representation {rep_bytes / 1e9:.2f} GB")
    ach = rep_bytes / (ms[("N", 1)] * 1e-3) / 1e9
    # counter bytes of one pass from the committed profile of this workload
    # (none when the kernel sources changed since the counters were taken)
    fig = profile_figures(f"matvec_{args.workload}")
    traffic = float(fig["matvec_hbm_bytes_per_pass_nrhs1"]) if fig else None
    out = {
        "metric": "matvec ms, y = G~x with the compressed representation, n=%d kappa=%g" % (n, kappa),
        "value": ms[("N", 1)], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms[("N", 1)], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "kappa": kappa, "leaf_size": leaf,
                   "eps": eps, "form": form, "nrhs": 1},
        "roofline": {"bound": "hbm", "kernel": "matvec (representation read once per pass)",
                     "achieved": ach, "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                     "traffic": traffic,
                     **({"profile": f"profiles/matvec_{args.workload}.md"} if fig else {})},
        "adjoint_ms": ms[("C", 1)],
        "nrhs8_ms_per_rhs": {"N": ms[("N", 8)] / 8, "C": ms[("C", 8)] / 8},
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
    ap.add_argument("--err-iters", type=int, default=50,
                    help="power iterations of the error estimate (it also stops once the "
                         "Rayleigh quotient changes by less than 1e-4)")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", type=float, default=None,
                    help="HBM bytes per launch of the roofline kernel from the counter runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy first (counter scale calibration)")
    ap.add_argument("--source", choices=("slp", "dlp"), default="slp",
                    help="slp (default): the single-layer matrix of the workload; dlp: the "
                         "double-layer matrix on the same points (sphere and ellipsoid "
                         "workloads), timed as a separate line")
    ap.add_argument("--sequential", action="store_true",
                    help="profiling aid: a device-memory cap equal to the device's memory, "
                         "which makes the row and column sweeps run one after the other, so "
                         "that each kernel's duration is its own (not a bench line)")
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
    normals = None
    if args.source == "dlp":
        if args.workload.startswith("sphere"):
            normals = synth.sphere_normals(p)
        elif args.workload.startswith("ellip"):
            normals = synth.ellipsoid_normals(n)
        else:
            raise SystemExit("--source dlp needs a sphere or ellipsoid workload")
    res = {}
    cap = torch.cuda.get_device_properties(0).total_memory if args.sequential else 0
    for form in forms:
        m, st, times = run_form(dh2, torch, blocks, w, eps, leaf, form, args.steps, args.warmup,
                                args.groups, normals, cap)
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
    # counter figures of the committed profile of this workload and form
    # (empty when the kernels changed since they were taken)
    dlp = args.source == "dlp"
    fig = {} if dlp else profile_figures(f"compress_{args.workload}_{head}")
    if head == "mixed" and dlp:
        kern = "k_gram_i8<2> (double-layer leaf Gram matrices, exact int8 slices on int8 MFMA)"
        peak, unit, key = PEAK_INT8_MFMA, "TOP/s", "k_gram_i8_2"
        extra = {"int8_ops_per_flop": st["ops_gram_leaf_i8"] / max(1.0, st["flops_gram_leaf"])}
    elif head == "mixed":
        # dominant kernel: the int8-sliced leaf Gram (k_gram_i8<0>); its work is
        # the reduction's algorithmic 8 r^2 N real flops, against the peak of the
        # MFMA it runs on (int8); the emulation's own int8 operations per flop
        # are reported beside it
        kern = "k_gram_i8<0> (leaf Gram matrices, exact int8 slices on int8 MFMA)"
        peak, unit, key = PEAK_INT8_MFMA, "TOP/s", "k_gram_i8_0"
        extra = {"int8_ops_per_flop": st["ops_gram_leaf_i8"] / max(1.0, st["flops_gram_leaf"])}
    else:
        kern = "k_gram_leaf_w (leaf Gram matrices on FP64 MFMA)"
        peak, unit, key = PEAK_FP64_MFMA, "TFLOP/s", "k_gram_leaf_w"
        extra = {}
    work = st["flops_gram_leaf"]
    achieved = work / st["t_gram_leaf"] if st["t_gram_leaf"] > 0 else 0.0
    traffic = args.traffic
    if traffic is None and f"{key}_hbm_bytes_per_dispatch" in fig:
        traffic = float(fig[f"{key}_hbm_bytes_per_dispatch"])
    if f"{key}_valu_insts_per_compression" in fig and st["t_gram_leaf"] > 0:
        # VALU view of the same launches: wave instructions issued (counter run)
        # over this run's event-timed durations, against the issue ceiling
        extra["valu_issue_frac"] = (float(fig[f"{key}_valu_insts_per_compression"]) /
                                    st["t_gram_leaf"] / PEAK_VALU_WAVE_INSTS)
    if fig:
        extra["profile"] = f"profiles/compress_{args.workload}_{head}.md"
    pk_prj = PEAK_FP32_MFMA if head == "mixed" else PEAK_FP64_MFMA
    # the stacked projection also against HBM: counter bytes per compression
    prj_hbm = {}
    if "project_hbm_bytes_per_compression" in fig and st["t_prj"] > 0:
        pb = float(fig["project_hbm_bytes_per_compression"])
        prj_hbm = {"traffic": pb, "hbm_achieved_GBps": pb / st["t_prj"] / 1e9,
                   "hbm_frac": pb / st["t_prj"] / PEAK_HBM}
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
                   "matrix": "double layer" if dlp else "single layer",
                   "entries": "generated on the fly",
                   "sweeps": "sequential (profiling aid)" if args.sequential else "concurrent"},
        "roofline": {"bound": "mfma", "kernel": kern,
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic,
                     "launches": st["n_gram_leaf"],
                     "avg_launch_ms": st["t_gram_leaf"] / nl * 1e3,
                     "work_per_launch": work / nl,
                     "work": "8 r^2 N real flops per leaf block row (r = #t, N = #F_tc)",
                     **extra},
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
    if not args.no_cpu_baseline and not dlp:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget, st["k_max"], n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
