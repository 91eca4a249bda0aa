"""Benchmark of the FP64 GEMM hot path on one MI355X.

A step is one pass over the three FP64 shapes of the headline workload:
square m=n=k=16384, large-k m=n=2048 k=2^20 (split-K + reduction) and flat
m=n=32768 k=256, C = A*B with uniform[-1,1] inputs already resident in HBM.
`value` is the whole step's useful flops (2mnk per product) over its time.

Printed: one JSON line with the driver's keys plus
  roofline      the dominant kernel (the square product's GEMM launch) from
                HIP events on the launch stream, against the FP64 MFMA peak;
                `traffic` is the HBM bytes per launch from the committed
                rocprofv3 counter summary when it matches the current kernel
                source, else null
  config_512    the small FP64 product 512^3 (launch-bound), timed
  cpu_baseline  the oracle timed on the host cores: `value` on a bounded
                sample (rows of the square product), plus the 512^3 product
                and the 512-problem batch in full; every GPU result it
                covers is compared with it
  variants      the precision and batching variants (BF16x3 vs FP32, Ozaki
                INT8 vs FP64, batched vs single launches), each timed on its
                own workload

Timing: `--warmup` untimed steps (default 3), then `--steps` timed steps
(default 20) with HIP events around every launch; each shape and variant
reports its median with a distribution-free 95 % confidence interval
(order statistics), the roofline uses the average launch duration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GEMM TFLOP/s & %peak at stated error vs FP64; HBM bytes vs I/O lower bound"
PEAK_F64 = 78.6    # TFLOP/s, FP64 MFMA
PEAK_F32 = 157.3   # TFLOP/s, FP32 MFMA
PEAK_BF16 = 2500.0
PEAK_I8 = 5000.0
SHAPES = [("square", 16384, 16384, 16384), ("large_k", 2048, 2048, 1 << 20),
          ("flat", 32768, 32768, 256)]
SEED = 1


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of what decides the FP64 square launch's memory traffic: the
    kernel source, its launch interface and the work-item raster.  The plan
    (tile, group_m) is pinned separately by the record's kernel tag."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1908_09606_amd", "csrc")
    for name in ("gemm_f64.hip", "kernels.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(csrc, "tiles.hpp"), "rb") as f:
        tiles = f.read()
    h.update(tiles[tiles.index(b"// Workgroups are handed to the XCDs"):])
    return h.hexdigest()[:16]


def committed_traffic(kernel_tag: str):
    """HBM bytes per launch from profiles/traffic_*.json, if taken on the
    current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_gemm_f64_square_16384.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("kernel") != kernel_tag:
        return None
    return rec.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=20,
                    help="timed repetitions of each variant (after min(3, reps) warm-ups)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--shapes", default="square,large_k,flat")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark step: FP64 shapes across the planner's "
                         "regimes and the three tile sizes of one shape (one JSON line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run one plain copy kernel (out = in * 1.0 over float64) "
                         "moving BYTES each way, to calibrate memory counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "runs each product on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1908_09606_amd as cm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.sweep:
        print(json.dumps({"sweep": run_sweep(torch, cm, synth, dev, stream, args.reps)}),
              flush=True)
        return
    wanted = args.shapes.split(",")
    shapes = [s for s in SHAPES if s[0] in wanted]

    # ---- inputs resident in HBM, plans, workspace
    probs = []
    ws_need = 0
    for name, m, n, k in shapes:
        A = torch.empty((m, k), dtype=torch.float64, device=dev)
        B = torch.empty((k, n), dtype=torch.float64, device=dev)
        C = torch.empty((m, n), dtype=torch.float64, device=dev)
        synth.fill_device(A, SEED, synth.STREAM_A, synth.UNIFORM_F64)
        synth.fill_device(B, SEED, synth.STREAM_B, synth.UNIFORM_F64)
        rc, plan = cm.cosma_plan_query(m, n, k, cm.COSMA_F64)
        cm.check(rc, "plan")
        ws_need = max(ws_need, plan.workspace_bytes)
        probs.append(dict(name=name, m=m, n=n, k=k, A=A, B=B, C=C, plan=plan))
    cm.ensure_workspace(ws_need)
    torch.cuda.synchronize()

    def launch(p):
        rc = cm.cosma_gemm(p["m"], p["n"], p["k"], 1.0, p["A"], p["k"], p["B"], p["n"], 0.0,
                           p["C"], p["n"], cm.COSMA_F64, stream)
        cm.check(rc, "cosma_gemm")

    for _ in range(args.warmup):
        for p in probs:
            launch(p)
    torch.cuda.synchronize()

    # ---- timed region: events around every launch on the launch stream
    events = {p["name"]: [] for p in probs}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for p in probs:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            launch(p)
            e1.record(stream)
            events[p["name"]].append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    step_flops = sum(2.0 * p["m"] * p["n"] * p["k"] for p in probs)
    value = step_flops * args.steps / wall / 1e12
    shape_rows = []
    for p in probs:
        ms = [a.elapsed_time(b) for a, b in events[p["name"]]]
        avg = sum(ms) / len(ms)
        tf = 2.0 * p["m"] * p["n"] * p["k"] / (avg * 1e-3) / 1e12
        st = timing_stats(ms)
        pl = p["plan"]
        shape_rows.append(dict(
            shape=p["name"], m=p["m"], n=p["n"], k=p["k"], ms_avg=round(avg, 4),
            ms_min=round(min(ms), 4), ms_median=st["median"], ms_ci95=st["ci95"],
            tflops=round(tf, 3), frac_peak=round(tf / PEAK_F64, 4),
            tile=f"{pl.tile_m}x{pl.tile_n}x{pl.tile_k}", p_k=pl.p_k, group_m=pl.group_m,
            planner_q_ea_bytes=pl.q_ea_bytes, planner_q_cu_words=pl.q_cu_words,
            thm1_words=pl.thm1_words, q_cu_over_thm1=round(pl.q_cu_words / pl.thm1_words, 4)))

    # dominant kernel: the square product's GEMM launch (one kernel per call)
    dom = next((r for r in shape_rows if r["shape"] == "square"), shape_rows[0])
    dom_plan = next(p["plan"] for p in probs if p["name"] == dom["shape"])
    kernel_tag = (f"gemm_f64<{dom_plan.tile_m}x{dom_plan.tile_n}x{dom_plan.tile_k}> "
                  f"group_m={dom_plan.group_m}")
    achieved = 2.0 * dom["m"] * dom["n"] * dom["k"] / (dom["ms_avg"] * 1e-3) / 1e12
    traffic = committed_traffic(kernel_tag)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_F64,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64, 4),
                "traffic": traffic, "kernel": kernel_tag,
                "launch": f"{dom['shape']} {dom['m']}x{dom['n']}x{dom['k']}",
                "planner_q_ea_bytes": dom["planner_q_ea_bytes"],
                "traffic_over_q_ea": (round(traffic / dom["planner_q_ea_bytes"], 3)
                                      if traffic else None)}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "FP64 GEMM C=A*B row-major, uniform[-1,1] seeded: "
                               + ", ".join(f"{p['name']} {p['m']}x{p['n']}x{p['k']}" for p in probs),
                   "alpha": 1.0, "beta": 0.0, "seed": SEED},
        "roofline": roofline,
        "shapes": shape_rows,
    }
    # The paper's own figures, measured on a CPU cluster: context, not a
    # baseline for this metric (hence vs_baseline is null).
    sq = next((r for r in shape_rows if r["shape"] == "square"), None)
    out["paper_context"] = {
        "machine": "Piz Daint XC40 CPU partition (2 x 18-core Xeon E5-2695 v4 per node)",
        "best_fraction_of_machine_peak": 0.88,
        "square_16384_ms_on_9216_cores": 142.0,
        "square_16384_ms_here": sq["ms_median"] if sq else None,
    }

    if args.copy_calibration > 0:
        nel = args.copy_calibration // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nel * 8
        del src, dst

    keep = []
    small = run_small(torch, cm, synth, dev, stream, args.reps)
    out["config_512"] = {k_: v for k_, v in small.items() if k_ != "C"}
    if not args.no_variants:
        out["variants"] = run_variants(torch, cm, synth, dev, stream, keep, args.reps)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs, small, keep, torch)
        out["accuracy"] = sampled_accuracy(probs, keep)

    # release inputs before printing
    for p in probs:
        p.clear()
    print(json.dumps(out), flush=True)


def timing_stats(ms):
    """Median of the samples with a distribution-free 95 % confidence
    interval: order statistics x_(j) .. x_(n+1-j), j the largest index with
    P(Bin(n, 1/2) <= j - 1) <= 0.025 (the whole range when n < 6)."""
    xs = sorted(ms)
    n = len(xs)
    cdf, j = 0.0, 0
    while j < n:
        p = math.comb(n, j) / 2.0 ** n
        if cdf + p > 0.025:
            break
        cdf += p
        j += 1
    j = max(j, 1)
    med = xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])
    return {"median": round(med, 4), "ci95": [round(xs[j - 1], 4), round(xs[n - j], 4)], "n": n}


def _time(torch, stream, fn, reps=20, warm=3):
    """Median time of fn (HIP events on `stream`, one synchronisation per
    repetition) after `warm` untimed calls; returns (median_ms, stats)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    st = timing_stats(ts)
    return st["median"], st


def run_variants(torch, cm, synth, dev, stream, keep, reps=20):
    """Precision and batching variants, each on its own workload:
    BF16x3 vs native FP32 (16384^3 and 4096^2 x 2^18, uniform FP32),
    Ozaki INT8 slices, Ozaki II and Ozaki bf16 slices vs native FP64 (8192^3,
    sign*U[1,2)*2^e, e in [-20,20]),
    512 uneven FP32 products: one graph launch vs 512 single launches.
    Results needed for the accuracy check are appended to `keep`."""
    out = {}
    rows = []
    for (m, n, k) in ((16384, 16384, 16384), (4096, 4096, 1 << 18)):
        A = torch.empty((m, k), dtype=torch.float32, device=dev)
        B = torch.empty((k, n), dtype=torch.float32, device=dev)
        synth.fill_device(A, SEED, synth.STREAM_A, synth.UNIFORM_F32)
        synth.fill_device(B, SEED, synth.STREAM_B, synth.UNIFORM_F32)
        res = {}
        for dt in ("f32", "bf16x3"):
            C = torch.empty((m, n), dtype=torch.float32, device=dev)
            rc, plan = cm.cosma_plan_query(m, n, k, dt)
            cm.ensure_workspace(plan.workspace_bytes)
            ms, st = _time(torch, stream, lambda: cm.gemm(A, B, C, dtype=dt, stream=stream),
                           reps, min(3, reps))
            res[dt] = (ms, 2.0 * m * n * k / (ms * 1e-3) / 1e12, plan, st["ci95"])
            keep.append((f"{dt} {m}x{n}x{k}", C, m, n, k, synth.UNIFORM_F32, "f32"))
        f32, x3 = res["f32"], res["bf16x3"]
        rows.append({"shape": f"{m}x{n}x{k}", "f32_ms": round(f32[0], 3), "f32_ms_ci95": f32[3],
                     "f32_tflops": round(f32[1], 2), "f32_frac_peak": round(f32[1] / PEAK_F32, 4),
                     "f32_tile": f"{f32[2].tile_m}x{f32[2].tile_n}", "f32_p_k": f32[2].p_k,
                     "bf16x3_ms": round(x3[0], 3), "bf16x3_ms_ci95": x3[3],
                     "bf16x3_tflops": round(x3[1], 2),
                     "bf16x3_frac_bf16_peak": round(3 * x3[1] / PEAK_BF16, 4),
                     "bf16x3_tile": f"{x3[2].tile_m}x{x3[2].tile_n}",
                     "speedup_vs_f32": round(f32[0] / x3[0], 3)})
        del A, B
    out["bf16x3_vs_f32"] = rows

    m = n = k = 8192
    A = torch.empty((m, k), dtype=torch.float64, device=dev)
    B = torch.empty((k, n), dtype=torch.float64, device=dev)
    synth.fill_device(A, SEED, synth.STREAM_A, synth.WIDE_F64)
    synth.fill_device(B, SEED, synth.STREAM_B, synth.WIDE_F64)
    res = {}
    for dt in ("f64", "ozaki", "ozaki2", "ozaki_bf16"):
        C = torch.empty((m, n), dtype=torch.float64, device=dev)
        rc, plan = cm.cosma_plan_query(m, n, k, dt)
        cm.ensure_workspace(plan.workspace_bytes)
        ms, st = _time(torch, stream, lambda: cm.gemm(A, B, C, dtype=dt, stream=stream),
                           reps, min(3, reps))
        res[dt] = (ms, 2.0 * m * n * k / (ms * 1e-3) / 1e12, plan, st["ci95"])
        keep.append((f"{dt} {m}^3 wide", C, m, n, k, synth.WIDE_F64, "f64"))
    s_ = res["ozaki"][2].slices
    out["ozaki_vs_f64"] = {
        "shape": "8192^3, sign*U[1,2)*2^e, e in [-20,20]", "slices": s_,
        "int8_products": s_ * (s_ + 1) // 2,
        "f64_ms": round(res["f64"][0], 3), "f64_ms_ci95": res["f64"][3],
        "f64_tflops": round(res["f64"][1], 2),
        "ozaki_ms": round(res["ozaki"][0], 3), "ozaki_ms_ci95": res["ozaki"][3],
        "ozaki_tflops": round(res["ozaki"][1], 2),
        "ozaki_frac_int8_peak": round(res["ozaki"][1] * s_ * (s_ + 1) / 2 / PEAK_I8, 4),
        "speedup_vs_f64": round(res["f64"][0] / res["ozaki"][0], 3)}
    nm = res["ozaki2"][2].slices
    out["ozaki2_vs_f64"] = {
        "shape": "8192^3, sign*U[1,2)*2^e, e in [-20,20]", "moduli": nm,
        "beta": cm.cosma_ozaki2_params(k, nm)[1], "int8_products": nm,
        "f64_ms": round(res["f64"][0], 3),
        "ozaki2_ms": round(res["ozaki2"][0], 3), "ozaki2_ms_ci95": res["ozaki2"][3],
        "ozaki2_tflops": round(res["ozaki2"][1], 2),
        "ozaki2_frac_int8_peak": round(res["ozaki2"][1] * nm / PEAK_I8, 4),
        "speedup_vs_f64": round(res["f64"][0] / res["ozaki2"][0], 3),
        "speedup_vs_ozaki": round(res["ozaki"][0] / res["ozaki2"][0], 3)}
    sb = res["ozaki_bf16"][2].slices
    out["ozaki_bf16_vs_f64"] = {
        "shape": "8192^3, sign*U[1,2)*2^e, e in [-20,20]", "slices": sb,
        "bf16_products": sb * (sb + 1) // 2,
        "f64_ms": round(res["f64"][0], 3),
        "ozaki_bf16_ms": round(res["ozaki_bf16"][0], 3),
        "ozaki_bf16_ms_ci95": res["ozaki_bf16"][3],
        "ozaki_bf16_tflops": round(res["ozaki_bf16"][1], 2),
        "ozaki_bf16_frac_bf16_peak": round(res["ozaki_bf16"][1] * sb * (sb + 1) / 2 / PEAK_BF16, 4),
        "speedup_vs_f64": round(res["f64"][0] / res["ozaki_bf16"][0], 3),
        "speedup_vs_ozaki": round(res["ozaki"][0] / res["ozaki_bf16"][0], 3)}
    del A, B

    dims = [tuple(int(x) for x in d) for d in synth.batch_dims(512, seed=5)]
    flops = sum(2.0 * a * b * c for a, b, c in dims)
    mats = []
    for i, (bm, bn, bk) in enumerate(dims):
        A = torch.empty((bm, bk), dtype=torch.float32, device=dev)
        B = torch.empty((bk, bn), dtype=torch.float32, device=dev)
        C = torch.empty((bm, bn), dtype=torch.float32, device=dev)
        synth.fill_device(A, 1000 + i, synth.STREAM_A, synth.UNIFORM_F32)
        synth.fill_device(B, 1000 + i, synth.STREAM_B, synth.UNIFORM_F32)
        mats.append((A, B, C))
    args = (512, [d[0] for d in dims], [d[1] for d in dims], [d[2] for d in dims], [1.0] * 512,
            [x[0] for x in mats], [d[2] for d in dims], [x[1] for x in mats],
            [d[1] for d in dims], [0.0] * 512, [x[2] for x in mats], [d[1] for d in dims])
    rc, h = cm.cosma_batch_create(*args, cm.COSMA_F32, stream)
    cm.check(rc, "cosma_batch_create")
    rc, policy, groups, items, pol_ms = cm.cosma_batch_info(h)
    t_graph, st_graph = _time(torch, stream, lambda: cm.cosma_batch_run(h, stream), reps,
                                min(3, reps))
    ws = max(cm.cosma_workspace_size(a, b, c, cm.COSMA_F32)[1] for a, b, c in dims)
    cm.ensure_workspace(ws)

    def loop():
        for i, (bm, bn, bk) in enumerate(dims):
            cm.cosma_gemm(bm, bn, bk, 1.0, mats[i][0], bk, mats[i][1], bn, 0.0, mats[i][2], bn,
                          cm.COSMA_F32, stream)
    t_loop, st_loop = _time(torch, stream, loop, reps, min(3, reps))
    # one-shot call: the planner's batch policy, workspace-staged, no graph
    rc, ws_b = cm.cosma_workspace_size_batched(*args[:5], cm.COSMA_F32)
    cm.check(rc, "cosma_workspace_size_batched")
    cm.ensure_workspace(ws_b)
    t_one, st_one = _time(torch, stream, lambda: cm.check(cm.cosma_gemm_batched(
        *args, cm.COSMA_F32, stream), "cosma_gemm_batched"), reps, min(3, reps))
    rc, splits = cm.cosma_batch_splits(h, 512)
    cm.cosma_batch_run(h, stream)  # final results come from the graph
    torch.cuda.synchronize()
    cm.cosma_batch_destroy(h)
    out["batched_512_f32"] = {
        "problems": 512, "dims": "m,n,k log-uniform in [64,4096], seeded per problem",
        "sum_2mnk": flops, "graph_ms": round(t_graph, 3), "graph_ms_ci95": st_graph["ci95"],
        "graph_tflops": round(flops / (t_graph * 1e-3) / 1e12, 2),
        "loop_of_single_launches_ms": round(t_loop, 3), "loop_ms_ci95": st_loop["ci95"],
        "loop_tflops": round(flops / (t_loop * 1e-3) / 1e12, 2),
        "speedup_vs_loop": round(t_loop / t_graph, 3), "autotuned_policy": policy,
        "policy_candidates_ms": [round(x, 3) for x in pol_ms], "persistent_launches": groups,
        "work_items": items, "problems_split": int(sum(1 for x in splits if x > 1)),
        "graph_frac_f32_peak": round(flops / (t_graph * 1e-3) / 1e12 / PEAK_F32, 4),
        "oneshot_ms": round(t_one, 3), "oneshot_ms_ci95": st_one["ci95"]}
    keep.append(("batched", mats, dims, None, None, synth.UNIFORM_F32, "f32"))
    return out


# Equal-work FP64 shapes (2 mnk = 2^41) from deep k to wide C: the planner
# cuts k (regime 1, split-K) while mn / S is below the number of CUs and
# parallelises i, j only (regime 0) above it; then large-M and flat.
SWEEP_SHAPES = [(1024, 1024, 1 << 20), (2048, 2048, 1 << 18), (4096, 4096, 1 << 16),
                (8192, 8192, 1 << 14), (16384, 16384, 1 << 12), (1 << 20, 1024, 1024),
                (65536, 65536, 256)]
# One shape under each FP64 tile: less fast memory per CU in use, more I/O.
SWEEP_TILES = (8192, 8192, 8192)


def run_sweep(torch, cm, synth, dev, stream, reps):
    out = {"regimes": [], "tiles": [], "memory_scenarios": []}

    def one(m, n, k, plan, tag, dtype="f64"):
        f32 = dtype == "f32"
        tdt = torch.float32 if f32 else torch.float64
        dist = synth.UNIFORM_F32 if f32 else synth.UNIFORM_F64
        A = torch.empty((m, k), dtype=tdt, device=dev)
        B = torch.empty((k, n), dtype=tdt, device=dev)
        C = torch.empty((m, n), dtype=tdt, device=dev)
        synth.fill_device(A, SEED, synth.STREAM_A, dist)
        synth.fill_device(B, SEED, synth.STREAM_B, dist)
        cm.ensure_workspace(plan.workspace_bytes)
        ms, st = _time(torch, stream, lambda: cm.gemm(A, B, C, dtype=dtype, plan=plan, stream=stream),
                       reps, min(3, reps))
        tf = 2.0 * m * n * k / (ms * 1e-3) / 1e12
        log(f"sweep {tag} {dtype} {m}x{n}x{k}: {ms:.3f} ms {tf:.2f} TFLOP/s")
        row = {"m": m, "n": n, "k": k, "tile": f"{plan.tile_m}x{plan.tile_n}", "p_k": plan.p_k,
               "group_m": plan.group_m, "regime": plan.regime, "p1": round(plan.p1, 2),
               "a_par": round(plan.a_par, 1), "sqrt_S": round(plan.S_words ** 0.5, 1),
               "items": plan.items, "waves": plan.waves, "ms": ms, "ms_ci95": st["ci95"],
               "tflops": round(tf, 3), "frac_peak": round(tf / (PEAK_F32 if f32 else PEAK_F64), 4),
               "predicted_ms": round(plan.predicted_ms, 3),
               "q_cu_words": plan.q_cu_words, "thm1_words": plan.thm1_words,
               "q_cu_over_thm1": round(plan.q_cu_words / plan.thm1_words, 4),
               "q_ea_bytes": plan.q_ea_bytes}
        del A, B, C
        torch.cuda.empty_cache()
        return row

    for (m, n, k) in SWEEP_SHAPES:
        rc, plan = cm.cosma_plan_query(m, n, k, cm.COSMA_F64)
        cm.check(rc, "plan")
        out["regimes"].append(one(m, n, k, plan, "regime"))
    m, n, k = SWEEP_TILES
    for t in range(3):
        rc, plan = cm.cosma_plan_make(m, n, k, cm.COSMA_F64, t, 1)
        cm.check(rc, "plan")
        row = one(m, n, k, plan, f"tile {t}")
        row["tile_words_per_cu"] = plan.tile_m * plan.tile_n * plan.wg_per_cu
        out["tiles"].append(row)
    # the paper's limited / extra-memory shapes for p = 256 CUs of S_CU words
    for dtype, dt in (("f64", cm.COSMA_F64), ("f32", cm.COSMA_F32)):
        rc, probe = cm.cosma_plan_query(1024, 1024, 1024, dt)
        for name, (m, n, k) in synth.memory_scenarios(probe.S_words, 256):
            rc, plan = cm.cosma_plan_query(m, n, k, dt)
            cm.check(rc, "plan")
            row = one(m, n, k, plan, name, dtype)
            row["scenario"] = name
            row["dtype"] = dtype
            out["memory_scenarios"].append(row)
    return out


def run_small(torch, cm, synth, dev, stream, reps):
    """The small FP64 product 512^3 (uniform[-1,1], seed 0): launch-bound;
    timed like the variants, its result kept for the oracle."""
    m = n = k = 512
    A = torch.empty((m, k), dtype=torch.float64, device=dev)
    B = torch.empty((k, n), dtype=torch.float64, device=dev)
    C = torch.empty((m, n), dtype=torch.float64, device=dev)
    synth.fill_device(A, 0, synth.STREAM_A, synth.UNIFORM_F64)
    synth.fill_device(B, 0, synth.STREAM_B, synth.UNIFORM_F64)
    rc, plan = cm.cosma_plan_query(m, n, k, cm.COSMA_F64)
    cm.ensure_workspace(plan.workspace_bytes)
    ms, st = _time(torch, stream, lambda: cm.gemm(A, B, C, dtype="f64", stream=stream), reps,
                   min(3, reps))
    torch.cuda.synchronize()
    tf = 2.0 * m * n * k / (ms * 1e-3) / 1e12
    return {"shape": "512x512x512", "seed": 0, "ms": ms, "ms_ci95": st["ci95"],
            "tflops": round(tf, 3), "frac_peak": round(tf / PEAK_F64, 4),
            "tile": f"{plan.tile_m}x{plan.tile_n}", "p_k": plan.p_k, "C": C.cpu().numpy()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _regen(jobs, threads):
    """Run independent synth.gen calls on a thread pool (numpy releases the
    GIL inside its array kernels)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda a: a[0](*a[1:]), jobs))


def cpu_baseline(probs, small, keep, torch):
    """The oracle as it stands, timed on the host cores.

    value: the bench workload's square product on a bounded sample (its
    first R rows, A and B regenerated on the host, B bit-checked against the
    device fill on sampled entries).  Also, in full: the small 512^3 product
    and the 512-problem FP32 batch, whose GPU results are compared entry by
    entry."""
    import numpy as np
    import oracle
    import synth
    threads = oracle.default_threads()
    rows_out = []
    # small product, in full
    m = n = k = 512
    A1 = synth.gen(m, k, 0, synth.STREAM_A, synth.UNIFORM_F64)
    B1 = synth.gen(k, n, 0, synth.STREAM_B, synth.UNIFORM_F64)
    t0 = time.perf_counter()
    ref, D = oracle.gemm(A1, B1, threads=threads)
    dt = time.perf_counter() - t0
    err = oracle.normalised_err(small["C"], ref, D)
    rows_out.append({"config": "FP64 512x512x512, uniform[-1,1] seed 0 (in full)",
                     "seconds": round(dt, 4), "tflops": round(2.0 * m * n * k / dt / 1e12, 6),
                     "gpu_ms": small["ms"], "gpu_err": err, "err_bound": oracle.fp64_bound(k),
                     "within_bound": bool(err <= oracle.fp64_bound(k))})
    # square product: the first R rows
    p = next((q for q in probs if q["name"] == "square"), probs[0])
    m, n, k = p["m"], p["n"], p["k"]
    rows = int(os.environ.get("COSMA_BENCH_ORACLE_ROWS", "512"))
    rows = max(1, min(rows, m))
    Ar = synth.gen(m, k, SEED, synth.STREAM_A, synth.UNIFORM_F64, row_idx=np.arange(rows))
    blk = -(-k // threads)
    parts = _regen([(synth.gen, k, n, SEED, synth.STREAM_B, synth.UNIFORM_F64, 0,
                     np.arange(t0_, min(k, t0_ + blk))) for t0_ in range(0, k, blk)], threads)
    Bh = np.concatenate(parts, axis=0)
    del parts
    rng = np.random.default_rng(11)
    ri = rng.integers(0, k, 4096)
    ci = rng.integers(0, n, 4096)
    dev_b = p["B"][torch.as_tensor(ri, device=p["B"].device),
                   torch.as_tensor(ci, device=p["B"].device)].cpu().numpy()
    b_match = bool(np.array_equal(dev_b, Bh[ri, ci]))
    t0 = time.perf_counter()
    ref, D = oracle.gemm(Ar, Bh, threads=threads)
    dt = time.perf_counter() - t0
    del Bh
    got = p["C"][:rows].cpu().numpy()
    err = oracle.normalised_err(got, ref, D)
    flops = 2.0 * rows * n * k
    value = flops / dt / 1e12
    rows_out.append({"config": f"FP64 square {m}x{n}x{k}: first {rows} rows of C",
                     "seconds": round(dt, 3), "tflops": round(value, 6),
                     "device_B_equals_host_regeneration": b_match, "gpu_err": err,
                     "err_bound": oracle.fp64_bound(k),
                     "within_bound": bool(err <= oracle.fp64_bound(k))})
    # 512-problem FP32 batch, in full
    bt = next((e for e in keep if e[0] == "batched"), None)
    if bt is not None:
        _, mats, dims, _, _, dist, _ = bt
        jobs = []
        for i, (bm, bn, bk) in enumerate(dims):
            jobs.append((synth.gen, bm, bk, 1000 + i, synth.STREAM_A, dist))
            jobs.append((synth.gen, bk, bn, 1000 + i, synth.STREAM_B, dist))
        mats_h = _regen(jobs, threads)
        got = [mats[i][2].cpu().numpy() for i in range(len(dims))]
        t0 = time.perf_counter()
        worst, fl = 0.0, 0.0
        for i, (bm, bn, bk) in enumerate(dims):
            ref, D = oracle.gemm(mats_h[2 * i], mats_h[2 * i + 1], threads=threads)
            e = oracle.normalised_err(got[i], ref, D)
            worst = max(worst, e / oracle.fp32_bound(bk))
            fl += 2.0 * bm * bn * bk
        dt = time.perf_counter() - t0
        rows_out.append({"config": "512 FP32 problems, m,n,k log-uniform in [64,4096] (in full)",
                         "seconds": round(dt, 3), "tflops": round(fl / dt / 1e12, 6),
                         "gpu_worst_err_over_bound": worst, "within_bound": bool(worst <= 1.0)})
    return {"value": round(value, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"first {rows} rows of C for the square {m}x{n}x{k} FP64 product "
                      f"({flops:.3e} flops, {rows_out[1]['seconds']:.2f} s)",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(), "per_config": rows_out}


def sampled_accuracy(probs, keep):
    """Normalised error of every measured result on sampled rows and columns
    (random ones plus the last), against the oracle on regenerated inputs."""
    import numpy as np
    import oracle
    import synth
    rng = np.random.default_rng(7)
    out = []

    def one(name, C, m, n, k, seed, dist, cls, nsamp=12):
        rows = np.unique(np.concatenate([rng.integers(0, m, nsamp), [0, m - 1]]))
        cols = np.unique(np.concatenate([rng.integers(0, n, nsamp), [0, n - 1]]))
        Ar = synth.gen(m, k, seed, synth.STREAM_A, dist, row_idx=rows)
        Bc = synth.gen(k, n, seed, synth.STREAM_B, dist, col_idx=cols)
        ref, D = oracle.gemm(Ar, Bc)
        import torch
        ri = torch.as_tensor(rows, device=C.device)
        ci = torch.as_tensor(cols, device=C.device)
        got = C.index_select(0, ri).index_select(1, ci).double().cpu().numpy()
        err = oracle.normalised_err(got, ref, D)
        bound = oracle.fp64_bound(k) if cls == "f64" else oracle.fp32_bound(k)
        return {"result": name, "err": err, "bound": bound, "within": bool(err <= bound)}

    for p in probs:
        out.append(one(f"f64 {p['name']}", p["C"], p["m"], p["n"], p["k"], SEED,
                       synth.UNIFORM_F64, "f64", 8 if p["k"] > 100000 else 16))
    for entry in keep:
        if entry[0] == "batched":
            _, mats, dims, _, _, dist, cls = entry
            worst = None
            for i in range(0, len(dims), 8):
                m, n, k = dims[i]
                r = one(f"batched #{i}", mats[i][2], m, n, k, 1000 + i, dist, cls, 2)
                if worst is None or r["err"] / r["bound"] > worst["err"] / worst["bound"]:
                    worst = r
            worst["result"] = "batched 512 (every 8th problem, worst)"
            out.append(worst)
        else:
            name, C, m, n, k, dist, cls = entry
            out.append(one(name, C, m, n, k, SEED, dist, cls, 8 if k > 100000 else 12))
    return out


if __name__ == "__main__":
    main()
