#!/usr/bin/env python3
"""Benchmark of the rpForests kNN path on one MI355X.

One step = the whole hot path on one batch: grow the forest (rpf_build) over the 1M x 128
anisotropic Gaussian mixture (leaf size 256) and find the K = 20 nearest neighbours of every
point among the union of its leaves (rpf_all_knn), then release the forest.  Inputs are
resident in device memory before the timed region.

The metric is queries/s at recall >= 0.99.  The recall (1 - the missing rate of Sec. 5.1)
is measured against the exact kNN of a seeded sample of 10 000 points (rpf_exact_knn);
the forest is grown tree by tree (nested forests: 32, 48, 56, 64, 68, 72, ... trees) until
it reaches 0.99, and the step is timed there: bfloat16 tiles + binary32/binary64 re-rank
(`value`) and plain binary32 tiles beside it, same steps and warm-up.  The named
configuration (32 trees) is timed as a sub-record.  Also: the roofline of the dominant
kernel (HIP events on the launch stream, inside the library), the precision path on 1M x 784
quantised data, the serving loop on the 4M x 96 forest, many uneven data sets in one
recorded launch, and the CPU oracle timed on the host.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kNN queries/s at ≥0.99 recall, FP32 vs BF16+rerank; p50/p99 latency"
PROFILES = os.path.join(ROOT, "profiles")
# HBM bytes per dispatch of the headline step's kernels at T trees (two rocprofv3 counter runs
# of `--only-step T:bf16x3`), valid while the HIP sources hash to the value recorded in it


def traffic_file(T):
    return os.path.join(PROFILES, f"hbm_traffic_allknn_1M_d128_T{T}_bf16x3.md")
PREC_INDEX = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16x3": 3, "u8grid": 4}
# kernel (name prefix in the counter summary) behind each timed record of the library for the
# 1M x 128 workload (leaves of 244/245 points: the 8 x 8 symmetric tile)
RECORD_KERNEL = {
    "tile_phase2": "k_tile_sym<8, {p}, 2, 0>",
    "tile_phase1": "k_tile_sym<8, {p}, 0, 0>",
    "proj_chunks_x3": "k_proj_chunks<true, true, false>",
    "level_small": "k_level_small<true, true, false>",
    "leaf_finalize": "k_leaf_stats<",
    "merge_first": "k_merge_first<",
    "final_rerank": "k_final<true",
}
BUILD_KERNELS = ("k_proj_root", "k_proj_chunks", "k_level_small", "k_sel_", "k_part_")
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
INT8_MFMA_PEAK_TOPS = 5000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="fewer points (same recipe), for quick checks")
    ap.add_argument("--recall-sample", type=int, default=10000, help="points whose exact kNN is the recall truth")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the recorded-plan (HIP graph) leg")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script with "
                         "--copy-probe into per-kernel HBM traffic (markdown on stdout) and exit")
    ap.add_argument("--mfma-summary", metavar="DIR", help="summarise a rocprofv3 --pmc run of MFMA counters")
    ap.add_argument("--kt-summary", metavar="DIR", help="summarise a rocprofv3 --kernel-trace --stats run "
                                                        "(markdown on stdout) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference kernel for HBM counters)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the 1M x 784 precision-path leg")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy sweep of Sec. 5 (Table 1 shapes)")
    ap.add_argument("--accuracy-runs", type=int, default=5, help="independent runs averaged per accuracy point")
    ap.add_argument("--precision-n", type=int, default=None, help="points of the precision-path leg (default 1M)")
    ap.add_argument("--only-step", default=None, metavar="T:PREC",
                    help="run only the 1M x 128 step with T trees and PREC tiles (--steps, --warmup), for profiling")
    ap.add_argument("--only-precision", action="store_true", help="run the precision-path leg alone (profiling)")
    ap.add_argument("--only-serve", action="store_true", help="run the serving leg alone (profiling)")
    ap.add_argument("--serve-n", type=int, default=None, help="points of the served forest (default: 4M)")
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests per serving measurement")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.8, 0.95],
                    help="open-loop loads as fractions of the saturated request rate")
    ap.add_argument("--serve-recall-rows", type=int, default=700, help="sampled request rows per K for recall")
    ap.add_argument("--serve-curve", default="16,32,64,96,128", help="tree counts of the served recall curve")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-data-sets leg")
    ap.add_argument("--no-uniform", action="store_true", help="skip the uniform-rule leg")
    ap.add_argument("--only-uniform", default=None, metavar="T:PREC",
                    help="run only the uniform-rule 1M x 128 step with T trees and PREC tiles, for profiling")
    ap.add_argument("--only-batched", action="store_true", help="run the many-data-sets leg alone (profiling)")
    ap.add_argument("--batch-count", type=int, default=512, help="data sets of the many-data-sets leg")
    ap.add_argument("--cpu-sample", type=int, default=20000,
                    help="points whose all-points kNN the CPU baseline times (extrapolated to n)")
    ap.add_argument("--headline-prec", default="bf16x3", choices=["bf16x3", "bf16", "fp16"],
                    help="tile precision of the headline (low-precision + re-rank) path")
    ap.add_argument("--target-recall", type=float, default=0.99,
                    help="recall the at-target leg looks for by growing more trees (0 = skip the leg)")
    ap.add_argument("--target-trees", default="48,56,64,68,72,76,80,88,96,112,128",
                    help="tree counts the at-target leg tries, in order (the first T trees are the bench's)")
    ap.add_argument("--cpu-trees", type=int, default=0,
                    help="trees the CPU baseline builds (its time is scaled to all trees; 0 = all)")
    return ap.parse_args()


def mfma_peak(prec):
    """Dense MFMA peak of the tile arithmetic: bf16 for bfloat16 and split bfloat16 tiles (the
    algorithmic flops count the plain product once), int8 for grid tiles, else fp32."""
    if prec in ("bf16", "bf16x3", "fp16"):
        return BF16_MFMA_PEAK_TFLOPS
    if prec == "u8grid":
        return INT8_MFMA_PEAK_TOPS
    return FP32_MFMA_PEAK_TFLOPS


def roofline(prof):
    """Roofline of the dominant timed record (most time per step among records with
    algorithmic bytes or flops): its bound is the MFMA peak of its arithmetic when its
    algorithmic intensity (flops per algorithmic byte) is above that peak's ridge point
    (peak / 8 TB/s), HBM otherwise; achieved = algorithmic flops or bytes per launch over the
    launch's average duration (HIP events on the launch stream)."""
    best = None
    for name, r in prof.items():
        if r["algo_bytes"] <= 0 and r["algo_flops"] <= 0:
            continue
        if best is None or r["total_ms"] > prof[best]["total_ms"]:
            best = name
    if best is None:
        return None, None
    r = prof[best]
    avg_s = r["total_ms"] / r["launches"] / 1e3
    peak = mfma_peak(r.get("prec"))
    ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    ai = r["algo_flops"] / r["algo_bytes"] if r["algo_bytes"] > 0 else float("inf")
    if r["algo_flops"] > 0 and ai >= ridge:
        ach = r["algo_flops"] / r["launches"] / avg_s / 1e12
        return best, {"bound": "mfma", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
                      "frac": round(ach / peak, 4), "traffic": None,
                      "arithmetic_intensity": round(ai, 1), "ridge": round(ridge, 1)}
    ach = r["algo_bytes"] / r["launches"] / avg_s / 1e9
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    if r["algo_flops"] > 0:
        out.update(arithmetic_intensity=round(ai, 1), ridge=round(ridge, 1),
                   mfma_achieved_tflops=round(r["algo_flops"] / r["launches"] / avg_s / 1e12, 2), mfma_peak=peak)
    return best, out


BUILD_LEVEL_RECORDS = ("proj_roots", "proj_chunks_x3", "level_small", "select_passes", "partition")
KNN_RECORDS = ("tile_phase1", "merge_first", "tile_phase2", "final_rerank", "fallback")


def stage_summary(prof, steps, n, d, T, L, K):
    """Kernel time of the two halves of a step and their bounds.  The build levels: their
    time, the method's algorithmic bytes (n (4d + 36) bytes per tree and level: row, id, key
    write, one select read, partition read of key and id, id write) and the time those bytes
    would take at the HBM peak -- the linked levels read X once per two levels, so they move
    fewer bytes than that and the ratio is no fraction of a peak -- and the HBM bytes the
    counters measured (committed summary of the same step), with the rate they give.  The
    leaf pass apart; the search (queries/s of rpf_all_knn alone) with the MFMA fraction of
    its distance tiles in algorithmic flops."""
    def ms(names):
        return sum(prof[k]["total_ms"] for k in names if k in prof) / steps
    lv_ms, leaf_ms, knn_ms = ms(BUILD_LEVEL_RECORDS), ms(("leaf_finalize",)), ms(KNN_RECORDS)
    lv_bytes = float(n) * (4 * d + 36) * L * T
    tiles = [prof[k] for k in ("tile_phase1", "tile_phase2") if k in prof]
    t_flops = sum(r["algo_flops"] for r in tiles) / steps
    t_ms = sum(r["total_ms"] for r in tiles) / steps
    peak = mfma_peak(tiles[0].get("prec") if tiles else None)
    measured = build_traffic_per_step(T)
    return {
        "build_levels_ms": round(lv_ms, 3),
        "build_levels_algorithmic_bytes": lv_bytes,
        "build_levels_ms_at_hbm_peak_for_algorithmic_bytes": round(lv_bytes / (HBM_PEAK_GBS * 1e9) * 1e3, 3),
        "build_levels_hbm_bytes_measured": measured,
        "build_levels_hbm_GBps_measured": round(measured / (lv_ms / 1e3) / 1e9, 1) if measured and lv_ms else None,
        "build_levels_hbm_frac_measured": round(measured / (lv_ms / 1e3) / (HBM_PEAK_GBS * 1e9), 4)
        if measured and lv_ms else None,
        "leaf_pass_ms": round(leaf_ms, 3),
        "all_knn_ms": round(knn_ms, 3),
        "all_knn_queries_per_s": round(n / (knn_ms / 1e3), 1) if knn_ms else None,
        "tiles_mfma_frac": round(t_flops / (t_ms / 1e3) / (peak * 1e12), 4) if t_ms else None,
    }


def source_hash():
    """Hash of the HIP sources: traffic figures are valid only for the kernels they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1812_11689_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _csv_rows(d, suffix):
    import csv
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                with open(os.path.join(root, f)) as fh:
                    return list(csv.DictReader(fh))
    raise SystemExit(f"no *{suffix} under {d}")


def _short(name):
    name = name.split("(")[0]
    for pre in ("void ", "rpf::"):
        name = name.replace(pre, "")
    return name.strip()


def pmc_summary(fetch_dir, write_dir):
    """Per-kernel HBM bytes per dispatch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the counter reads for the plain copy of --copy-probe MiB."""
    fr = _csv_rows(fetch_dir, "counter_collection.csv")
    wr = _csv_rows(write_dir, "counter_collection.csv")
    probe_w = max((r for r in wr if "copyBuffer" in r["Kernel_Name"]), key=lambda r: float(r["Counter_Value"]))
    probe_id = probe_w["Dispatch_Id"]
    probe_f = next(r for r in fr if r["Dispatch_Id"] == probe_id)
    probe_bytes = round(float(probe_w["Counter_Value"]) / 1024.0) * (1 << 20)  # whole MiB written
    kf = probe_bytes / (float(probe_f["Counter_Value"]) * 1024.0)
    kw = probe_bytes / (float(probe_w["Counter_Value"]) * 1024.0)
    agg = {}
    for rows, key in ((fr, "fetch"), (wr, "write")):
        for r in rows:
            k = _short(r["Kernel_Name"])
            a = agg.setdefault(k, {"fetch": [], "write": []})
            a[key].append(float(r["Counter_Value"]) * 1024.0)
    out = {"source_hash": source_hash(), "probe_bytes": probe_bytes, "fetch_scale": round(kf, 4),
           "write_scale": round(kw, 4), "kernels": {}}
    lines = ["| kernel | dispatches | FETCH_SIZE GB/dispatch | WRITE_SIZE GB/dispatch | HBM GB/dispatch (scaled) |",
             "|---|---|---|---|---|"]
    for k, a in sorted(agg.items(), key=lambda kv: -sum(kv[1]["fetch"]) - sum(kv[1]["write"])):
        if not a["fetch"] or not a["write"] or not k.startswith("k_"):  # the library's kernels only
            continue
        f = sum(a["fetch"]) / len(a["fetch"])
        w = sum(a["write"]) / len(a["write"])
        tot = f * kf + w * kw
        out["kernels"][k] = {"dispatches": len(a["fetch"]), "bytes_per_dispatch": round(tot)}
        if len(lines) < 24:
            lines.append(f"| {k} | {len(a['fetch'])} | {f / 1e9:.3f} | {w / 1e9:.3f} | {tot / 1e9:.3f} |")
    print(f"Copy probe: {probe_bytes / 2**30:.2f} GiB read and written; FETCH_SIZE reads "
          f"{float(probe_f['Counter_Value']) * 1024 / 2**30:.3f} GiB of it (scale {kf:.4f}), WRITE_SIZE "
          f"{float(probe_w['Counter_Value']) * 1024 / 2**30:.3f} GiB (scale {kw:.4f}).\n")
    print("\n".join(lines))
    print("\nMachine-readable (read by bench.py while the HIP sources hash to source_hash):\n")
    print(json.dumps(out))


XCDS = 8  # GRBM_GUI_ACTIVE sums the active cycles of the eight XCDs


def mfma_summary(d):
    """Per-kernel MFMA counters per dispatch from one rocprofv3 --pmc run: executed MFMA ops
    (SQ_INSTS_VALU_MFMA_MOPS_* x 512), MFMA-busy cycles over (GUI-active cycles of one XCD x
    SIMDs); GRBM_GUI_ACTIVE counts every XCD, so it is divided by their number."""
    rows = _csv_rows(d, "counter_collection.csv")
    agg = {}
    for r in rows:
        k = _short(r["Kernel_Name"])
        if not k.startswith("k_"):
            continue
        a = agg.setdefault(k, {})
        a.setdefault(r["Counter_Name"], {})[r["Dispatch_Id"]] = float(r["Counter_Value"])
    simds = 256 * 4
    print("| kernel | dispatches | MFMA Tops/dispatch (bf16, f32, i8) | MFMA busy / (GUI active per XCD x SIMDs) |")
    print("|---|---|---|---|")
    out = {}
    for k, a in sorted(agg.items(), key=lambda kv: -sum(kv[1].get("GRBM_GUI_ACTIVE", {}).values())):
        disp = len(a.get("GRBM_GUI_ACTIVE", {})) or 1
        ops = [sum(a.get(f"SQ_INSTS_VALU_MFMA_MOPS_{t}", {}).values()) * 512 / disp / 1e12 for t in ("BF16", "F32", "I8")]
        busy = sum(a.get("SQ_VALU_MFMA_BUSY_CYCLES", {}).values())
        gui = sum(a.get("GRBM_GUI_ACTIVE", {}).values())
        frac = busy / (gui / XCDS * simds) if gui else 0.0
        out[k] = {"mfma_tops": [round(v, 4) for v in ops], "mfma_busy_frac": round(frac, 4)}
        if sum(ops) > 0 or frac > 0:
            print(f"| {k} | {disp} | {ops[0]:.3f}, {ops[1]:.3f}, {ops[2]:.3f} | {frac:.4f} |")
    print("\n" + json.dumps(out))


def kt_summary(d):
    rows = _csv_rows(d, "kernel_stats.csv")
    print("| kernel | calls | total ms | average us | share |")
    print("|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:20]:
        print(f"| {_short(r['Name'])[:70]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")


def _traffic_table(T):
    """The committed counter summary of the headline step at T trees, or None when absent or
    stale."""
    if not os.path.exists(traffic_file(T)):
        return None
    with open(traffic_file(T)) as fh:
        js = [ln for ln in fh if ln.startswith("{")]
    if not js:
        return None
    t = json.loads(js[-1])
    return t if t.get("source_hash") == source_hash() else None


def traffic_for(record, prec, T):
    """HBM bytes per launch of a timed record at T trees (scaled FETCH_SIZE + WRITE_SIZE), or
    None."""
    pat = RECORD_KERNEL.get(record)
    t = _traffic_table(T)
    if not pat or t is None:
        return None
    pat = pat.format(p=PREC_INDEX.get(prec, 0))
    for k, v in t["kernels"].items():
        if k == pat or (pat.endswith("<") or pat.endswith("true")) and k.startswith(pat):
            return v["bytes_per_dispatch"]
    return None


def build_traffic_per_step(T):
    """HBM bytes of the build-level kernels in one step at T trees, from the counter summary
    (whose run is one step), or None."""
    t = _traffic_table(T)
    if t is None:
        return None
    return sum(v["bytes_per_dispatch"] * v["dispatches"] for k, v in t["kernels"].items()
               if k.startswith(BUILD_KERNELS))


def timed_steps(step, steps, warmup):
    """W untimed warm-up steps, then K timed steps bracketed by synchronisations; per-kernel
    records from the library's HIP events on the launch stream over the timed steps."""
    import torch
    from paper_1812_11689_amd import rpf
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    rpf.profile_reset()
    rpf.profile_enable(True)
    times = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    out = None
    for _ in range(steps):
        ts = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    rpf.profile_enable(False)
    return out, elapsed, times, rpf.profile_read()


def step_record(n, steps, elapsed, times, prof):
    return {"value": round(n * steps / elapsed, 1), "ms_per_step": round(elapsed / steps * 1e3, 3),
            "step_ms_p50": round(float(np.percentile(times, 50)) * 1e3, 3),
            "step_ms_p99": round(float(np.percentile(times, 99)) * 1e3, 3),
            "breakdown_ms_per_step": {k: round(v["total_ms"] / steps, 3)
                                      for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])}}


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.kt_summary:
        kt_summary(args.kt_summary)
        return
    if args.mfma_summary:
        mfma_summary(args.mfma_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding "
                                   "by trees is a design note only)"}))
        sys.exit(2)
    import torch
    from paper_1812_11689_amd import metrics, rpf
    from paper_1812_11689_amd import workloads as W

    if args.only_serve:
        print(json.dumps({"serving": serving_leg(args)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": batched_leg(args)}), flush=True)
        return
    if args.only_precision:
        print(json.dumps({"precision_path": precision_leg(args)}), flush=True)
        return
    if args.only_step:
        Ts, prec = args.only_step.split(":")
        w = W.make_config(2, n=args.n)
        n, d = w.x.shape
        Tq, n0, K = int(Ts), w.leaf_size, w.k
        Lq = rpf.depth(n, n0)
        Xq = torch.from_numpy(w.x).cuda()
        Rq = torch.from_numpy(W.directions(w.dir_seed, Tq, (1 << Lq) - 1, 1, d)).cuda()
        if args.copy_probe:  # a plain device copy of known size, whose counters give their scale
            src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst

        def one():
            f = rpf.build(Xq, Tq, n0, Rq, dist_prec=prec)
            out = f.all_knn(K)
            f.free()
            return out
        _, el, times, prof = timed_steps(one, args.steps, args.warmup)
        print(json.dumps({"only_step": f"allknn_1M_d128_T{Tq}", "prec": prec, **step_record(n, args.steps, el, times, prof)}),
              flush=True)
        return
    if args.only_uniform:
        Ts, prec = args.only_uniform.split(":")
        w = W.make_config(2, n=args.n)
        Xq = torch.from_numpy(w.x).cuda()

        def one():
            f = rpf.build(Xq, int(Ts), w.leaf_size, None, dist_prec=prec, split_rule="uniform", seed=UNIFORM_SEED)
            out = f.all_knn(w.k)
            f.free()
            return out
        _, el, times, prof = timed_steps(one, args.steps, args.warmup)
        print(json.dumps({"only_uniform": f"allknn_1M_d128_T{Ts}_uniform", "prec": prec,
                          **step_record(len(w.x), args.steps, el, times, prof)}), flush=True)
        return
    t0 = time.time()
    w = W.make_config(2, n=args.n)
    n, d = w.x.shape
    T0, n0, K = w.n_trees, w.leaf_size, w.k
    L = rpf.depth(n, n0)
    trees = sorted({T0, *[int(v) for v in args.target_trees.split(",") if int(v) > T0]})
    # directions of the largest forest; tree t always uses stream (seed, t), so every smaller
    # forest is a prefix of it
    R = W.directions(w.dir_seed, trees[-1], (1 << L) - 1, 1, d)
    X = torch.from_numpy(w.x).cuda()
    torch.cuda.synchronize()
    print(f"# workload {w.name}: n={n} d={d} T={T0} n0={n0} K={K} L={L} (generated in {time.time() - t0:.1f}s)",
          file=sys.stderr, flush=True)

    if args.copy_probe:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written", file=sys.stderr, flush=True)
        del src, dst

    # ground truth of the recall (Sec. 5.1): exact kNN of a seeded sample of points by the
    # library's brute-force kernel (binary64 distances, ties by index), each point left out
    rng = np.random.default_rng(W.SEED_BASE + 300 + 2)
    pts = np.sort(rng.choice(n, size=min(args.recall_sample, n), replace=False))
    pts_d = torch.from_numpy(pts.astype(np.int64)).cuda()
    torch.cuda.synchronize()
    te = time.perf_counter()
    ti, td = rpf.exact_knn(X, X[pts_d], K, pts_d)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - te
    truth, truth_d = ti.cpu().numpy(), td.cpu().numpy()
    exact = {"sample": len(pts), "ms": round(t_exact * 1e3, 2), "queries_per_s": round(len(pts) / t_exact, 1),
             "binary64_distances_per_s": round(len(pts) * n / t_exact, 1)}
    print(f"# exact truth of {len(pts)} points: {t_exact * 1e3:.1f} ms", file=sys.stderr, flush=True)

    Rd = {}

    def dirs(T):
        if T not in Rd:
            Rd[T] = torch.from_numpy(np.ascontiguousarray(R[:T])).cuda()
        return Rd[T]

    def step_fn(T, prec):
        def step():
            f = rpf.build(X, T, n0, dirs(T), dist_prec=prec)
            out = f.all_knn(K)
            f.free()
            return out
        return step

    # recall of the forest as it grows (nested forests: the first T trees are the T-tree forest)
    sweep, t_star, ref_idx = [], None, {}
    for T in trees:
        f = rpf.build(X, T, n0, dirs(T), dist_prec="fp32")
        it, dt = f.all_knn(K)
        st_t = f.knn_stats()
        f.free()
        found = it.cpu().numpy()[pts]
        r_t = metrics.recall(found, truth)
        sweep.append({"n_trees": T, "recall": round(r_t, 5),
                      "kth_distance_excess": round(metrics.kth_distance_excess(dt.cpu().numpy()[pts], truth_d), 6),
                      "fallback_rows": st_t.get("fallback_rows")})
        ref_idx[T] = it
        print(f"# T={T}: recall {r_t:.4f}", file=sys.stderr, flush=True)
        if r_t >= args.target_recall and t_star is None:
            t_star = T
            break
    if t_star is None:
        t_star = trees[-1]
    recall_star = next(s_["recall"] for s_ in sweep if s_["n_trees"] == t_star)

    # the headline: the whole step (build + all-points kNN + free) at the tree count that
    # reaches the target recall, bfloat16 tiles + re-rank, and plain binary32 beside it
    res = {}
    profs = {}
    for prec in (args.headline_prec, "bf16", "fp32") if args.headline_prec != "bf16" else ("bf16", "fp32"):
        (idx, _), el, times, prof = timed_steps(step_fn(t_star, prec), args.steps, args.warmup)
        for r_ in prof.values():
            r_["prec"] = prec
        profs[prec] = prof
        res[prec] = step_record(n, args.steps, el, times, prof)
        res[prec]["identical_to_sweep"] = bool(torch.equal(idx, ref_idx[t_star]))
        print(f"# T={t_star} {prec}: {res[prec]['ms_per_step']} ms/step", file=sys.stderr, flush=True)
    head = res[args.headline_prec]
    head_prof = profs[args.headline_prec]

    # the named configuration (T = 32), same steps
    named = {"n_trees": T0, "recall": next(s_["recall"] for s_ in sweep if s_["n_trees"] == T0)}
    for prec in ("fp32", "bf16"):
        (idx, _), el, times, prof = timed_steps(step_fn(T0, prec), args.steps, args.warmup)
        named[prec] = step_record(n, args.steps, el, times, prof)
        named[prec]["identical_to_sweep"] = bool(torch.equal(idx, ref_idx[T0]))
        print(f"# T={T0} {prec}: {named[prec]['ms_per_step']} ms/step", file=sys.stderr, flush=True)

    # the uniform split rule of Alg. 1 (c uniform between the node's extreme projections,
    # directions and split points from the library's counter-based generator) on the same
    # data and K, at the headline's tree count and tile precision
    uniform = None
    if not args.no_uniform:
        uniform = uniform_leg(args, X, n0, K, t_star, pts, truth, truth_d, res[args.headline_prec])
        print(f"# uniform rule: {uniform}", file=sys.stderr, flush=True)

    # the same step recorded once as a HIP graph (rpf_plan_*: build and candidate stage, tuned
    # first-phase tree count), inputs set once before the timed launches
    def plan_leg(prec, T, ref):
        plan = rpf.Plan([n], [d], T, n0, K, dist_prec=prec)
        try:
            plan.set_inputs([X], [dirs(T)])
            plan.launch()
            plan.check()
            plan.tune()
            for _ in range(max(args.warmup, 1)):
                plan.launch()
            plan.check()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                plan.launch()
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            plan.check()
            return dict(value=round(n * args.steps / el, 1), ms_per_step=round(el / args.steps * 1e3, 3),
                        first_trees=plan.parts[0].get("first_trees"),
                        identical_to_plain=bool(torch.equal(plan.result(0)[0], ref)))
        finally:
            plan.close()

    graph = None
    if not args.no_graph:
        graph = {prec: plan_leg(prec, t_star, ref_idx[t_star]) for prec in res}
        print(f"# recorded plan: {graph}", file=sys.stderr, flush=True)

    dom, roof = roofline(head_prof)
    if roof is not None and dom is not None:
        tr = traffic_for(dom, args.headline_prec, t_star)
        roof["traffic"] = tr  # HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE), or None
        if tr is not None:
            roof["traffic_source"] = os.path.relpath(traffic_file(t_star), ROOT)
    stages = stage_summary(head_prof, args.steps, n, d, t_star, L, K)

    f = rpf.build(X, t_star, n0, dirs(t_star), dist_prec=args.headline_prec)
    f.all_knn(K)
    st = f.knn_stats()
    f.free()
    del Rd
    torch.cuda.empty_cache()
    rpf.release_cached_memory()

    accuracy_sweep = None
    if not args.no_accuracy:
        from paper_1812_11689_amd import accuracy
        ta = time.time()
        accuracy_sweep = accuracy.run(runs=args.accuracy_runs,
                                      progress=lambda m: print(f"# accuracy: {m}", file=sys.stderr, flush=True))
        accuracy_sweep["seconds"] = round(time.time() - ta, 1)
        torch.cuda.empty_cache()
        rpf.release_cached_memory()

    precision = None
    if not args.no_precision:
        precision = precision_leg(args)
        torch.cuda.empty_cache()
        rpf.release_cached_memory()

    serving = None
    if not args.no_serve:
        del X
        torch.cuda.empty_cache()
        rpf.release_cached_memory()
        serving = serving_leg(args)

    batched = None
    if not args.no_batched:
        torch.cuda.empty_cache()
        rpf.release_cached_memory()
        batched = batched_leg(args)

    cpu = None
    if not args.no_cpu_baseline:
        crng = np.random.default_rng(W.SEED_BASE + 300 + 3)
        cpts = np.sort(crng.choice(n, size=min(args.cpu_sample, n), replace=False))
        cpu = cpu_baseline(w, R[:t_star], cpts, K, args.cpu_trees)

    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.headline_prec,
        "data": "synthetic",
        "config": {"workload": f"allknn_1M_d128_T{t_star}", "n": n, "d": d, "n_trees": t_star, "leaf_size": n0,
                   "K": K, "tile_prec": args.headline_prec, "split_projection": "f64", "rerank": "fp32+f64",
                   "trees_chosen_for_recall": args.target_recall, "named_config_trees": T0},
        "recall": recall_star,
        "recall_truth": "exact kNN (rpf_exact_knn, binary64) of a seeded sample of points; Sec. 5.1 missing rate",
        "step_ms_p50": head["step_ms_p50"],
        "step_ms_p99": head["step_ms_p99"],
        "headline_path": f"{args.headline_prec} tiles + fp32/f64 re-rank",
        "bf16_rerank": res["bf16"],
        "bf16x3_rerank": res.get("bf16x3"),
        "fp32": res["fp32"],
        "speedup_over_fp32": round(head["value"] / res["fp32"]["value"], 4),
        "recall_sweep": sweep,
        "named_config": named,
        "recorded_plan": graph,
        "exact_truth": exact,
        "knn_stats": st,
        "stages": stages,
        "roofline_kernel": dom,
        "roofline": roof,
        "cpu_baseline": cpu,
        "uniform_rule": uniform,
        "precision_path": precision,
        "accuracy_sweep": accuracy_sweep,
        "serving": serving,
        "batched": batched,
    }
    print(json.dumps(line), flush=True)


UNIFORM_SEED = 11689400  # key of the uniform rule's generator in the bench


def uniform_leg(args, X, n0, K, T, pts, truth, truth_d, median_rec):
    """Alg. 1 as printed (RPF_SPLIT_UNIFORM) over the headline's data, K, tree count and tile
    precision: the whole step (build + all-points kNN + free), its recall against the same
    exact truth, the forest's shape, and the step time against the median rule's."""
    import torch
    from paper_1812_11689_amd import metrics, rpf
    n = X.shape[0]
    prec = args.headline_prec

    def step():
        f = rpf.build(X, T, n0, None, dist_prec=prec, split_rule="uniform", seed=UNIFORM_SEED)
        out = f.all_knn(K)
        f.free()
        return out
    (idx, dist), el, times, prof = timed_steps(step, args.steps, args.warmup)
    rec = step_record(n, args.steps, el, times, prof)
    f = rpf.build(X, T, n0, None, dist_prec=prec, split_rule="uniform", seed=UNIFORM_SEED)
    info = f.info()
    i2, _ = f.all_knn(K)
    st = f.knn_stats()
    f.free()
    torch.cuda.synchronize()
    rec.update({
        "workload": f"allknn_1M_d128_T{T}_uniform", "n_trees": T, "tile_prec": prec, "seed": UNIFORM_SEED,
        "recall": round(metrics.recall(idx.cpu().numpy()[pts], truth), 5),
        "kth_distance_excess": round(metrics.kth_distance_excess(dist.cpu().numpy()[pts], truth_d), 6),
        "deepest_leaf": info["depth"], "most_leaves_per_tree": info["n_leaves"],
        "repeatable": bool(torch.equal(idx, i2)), "knn_stats": st,
        "median_rule_ms_per_step": median_rec["ms_per_step"],
        "time_vs_median_rule": round(rec["ms_per_step"] / median_rec["ms_per_step"], 4),
    })
    return rec


def precision_leg(args):
    """The precision path on quantised image-like data: 10^6 x 784, 70 % exact zeros, other
    entries k/255; T 48, n0 512 (leaves of 488/489 points), K 10.  Tile precisions: int8 grid
    tiles (exact integer grid distances, the data lying on the 1/255 grid) timed over steps;
    bfloat16 (the loose bf16 bounds send rows to the exhaustive scan on these concentrated
    distances), binary32 and split bfloat16 once each.  Every output must be identical (each is
    the exact top-K of the leaf union).  Reports step times, tile throughput, recall against
    exact kNN of a seeded sample, and the error of the bfloat16 distance model against
    binary64 on sampled leaf pairs."""
    import torch
    from paper_1812_11689_amd import metrics, rpf
    from paper_1812_11689_amd import workloads as W

    t0 = time.time()
    w = W.make_config(3, n=args.precision_n)
    n, d = w.x.shape
    T, n0, K = w.n_trees, w.leaf_size, w.k
    L = rpf.depth(n, n0)
    X = torch.from_numpy(w.x).cuda()
    R = torch.from_numpy(W.directions(w.dir_seed, T, (1 << L) - 1, 1, d)).cuda()
    torch.cuda.synchronize()
    print(f"# precision workload {w.name}: n={n} d={d} T={T} n0={n0} K={K} (generated in {time.time() - t0:.1f}s)",
          file=sys.stderr, flush=True)
    res = {"workload": w.name, "n": n, "d": d, "n_trees": T, "leaf_size": n0, "K": K}

    def step_fn(prec):
        def step():
            f = rpf.build(X, T, n0, R, dist_prec=prec)
            out = f.all_knn(K)
            f.free()
            return out
        return step

    def tiles(prof, steps, peak):
        tl = [prof[k] for k in ("tile_phase1", "tile_phase2") if k in prof]
        t_ms = sum(r["total_ms"] for r in tl) / steps
        t_fl = sum(r["algo_flops"] for r in tl) / steps
        return {"tiles_ms": round(t_ms, 3), "tiles_algorithmic_tera_ops": round(t_fl / 1e12, 3),
                "tiles_frac_of_peak": round(t_fl / (t_ms / 1e3) / (peak * 1e12), 4) if t_ms else None,
                "peak_tera_ops": peak}

    steps = max(1, min(args.steps, 3))
    (ig, _), el, times, prof = timed_steps(step_fn("u8grid"), steps, 1)
    res["u8grid"] = {**step_record(n, steps, el, times, prof), **tiles(prof, steps, INT8_MFMA_PEAK_TOPS)}
    print(f"# precision u8grid: {res['u8grid']['ms_per_step']} ms/step", file=sys.stderr, flush=True)
    for prec, peak in (("bf16", BF16_MFMA_PEAK_TFLOPS), ("fp32", FP32_MFMA_PEAK_TFLOPS),
                       ("bf16x3", BF16_MFMA_PEAK_TFLOPS)):
        (ip, _), el, times, prof = timed_steps(step_fn(prec), 1, 0)
        res[prec + "_once"] = {"ms": round(el * 1e3, 3), "identical_to_u8grid": bool(torch.equal(ip, ig)),
                               "breakdown_ms": step_record(n, 1, el, times, prof)["breakdown_ms_per_step"],
                               **tiles(prof, 1, peak)}
        print(f"# precision {prec}: {el * 1e3:.1f} ms", file=sys.stderr, flush=True)
        del ip
    res["missing_rate_vs_each_other"] = 0.0 if all(res[p + "_once"]["identical_to_u8grid"]
                                                   for p in ("bf16", "fp32", "bf16x3")) else None
    rng = np.random.default_rng(W.SEED_BASE + 303)
    pts = np.sort(rng.choice(n, size=min(2000, n), replace=False))
    pts_d = torch.from_numpy(pts.astype(np.int64)).cuda()
    ti, _ = rpf.exact_knn(X, X[pts_d], K, pts_d)
    res["recall"] = round(metrics.recall(ig.cpu().numpy()[pts], ti.cpu().numpy()), 5)
    res["recall_sample"] = len(pts)
    # the bfloat16 tile arithmetic against binary64 on the leaf pairs of sampled points (tree 0):
    # rows centred on their leaf's binary32 mean, rounded to bfloat16, products accumulated in
    # binary32 -- a model of what the bf16 tiles compute, with the same operand rounding
    f = rpf.build(X, T, n0, R, dist_prec="bf16")
    dump = f.tree_dump(0)
    f.free()
    leaf_of = dump["leaf_of"]
    errs = []
    for p in pts[:64]:
        mates = torch.nonzero(leaf_of == leaf_of[int(p)]).flatten()
        xs = X[mates]
        mu = xs.mean(0)
        c = (xs - mu).to(torch.bfloat16).float()
        a = c[(mates == int(p)).nonzero().flatten()[0]]
        Dt = (a * a).sum() + (c * c).sum(1) - 2.0 * (c @ a)
        D64 = ((xs.double() - X[int(p)].double()) ** 2).sum(1)
        ok = D64 > 0
        errs.append(((Dt.double() - D64).abs()[ok] / D64[ok]).cpu().numpy())
    e = np.concatenate(errs)
    res["bf16_distance_rel_error_vs_f64"] = {"max": float(e.max()), "mean": float(e.mean()), "pairs": int(e.size),
                                             "what": "bf16-rounded centred rows, fp32 products (tile model), tree 0"}
    print(f"# precision: {res}", file=sys.stderr, flush=True)
    return res


def serving_leg(args):
    """Continuous-batching server over the resident 4M x 96 forest (T 64, n0 256): a closed
    burst of requests gives the saturated rate; open-loop Poisson streams at 0.5, 0.8 and 0.95
    of it give request latency (p50 / p99).  Batch sizes lognormal (median 64, sigma 1.5) in
    [1, 4096], K uniform over {1, 10, 100}; queries from the served mixture with 5 % uniform
    outliers.  Recall of the served results against exact kNN (rpf_exact_knn) on sampled
    request rows, and the recall of the same rows as the forest grows (nested forests: the
    first T' trees of the T-tree forest)."""
    import torch
    from paper_1812_11689_amd import metrics, rpf
    from paper_1812_11689_amd import workloads as W

    t0 = time.time()
    w = W.make_config(4, n=args.serve_n)
    n, d = w.x.shape
    T, n0 = w.n_trees, w.leaf_size
    L = rpf.depth(n, n0)
    curve_trees = [int(v) for v in args.serve_curve.split(",") if v]
    Tmax = max([T] + curve_trees)
    X = torch.from_numpy(w.x).cuda()
    Rall = W.directions(w.dir_seed, Tmax, (1 << L) - 1, 1, d)
    R = torch.from_numpy(np.ascontiguousarray(Rall[:T])).cuda()
    nreq = args.serve_requests
    seed = W.SEED_BASE + 200 + 4
    _, sizes, ks = W.serving_requests(seed, nreq, 1.0)
    pool = int(sizes.sum())
    Qh = W.mixture_queries(seed, w.x, pool, 1000, mean_seed=W.SEED_BASE + 4)
    Q = torch.from_numpy(Qh).cuda()
    offs = np.concatenate([[0], np.cumsum(sizes)])
    reqs = [(Q[offs[i]:offs[i + 1]], int(ks[i])) for i in range(nreq)]
    outs = [(torch.empty((int(sizes[i]), int(ks[i])), dtype=torch.int32, device="cuda"),
             torch.empty((int(sizes[i]), int(ks[i])), dtype=torch.float32, device="cuda")) for i in range(nreq)]
    torch.cuda.synchronize()
    print(f"# serving workload {w.name}: n={n} d={d} T={T} n0={n0}, {nreq} requests, {pool} rows "
          f"(generated in {time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    res = {"workload": w.name, "requests_per_load": nreq, "rows_per_load": pool,
           "batch_rows": "lognormal(ln 64, 1.5) in [1, 4096]", "K": "uniform {1, 10, 100}",
           "loads": list(args.serve_loads)}

    # sampled request rows per K and their exact neighbours (the recall truth)
    samp = {}
    for k in (1, 10, 100):
        rows = []
        for i in range(nreq):
            if ks[i] == k:
                rows.extend(range(offs[i], min(offs[i + 1], offs[i] + 8)))
            if len(rows) >= args.serve_recall_rows:
                break
        rows = np.asarray(rows[:args.serve_recall_rows], dtype=np.int64)
        if len(rows):
            rd = torch.from_numpy(rows).cuda()
            ti, _ = rpf.exact_knn(X, Q[rd], k)
            samp[k] = (rows, rd, ti.cpu().numpy())
    req_of_row = np.searchsorted(offs, np.arange(pool), side="right") - 1

    def served_recall():
        hits = tot = 0
        for k, (rows, _, truth) in samp.items():
            got = np.stack([outs[req_of_row[r]][0][r - offs[req_of_row[r]]].cpu().numpy() for r in rows])
            hits += (1.0 - metrics.missing_rate(got, truth)) * truth.size
            tot += truth.size
        return round(hits / max(tot, 1), 5)

    def run(prec):
        f = rpf.build(X, T, n0, R, dist_prec=prec)
        torch.cuda.synchronize()
        srv = rpf.Server(f, slots=4, max_batch_rows=8192)
        for q, k in reqs[:64]:  # warm-up
            srv.wait(srv.submit(q, k))
        # closed burst: every request queued at once
        srv.reset_stats()
        ts = [srv.submit(q, k, out=o) for (q, k), o in zip(reqs, outs)]
        for t in ts:
            srv.wait(t)
        burst = srv.stats()
        rate = burst["requests"] / (burst["rows"] / burst["rows_per_s"])  # requests/s at saturation
        out = {"saturated_rows_per_s": round(burst["rows_per_s"], 1),
               "saturated_requests_per_s": round(rate, 1),
               "burst_mean_batch_rows": round(burst["mean_batch_rows"], 1),
               "recall": served_recall(), "open_loop": {}}
        for rho in args.serve_loads:
            srv.reset_stats()
            arr, _, _ = W.serving_requests(seed + 1, nreq, rho * rate)
            start = time.perf_counter()
            ts = []
            for i, ((q, k), o) in enumerate(zip(reqs, outs)):
                now = time.perf_counter() - start
                if arr[i] > now:
                    time.sleep(arr[i] - now)
                ts.append(srv.submit(q, k, out=o))
            for t in ts:
                srv.wait(t)
            ol = srv.stats()
            spans = srv.batch_log()
            out["open_loop"][str(rho)] = {
                "offered_requests_per_s": round(rho * rate, 1), "rows_per_s": round(ol["rows_per_s"], 1),
                "p50_ms": round(ol["p50_s"] * 1e3, 3), "p99_ms": round(ol["p99_s"] * 1e3, 3),
                "max_ms": round(ol["max_s"] * 1e3, 3), "mean_batch_rows": round(ol["mean_batch_rows"], 1),
                "failed_requests": ol["failed_requests"], "recall": served_recall(),
                "device_busy_frac": round(_busy(spans) / max(1e-9, (time.perf_counter() - start) * 1e3), 4)}
        srv.close()
        print(f"# serving {prec}: {out}", file=sys.stderr, flush=True)
        return f, out

    f16, res["fp16"] = run("fp16")
    f16.free()
    torch.cuda.empty_cache()
    f32, res["fp32"] = run("fp32")
    f32.free()
    del outs
    torch.cuda.empty_cache()
    rpf.release_cached_memory()
    # recall of the sampled rows as the forest grows (fp16 tiles; results are exact for the
    # union, so the precision does not change them)
    curve = []
    for Tc in curve_trees:
        Rc = torch.from_numpy(np.ascontiguousarray(Rall[:Tc])).cuda()
        f = rpf.build(X, Tc, n0, Rc, dist_prec="fp16")
        hits = tot = 0
        for k, (rows, rd, truth) in samp.items():
            gi, _ = f.query(Q[rd], k)
            hits += (1.0 - metrics.missing_rate(gi.cpu().numpy(), truth)) * truth.size
            tot += truth.size
        f.free()
        del Rc
        rpf.release_cached_memory()
        curve.append({"n_trees": Tc, "recall": round(hits / max(tot, 1), 5)})
        print(f"# serving recall T'={Tc}: {curve[-1]['recall']}", file=sys.stderr, flush=True)
    res["recall_by_trees"] = curve
    res["recall_sample_rows"] = int(sum(len(v[0]) for v in samp.values()))
    return res


def _busy(spans):
    """Milliseconds in which at least one batch was in flight on the device (union of spans)."""
    iv = sorted((b["start_ms"], b["end_ms"]) for b in spans if b["start_ms"] >= 0)
    tot, cur = 0.0, None
    for a, b in iv:
        if cur is None or a > cur[1]:
            if cur is not None:
                tot += cur[1] - cur[0]
            cur = [a, b]
        else:
            cur[1] = max(cur[1], b)
    if cur is not None:
        tot += cur[1] - cur[0]
    return tot


def batched_leg(args):
    """Many uneven data sets (default 512: n log-uniform in [2000, 200000], d in {8, 32, 64,
    256}, 5..50 clusters), T 16, n0 64, K 16, fp16 tiles: one recorded plan (build + all-points
    kNN of every data set in one graph launch), tuned once, timed over replays; beside it the
    eager batched path over the same parts and a one-forest-per-data-set loop on a sample."""
    from concurrent.futures import ThreadPoolExecutor

    import torch
    from paper_1812_11689_amd import rpf
    from paper_1812_11689_amd import workloads as W

    T, n0, K, prec = 16, 64, 16, "fp16"
    count = args.batch_count
    t0 = time.time()
    shapes = W.batched_shapes(count=count)
    xs = W.batched_datasets(count=count, workers=16)

    def dirs(i):
        n, d, _ = shapes[i]
        return W.directions((W.SEED_BASE + 105) * 1000 + i, T, (1 << rpf.depth(n, n0)) - 1, 1, d)

    with ThreadPoolExecutor(16) as ex:
        Rs = list(ex.map(dirs, range(count)))
    sizes = [s_[0] for s_ in shapes]
    dims = [s_[1] for s_ in shapes]
    N = sum(sizes)
    print(f"# many-data-sets workload: {count} sets, {N} points, d in {sorted(set(dims))} "
          f"(generated in {time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    res = {"workload": f"batched_{count}_sets_T16_fp16", "data_sets": count, "points": N, "K": K, "n_trees": T,
           "leaf_size": n0}
    t0 = time.time()
    plan = rpf.Plan(sizes, dims, T, n0, K, dist_prec=prec)
    plan.set_inputs(xs, Rs)
    torch.cuda.synchronize()
    res["plan_create_s"] = round(time.time() - t0, 2)
    res["parts"] = len(plan.parts)
    plan.launch()
    plan.check()
    res["tuned_ms"] = round(plan.tune(), 3)
    ch = plan.choices()
    res["first_trees"] = [c["first_trees"] for c in ch]
    res["tile_shape"] = [c["tile_shape"] for c in ch]
    res["bucket_size"] = [c["bucket_size"] for c in ch]
    res["subtree_build"] = [c["subtrees"] for c in ch]
    plan.launch()
    plan.check()
    times = []
    for _ in range(max(args.steps, 3)):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        plan.launch()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
    plan.check()
    ms = float(np.median(times)) * 1e3
    res["graph_ms_per_job"] = round(ms, 3)
    res["graph_points_per_s"] = round(N / (ms / 1e3), 1)
    # recall of a sample of data sets against exact kNN (rpf_exact_knn), Sec. 5.1 missing rate
    from paper_1812_11689_amd import metrics
    rng = np.random.default_rng(W.SEED_BASE + 305)
    hit = tot = 0
    for i in rng.choice(count, size=min(16, count), replace=False):
        X = torch.from_numpy(xs[i]).cuda()
        pts = np.sort(rng.choice(sizes[i], size=min(500, sizes[i]), replace=False))
        pd = torch.from_numpy(pts.astype(np.int64)).cuda()
        ti, _ = rpf.exact_knn(X, X[pd], K, pd)
        truth = ti.cpu().numpy()
        got = plan.result(int(i))[0][pd].cpu().numpy()
        hit += metrics.recall(got, truth) * truth.size
        tot += truth.size
    res["recall"] = round(hit / max(tot, 1), 5)
    parts = [[e_i for e_i, e in enumerate(plan.entries) if e["part"] == k] for k in range(len(plan.parts))]
    plan.close()
    torch.cuda.empty_cache()
    # the eager batched path over the same parts (one warm-up pass, then timed per part,
    # uploads excluded)
    eager = []
    for rep in range(2):
        eager = []
        for ids in parts:
            dev = [torch.from_numpy(xs[i]).cuda() for i in ids]
            R = torch.from_numpy(np.concatenate([Rs[i] for i in ids], axis=1)).cuda()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            f = rpf.build_batched(dev, T, n0, R, dist_prec=prec)
            f.all_knn(K)
            f.free()
            torch.cuda.synchronize()
            eager.append(time.perf_counter() - t1)
            del dev, R
    res["eager_batched_ms_per_job"] = round(sum(eager) * 1e3, 3)
    # one forest per data set, on a sample of data sets
    sample = list(range(min(64, count)))
    pts_s = sum(sizes[i] for i in sample)
    dev = [torch.from_numpy(xs[i]).cuda() for i in sample]
    Rd = [torch.from_numpy(Rs[i]).cuda() for i in sample]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for x, r in zip(dev, Rd):
        f = rpf.build(x, T, n0, r, dist_prec=prec)
        f.all_knn(K)
        f.free()
    torch.cuda.synchronize()
    per = time.perf_counter() - t1
    res["per_data_set_points_per_s"] = round(pts_s / per, 1)
    res["per_data_set_sample"] = f"first {len(sample)} data sets, {pts_s} points, {per * 1e3:.1f} ms"
    print(f"# many data sets: {res}", file=sys.stderr, flush=True)
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, R, sample_pts, K, cpu_trees):
    """The oracle as it stands, on the host cores: the forest build timed in full on all n
    points (all T trees, or `cpu_trees` of them scaled by T/cpu_trees), plus all-points kNN
    timed on a seeded sample of points and extrapolated linearly to n; then one thread on a
    smaller sample (two trees, scaled; 200 points) for the single-core rate."""
    import oracle
    oracle.build(force=False)
    n = w.x.shape[0]
    Tw = R.shape[0]
    T = Tw if not cpu_trees else min(cpu_trees, Tw)
    t0 = time.perf_counter()
    f = oracle.build_forest(w.x, R, T, w.leaf_size)
    t_build = (time.perf_counter() - t0) * (Tw / T)
    t0 = time.perf_counter()
    oracle.all_knn(f, K, points=sample_pts)
    t_knn = (time.perf_counter() - t0) * (n / len(sample_pts)) * (Tw / T)
    out = {"value": round(n / (t_build + t_knn), 1), "unit": "queries/s", "cores": oracle.threads(),
           "kind": "oracle", "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "sample": f"build of {T} of {Tw} trees on all {n} points (scaled by {Tw}/{T}) + "
                     f"kNN of {len(sample_pts)} sampled points extrapolated to {n}",
           "build_s": round(t_build, 2), "knn_s_extrapolated": round(t_knn, 2)}
    # one thread: a child process with OMP_NUM_THREADS=1 (the thread count is fixed per process)
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; "
            "from paper_1812_11689_amd import workloads as W; "
            "w = W.make_config(2, n=%d); L = oracle.depth(w.x.shape[0], w.leaf_size); "
            "R = W.directions(w.dir_seed, 2, (1 << L) - 1, 1, w.x.shape[1]); "
            "t0 = time.perf_counter(); f = oracle.build_forest(w.x, R, 2, w.leaf_size); tb = time.perf_counter() - t0; "
            "p = np.sort(np.random.default_rng(5).choice(w.x.shape[0], 200, replace=False)); "
            "t0 = time.perf_counter(); oracle.all_knn(f, %d, points=p); tk = time.perf_counter() - t0; "
            "print(oracle.threads(), tb, tk)") % (ROOT, n, K)
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        th, tb, tk = r.stdout.split()[-3:]
        b1 = float(tb) * Tw / 2
        k1 = float(tk) * (n / 200) * (Tw / 2)
        out["one_thread"] = {"value": round(n / (b1 + k1), 1), "cores": int(th), "build_s": round(b1, 1),
                             "knn_s_extrapolated": round(k1, 1),
                             "sample": f"build of 2 of {Tw} trees on all {n} points (scaled) + kNN of 200 sampled "
                                       f"points on those 2 trees (scaled to {Tw} trees and {n} points)"}
    except Exception as e:  # the all-cores figure stands on its own
        out["one_thread"] = {"error": str(e)[:200]}
    return out


if __name__ == "__main__":
    main()
