#!/usr/bin/env python3
"""Benchmark of the rpForests kNN path on one MI355X.

One step = the whole hot path on one batch: grow the forest (rpf_build) over the
1M x 128 anisotropic Gaussian mixture (T = 32 trees, leaf size 256) and find the K = 20
nearest neighbours of every point among the union of its leaves (rpf_all_knn), then
release the forest.  Inputs are resident in device memory before the timed region.

Prints one JSON line: whole-job throughput in queries/s (points whose exact top-K over
the leaf union is produced per second) with binary32 tiles, the same with bfloat16 tiles
plus re-rank, the recall against exact brute force on a sample of points, the roofline
of the dominant kernel (timed with HIP events on the launch stream, inside the library)
and the CPU oracle timed on the host.
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
TRAFFIC_FILE = os.path.join(PROFILES, "hbm_traffic_allknn_1M_d128_T32.md")
# kernel behind each timed record of the library, for the fp32 run of the 1M x 128 workload
RECORD_KERNEL = {
    "tile_phase2": "k_tile_sym<8, 0, 1>",
    "tile_phase1": "k_tile_sym<8, 0, 0>",
    "proj_chunks": "k_proj_chunks<true>",
    "level_small": "k_level_small<true>",
    "leaf_finalize": "k_leaf_finalize<float>",
    "merge_first": "k_merge_first<16>",
    "final_rerank": "k_final<true, 12>",
}
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="fewer points (same recipe), for quick checks")
    ap.add_argument("--recall-sample", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the recorded-plan (HIP graph) leg")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script with "
                         "--copy-probe into per-kernel HBM traffic (markdown on stdout) and exit")
    ap.add_argument("--kt-summary", metavar="DIR", help="summarise a rocprofv3 --kernel-trace --stats run "
                                                        "(markdown on stdout) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference kernel for HBM counters)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--only-serve", action="store_true", help="run the serving leg alone (profiling)")
    ap.add_argument("--serve-n", type=int, default=None, help="points of the served forest (default: 4M)")
    ap.add_argument("--serve-requests", type=int, default=4000, help="requests per serving measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-data-sets leg")
    ap.add_argument("--only-batched", action="store_true", help="run the many-data-sets leg alone (profiling)")
    ap.add_argument("--batch-count", type=int, default=512, help="data sets of the many-data-sets leg")
    ap.add_argument("--cpu-sample", type=int, default=20000,
                    help="points whose all-points kNN the CPU baseline times (extrapolated to n)")
    ap.add_argument("--target-recall", type=float, default=0.99,
                    help="recall the at-target leg looks for by growing more trees (0 = skip the leg)")
    ap.add_argument("--target-trees", default="48,64,80,96,128",
                    help="tree counts the at-target leg tries, in order (the first T trees are the bench's)")
    ap.add_argument("--cpu-trees", type=int, default=0,
                    help="trees the CPU baseline builds (its time is scaled to all trees; 0 = all)")
    return ap.parse_args()


def exact_knn_sample(X, pts, K):
    """Exact K nearest neighbours (excluding self) of the sampled points, by binary64
    distances on the device -- the ground truth of the recall measurement."""
    import torch
    Xd = X.double()
    nrm = (Xd * Xd).sum(1)
    out = []
    for s in range(0, len(pts), 256):
        p = pts[s:s + 256]
        q = Xd[p]
        D = nrm[p][:, None] + nrm[None, :] - 2.0 * (q @ Xd.T)
        D[torch.arange(len(p)), p] = float("inf")
        out.append(torch.topk(D, K, dim=1, largest=False).indices)
    return torch.cat(out).cpu().numpy()


def recall_of(found, truth):
    hit = 0
    for f, t in zip(found, truth):
        hit += len(set(f.tolist()) & set(t.tolist()))
    return hit / truth.size


def roofline(prof):
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
    if r["algo_flops"] > 0:
        peak = BF16_MFMA_PEAK_TFLOPS if r.get("prec") == "bf16" else FP32_MFMA_PEAK_TFLOPS
        ach = r["algo_flops"] / r["launches"] / avg_s / 1e12
        return best, {"bound": "mfma", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
                      "frac": round(ach / peak, 4), "traffic": None}
    ach = r["algo_bytes"] / r["launches"] / avg_s / 1e9
    return best, {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}


BUILD_LEVEL_RECORDS = ("proj_roots", "proj_chunks_x3", "level_small", "select_passes", "partition")
KNN_RECORDS = ("tile_phase1", "merge_first", "tile_phase2", "final_rerank", "fallback")


def stage_summary(prof, steps, n, d, T, L, K):
    """Kernel time of the two halves of a step and their bounds: the build levels against the
    algorithmic bytes of the method (n (4d + 36) bytes per tree and level: row, id, key write,
    one select read, partition read of key and id, id write), the leaf pass apart, and the
    search (queries/s of rpf_all_knn alone) with the MFMA fraction of its distance tiles."""
    def ms(names):
        return sum(prof[k]["total_ms"] for k in names if k in prof) / steps
    lv_ms, leaf_ms, knn_ms = ms(BUILD_LEVEL_RECORDS), ms(("leaf_finalize",)), ms(KNN_RECORDS)
    lv_bytes = float(n) * (4 * d + 36) * L * T
    tiles = [prof[k] for k in ("tile_phase1", "tile_phase2") if k in prof]
    t_flops = sum(r["algo_flops"] for r in tiles) / steps
    t_ms = sum(r["total_ms"] for r in tiles) / steps
    peak = FP32_MFMA_PEAK_TFLOPS if not tiles or tiles[0].get("prec") != "bf16" else BF16_MFMA_PEAK_TFLOPS
    return {
        "build_levels_ms": round(lv_ms, 3),
        "build_levels_algorithmic_bytes": lv_bytes,
        "build_levels_effective_hbm_frac": round(lv_bytes / (lv_ms / 1e3) / (HBM_PEAK_GBS * 1e9), 3) if lv_ms else None,
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


def kt_summary(d):
    rows = _csv_rows(d, "kernel_stats.csv")
    print("| kernel | calls | total ms | average us | share |")
    print("|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:20]:
        print(f"| {_short(r['Name'])[:70]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")


def traffic_for(record):
    """HBM bytes per launch of a timed record, from the committed counter summary, or None
    when there is none or the kernels changed since it was taken."""
    kname = RECORD_KERNEL.get(record)
    if not kname or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        js = [ln for ln in fh if ln.startswith("{")]
    if not js:
        return None
    t = json.loads(js[-1])
    if t.get("source_hash") != source_hash():
        return None
    k = t["kernels"].get(kname)
    return None if k is None else k["bytes_per_dispatch"]


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.kt_summary:
        kt_summary(args.kt_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding "
                                   "by trees is a design note only)"}))
        sys.exit(2)
    import torch
    from paper_1812_11689_amd import rpf
    from paper_1812_11689_amd import workloads as W

    if args.only_serve:
        print(json.dumps({"serving": serving_leg(args)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": batched_leg(args)}), flush=True)
        return
    t0 = time.time()
    w = W.make_config(2, n=args.n)
    n, d = w.x.shape
    T, n0, K = w.n_trees, w.leaf_size, w.k
    L = rpf.depth(n, n0)
    R = W.directions(w.dir_seed, T, (1 << L) - 1, 1, d)
    X = torch.from_numpy(w.x).cuda()
    Rd = torch.from_numpy(R).cuda()
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    print(f"# workload {w.name}: n={n} d={d} T={T} n0={n0} K={K} L={L} (generated in {gen_s:.1f}s)",
          file=sys.stderr, flush=True)

    if args.copy_probe:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written", file=sys.stderr, flush=True)
        del src, dst

    def step(prec):
        f = rpf.build(X, T, n0, Rd, dist_prec=prec)
        idx, dist = f.all_knn(K)
        f.free()
        return idx, dist

    def measure(prec, steps, warmup):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        rpf.profile_reset()
        rpf.profile_enable(True)
        times = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            idx, dist = step(prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        rpf.profile_enable(False)
        prof = rpf.profile_read()
        return idx, dist, elapsed, times, prof

    idx32, _, el32, times32, prof32 = measure("fp32", args.steps, args.warmup)
    print(f"# fp32: {el32 / args.steps * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    res_bf16 = None
    if not args.no_bf16:
        idx16, _, el16, times16, prof16 = measure("bf16", args.steps, 1)
        print(f"# bf16: {el16 / args.steps * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
        same = bool(torch.equal(idx16, idx32))
        res_bf16 = dict(value=round(n * args.steps / el16, 1), ms_per_step=round(el16 / args.steps * 1e3, 3),
                        identical_to_fp32=same,
                        breakdown_ms_per_step={k: round(v["total_ms"] / args.steps, 3) for k, v in
                                               sorted(prof16.items(), key=lambda kv: -kv[1]["total_ms"])})

    # the same job as one recorded HIP graph (rpf_plan_*: build and candidate stage, tuned
    # first-phase tree count), inputs set once before the timed launches
    def plan_leg(prec, ref_idx, n_trees=None, dirs=None):
        plan = rpf.Plan([n], [d], n_trees or T, n0, K, dist_prec=prec)
        try:
            plan.set_inputs([X], [Rd if dirs is None else dirs])
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
            same = bool(torch.equal(plan.result(0)[0], ref_idx))
            return dict(value=round(n * args.steps / el, 1), ms_per_step=round(el / args.steps * 1e3, 3),
                        first_trees=plan.parts[0].get("first_trees"), identical_to_plain=same)
        finally:
            plan.close()

    graph = None
    if not args.no_graph:
        graph = {"fp32": plan_leg("fp32", idx32)}
        if res_bf16 is not None:
            graph["bf16"] = plan_leg("bf16", idx16)
        print(f"# recorded plan: {graph}", file=sys.stderr, flush=True)

    # recall against exact brute force on a seeded sample of points
    rng = np.random.default_rng(W.SEED_BASE + 300 + 2)
    pts = np.sort(rng.choice(n, size=min(args.recall_sample, n), replace=False))
    truth = exact_knn_sample(X, torch.from_numpy(pts).cuda(), K)
    recall = recall_of(idx32.cpu().numpy()[pts], truth)

    # queries/s at the target recall: the same points and the same first T trees, plus more
    # trees of the same direction streams (tree t always uses stream (seed, t)), until the
    # sampled recall reaches the target; then the fp32 and bf16 steps are timed at that T
    target = None
    if args.target_recall > 0:
        sweep, Rt, hit = [], R, None
        for Tt in [int(v) for v in args.target_trees.split(",") if int(v) > T]:
            extra = W.directions(w.dir_seed, Tt - Rt.shape[0], (1 << L) - 1, 1, d, first_tree=Rt.shape[0])
            Rt = np.concatenate([Rt, extra])
            Rtd = torch.from_numpy(Rt).cuda()
            f = rpf.build(X, Tt, n0, Rtd, dist_prec="fp32")
            it, _ = f.all_knn(K)
            st_t = f.knn_stats()
            f.free()
            r_t = recall_of(it.cpu().numpy()[pts], truth)
            sweep.append({"n_trees": Tt, "recall": round(r_t, 5), "fallback_rows": st_t.get("fallback_rows")})
            print(f"# target leg: T={Tt} recall {r_t:.4f}", file=sys.stderr, flush=True)
            if r_t >= args.target_recall:
                hit = (Tt, Rtd, r_t, it)
                break
            del Rtd
        target = {"target": args.target_recall, "sweep": sweep, "n_trees": None}
        if hit is not None:
            Tt, Rtd, r_t, it = hit

            def step_t(prec):
                f = rpf.build(X, Tt, n0, Rtd, dist_prec=prec)
                out = f.all_knn(K)
                f.free()
                return out

            def time_t(prec, steps=3):
                step_t(prec)
                torch.cuda.synchronize()
                rpf.profile_reset()
                rpf.profile_enable(True)
                t = time.perf_counter()
                for _ in range(steps):
                    ib, _ = step_t(prec)
                torch.cuda.synchronize()
                el = (time.perf_counter() - t) / steps
                rpf.profile_enable(False)
                pr = rpf.profile_read()
                bd = {k: round(v["total_ms"] / steps, 3) for k, v in sorted(pr.items(), key=lambda kv: -kv[1]["total_ms"])}
                return ib, {"value": round(n / el, 1), "ms_per_step": round(el * 1e3, 3), "breakdown_ms_per_step": bd}

            i32, t32 = time_t("fp32")
            t32["identical_to_sweep"] = bool(torch.equal(i32, it))
            target.update(n_trees=Tt, recall=round(r_t, 5), fp32=t32)
            if not args.no_bf16:
                i16, t16 = time_t("bf16")
                t16["identical_to_fp32"] = bool(torch.equal(i16, i32))
                target["bf16"] = t16
            if not args.no_graph:  # the same step as a tuned, recorded plan (first-phase trees picked)
                target["recorded_plan"] = {"fp32": plan_leg("fp32", i32, Tt, Rtd)}
                if not args.no_bf16:
                    target["recorded_plan"]["bf16"] = plan_leg("bf16", i32, Tt, Rtd)
            print(f"# target leg: {target}", file=sys.stderr, flush=True)
            del Rtd, it

    for name, r in prof32.items():
        r["prec"] = "fp32"
    dom, roof = roofline(prof32)
    if roof is not None and dom is not None:
        tr = traffic_for(dom)
        roof["traffic"] = tr  # HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE), or None
        if tr is not None:
            roof["traffic_source"] = os.path.relpath(TRAFFIC_FILE, ROOT)
    breakdown = {k: round(v["total_ms"] / args.steps, 3) for k, v in sorted(prof32.items(), key=lambda kv: -kv[1]["total_ms"])}
    stages = stage_summary(prof32, args.steps, n, d, T, L, K)

    f = rpf.build(X, T, n0, Rd, dist_prec="fp32")
    f.all_knn(K)
    st = f.knn_stats()
    f.free()

    serving = None
    if not args.no_serve:
        del X, Rd
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
        cpu = cpu_baseline(w, R, cpts, K, args.cpu_trees)

    ms = el32 / args.steps * 1e3
    line = {
        "metric": METRIC,
        "value": round(n * args.steps / el32, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "d": d, "n_trees": T, "leaf_size": n0, "K": K,
                   "tile_prec": "fp32", "split_projection": "f64", "rerank": "fp32+f64"},
        "recall": round(recall, 5),
        "step_ms_p50": round(float(np.percentile(times32, 50)) * 1e3, 3),
        "step_ms_p99": round(float(np.percentile(times32, 99)) * 1e3, 3),
        "bf16_rerank": res_bf16,
        "recorded_plan": graph,
        "at_target_recall": target,
        "knn_stats": st,
        "breakdown_ms_per_step": breakdown,
        "stages": stages,
        "roofline_kernel": dom,
        "roofline": roof,
        "cpu_baseline": cpu,
        "serving": serving,
        "batched": batched,
    }
    print(json.dumps(line), flush=True)


def serving_leg(args):
    """Continuous-batching server over the resident 4M x 96 forest (T 64, n0 256): a closed
    burst of requests gives the saturated rate; an open-loop Poisson stream at 0.8 of it gives
    request latency.  Batch sizes lognormal (median 64, sigma 1.5) in [1, 4096], K uniform over
    {1, 10, 100}; queries from the served mixture with 5 % uniform outliers."""
    import torch
    from paper_1812_11689_amd import rpf
    from paper_1812_11689_amd import workloads as W

    t0 = time.time()
    w = W.make_config(4, n=args.serve_n)
    n, d = w.x.shape
    T, n0 = w.n_trees, w.leaf_size
    L = rpf.depth(n, n0)
    X = torch.from_numpy(w.x).cuda()
    R = torch.from_numpy(W.directions(w.dir_seed, T, (1 << L) - 1, 1, d)).cuda()
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
    res = {"workload": w.name, "requests": nreq, "rows": pool,
           "batch_rows": "lognormal(ln 64, 1.5) in [1, 4096]", "K": "uniform {1, 10, 100}"}

    def run(prec):
        f = rpf.build(X, T, n0, R, dist_prec=prec)
        torch.cuda.synchronize()
        srv = rpf.Server(f, slots=4, max_batch_rows=8192)
        # warm-up
        for q, k in reqs[:64]:
            srv.wait(srv.submit(q, k))
        # closed burst: every request queued at once
        srv.reset_stats()
        ts = [srv.submit(q, k, out=o) for (q, k), o in zip(reqs, outs)]
        for t in ts:
            srv.wait(t)
        burst = srv.stats()
        rate = burst["requests"] / (burst["rows"] / burst["rows_per_s"])  # requests/s at saturation
        # open loop at 0.8 of the saturated request rate
        srv.reset_stats()
        arr, _, _ = W.serving_requests(seed + 1, nreq, 0.8 * rate)
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
        srv.close()
        out = {"saturated_rows_per_s": round(burst["rows_per_s"], 1),
               "saturated_requests_per_s": round(rate, 1),
               "burst_mean_batch_rows": round(burst["mean_batch_rows"], 1),
               "open_loop": {"offered_requests_per_s": round(0.8 * rate, 1),
                             "rows_per_s": round(ol["rows_per_s"], 1),
                             "p50_ms": round(ol["p50_s"] * 1e3, 3), "p99_ms": round(ol["p99_s"] * 1e3, 3),
                             "max_ms": round(ol["max_s"] * 1e3, 3),
                             "mean_batch_rows": round(ol["mean_batch_rows"], 1)}}
        print(f"# serving {prec}: {out}", file=sys.stderr, flush=True)
        return f, out

    f16, res["fp16"] = run("fp16")
    # recall of the fp16 results on the first requests' rows (K as requested)
    Xd = X.double()
    nrm = (Xd * Xd).sum(1)
    hit = tot = 0
    for i in range(nreq):
        if tot >= 1500:
            break
        q, k = reqs[i]
        qd = q[:16].double()  # at most 16 rows of a request: [16][n] binary64 distances
        D = nrm[None, :] - 2.0 * (qd @ Xd.T)
        truth = torch.topk(D, k, dim=1, largest=False).indices.cpu().numpy()
        got = outs[i][0][:16].cpu().numpy()
        for a, b in zip(got, truth):
            hit += len(set(a.tolist()) & set(b.tolist()))
        tot += truth.size
    res["recall_fp16"] = round(hit / max(tot, 1), 5)
    res["recall_sample_neighbours"] = tot
    f16.free()
    del Xd, nrm
    torch.cuda.empty_cache()
    f32, res["fp32"] = run("fp32")
    f32.free()
    return res


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
    res["tuned_candidate_ms"] = round(plan.tune(), 3)
    res["first_trees"] = [pt.get("first_trees") for pt in plan.parts]
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
    # recall of a sample of data sets against exact brute force (binary64 on the device)
    rng = np.random.default_rng(W.SEED_BASE + 305)
    hit = tot = 0
    for i in rng.choice(count, size=min(8, count), replace=False):
        X = torch.from_numpy(xs[i]).cuda().double()
        pts = torch.from_numpy(rng.choice(sizes[i], size=min(300, sizes[i]), replace=False)).cuda()
        D = (X * X).sum(1)[None, :] - 2.0 * (X[pts] @ X.T)
        D[torch.arange(len(pts)), pts] = float("inf")
        truth = torch.topk(D, K, dim=1, largest=False).indices.cpu().numpy()
        got = plan.result(int(i))[0][pts].cpu().numpy()
        for a, b in zip(got, truth):
            hit += len(set(a.tolist()) & set(b.tolist()))
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


def cpu_baseline(w, R, sample_pts, K, cpu_trees):
    """The oracle as it stands, on the host cores: the forest build timed in full on all n
    points (all T trees, or `cpu_trees` of them scaled by T/cpu_trees), plus all-points kNN
    timed on a seeded sample of points and extrapolated linearly to n."""
    import oracle
    oracle.build(force=False)
    n = w.x.shape[0]
    T = w.n_trees if not cpu_trees else min(cpu_trees, w.n_trees)
    t0 = time.perf_counter()
    f = oracle.build_forest(w.x, R, T, w.leaf_size)
    t_build = (time.perf_counter() - t0) * (w.n_trees / T)
    t0 = time.perf_counter()
    oracle.all_knn(f, K, points=sample_pts)
    t_knn = (time.perf_counter() - t0) * (n / len(sample_pts)) * (w.n_trees / T)
    return {"value": round(n / (t_build + t_knn), 1), "unit": "queries/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"build of {T} of {w.n_trees} trees on all {n} points (scaled by {w.n_trees}/{T}) + "
                      f"kNN of {len(sample_pts)} sampled points extrapolated to {n}",
            "build_s": round(t_build, 2), "knn_s_extrapolated": round(t_knn, 2)}


if __name__ == "__main__":
    main()
