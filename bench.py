#!/usr/bin/env python3
"""GraphCage / TOCAB benchmark on one MI355X.

Metric: GTEPS per PageRank iteration (arcs / time per iteration), TOCAB
pull vs plain pull on the same GPU, and the fraction of HBM peak reached by
the dominant kernel. Workload: directed R-MAT graph of scale 24 (edge factor
16, a/b/c/d = .57/.19/.19/.05, seeded, labels permuted, self-loops and
duplicates removed), int32 CSR, FP32 ranks, damping 0.85, uniform dangling
redistribution. One step = one PageRank iteration over the whole graph; the
K timed steps run as one pagerank_iter call of K iterations on a resident
graph and partition (inputs already in HBM).

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS per PageRank iter and BFS/SSSP, TOCAB vs plain pull; % of HBM peak"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(name, n, m, info):
    """Algorithmic bytes one launch of `name` must move (each needed value once)."""
    P, B, k = info.get("P", 0), info.get("B", 0), info.get("k", 1)
    R = -(-n // k) if k else 0
    if name == "pr_tocab_pull":  # col + row_ptr + partial writes + one fill of every c slice
        return 4 * m + 4 * (P + 1) + 4 * P + 4 * n
    if name == "pr_merge":  # partials + id_map + range table + outdeg (rowptr) + c' writes
        return 4 * P + 4 * P + 4 * (R + 1) * B + 4 * (n + 1) + 4 * n
    if name == "pr_plain_pull":  # in-CSR + c once + outdeg + c' writes
        return 4 * m + 4 * (n + 1) + 4 * n + 4 * (n + 1) + 4 * n
    if name in ("pr_tocab_push", "pr_plain_push"):  # col + row_ptr (+ id_map) + c + sums line per arc...
        extra = 4 * P if name == "pr_tocab_push" else 0
        rows = P if name == "pr_tocab_push" else n
        return 4 * m + 4 * (rows + 1) + extra + 4 * rows + 8 * n
    if name == "pr_apply":  # sums read+clear, outdeg, c' writes
        return 4 * n + 4 * n + 4 * (n + 1) + 4 * n
    if name == "pr_init":
        return 4 * n + 4 * (n + 1) + 4 * n
    return 0


def run_form(gc, torch, g, part, plain_dir, n, m, steps, warmup):
    rin = torch.full((n,), 1.0 / n, dtype=torch.float32, device="cuda")
    rout = torch.empty_like(rin)
    gc.pagerank_iter(g, part, plain_dir, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, warmup)
    torch.cuda.synchronize()
    gc.gc_profile(1)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    gc.pagerank_iter(g, part, plain_dir, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, steps)
    stop.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    gc.gc_profile(0)
    prof = gc.gc_profile_read()
    ev_ms = start.elapsed_time(stop)
    ranks = rout.double()
    checks = {"sum": float(ranks.sum().item()), "min": float(ranks.min().item())}
    return {"ms_per_step": wall_ms / steps, "event_ms_per_step": ev_ms / steps,
            "gteps": m / (wall_ms / steps * 1e-3) / 1e9, "kernels": prof, "checks": checks}


def run_traversal(gc, torch, g, gh, part, sources, kind, policies):
    """Times BFS or SSSP from each source under each (name, policy, uses
    partition) entry. GTEPS per source (Graph500 style) = out-arcs of the
    reached vertices / time; reported as the harmonic mean over sources."""
    outdeg = np.diff(gh.rowptr).astype(np.int64)
    buf = torch.empty(gh.n, dtype=torch.int32, device="cuda")
    fn = gc.bfs_pull if kind == "bfs" else gc.sssp_pull
    out = {}
    for name, policy, use_part in policies:
        rates, times, levels = [], [], []
        for src in sources:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lv = fn(g, part if use_part else None, int(src), buf, policy)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            reached = buf.cpu().numpy() != gc.GC_UNREACHED
            arcs = int(outdeg[reached].sum())
            rates.append(arcs / dt / 1e9)
            times.append(dt * 1e3)
            levels.append(lv)
        hm = len(rates) / sum(1.0 / r for r in rates)
        out[name] = {"gteps_hmean": round(hm, 3), "ms_mean": round(float(np.mean(times)), 3),
                     "levels": levels}
        log(f"{kind} {name}: {hm:.2f} GTEPS (harmonic mean), {np.mean(times):.2f} ms mean, levels {levels}")
    return out


def traffic_from_profiles(kernel, src_file):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, or None
    when the kernel's source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    want = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    got = hashlib.sha256(open(src_file, "rb").read()).hexdigest()
    if not want or want.group(1) != got:
        return None
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    return float(b.group(1)) if b else None


def cpu_baseline(g, budget_s):
    import oracle
    r0 = np.full(g.n, 1.0 / g.n)
    t0 = time.perf_counter()
    oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 1, r0=r0)
    one = time.perf_counter() - t0
    iters = max(1, min(20, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, iters, r0=r0)
    dt = time.perf_counter() - t0
    return {"value": g.m * iters / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 single-thread oracle PageRank, {iters} of 20 iterations on the full graph "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--block-width", type=int, default=1 << 18)
    ap.add_argument("--merge-range", type=int, default=4096)
    ap.add_argument("--forms", default="tocab_pull,plain_pull,tocab_push,plain_push",
                    help="comma list; the first is the headline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bfs-sources", type=int, default=8, help="BFS sources on the same graph (0 = skip)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run a 1 GiB torch copy first (counter scale reference)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures a single GPU only: --gpus above 1 is not supported by this build",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as gg
    import paper_1904_02241_amd as gc

    torch.cuda.init()
    if args.traffic_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log(f"generating RMAT scale {args.scale}")
    t0 = time.perf_counter()
    gh = gg.rmat(args.scale, args.edge_factor, seed=1)
    n, m = gh.n, gh.m
    log(f"n={n} m={m} ({time.perf_counter() - t0:.1f} s, {gg.threads()} threads)")
    t0 = time.perf_counter()
    g = gc.graph_load_csr(gh.rowptr, gh.colidx)
    log(f"graph_load_csr {time.perf_counter() - t0:.2f} s")
    parts = {}
    forms = args.forms.split(",")
    results = {}
    for form in forms:
        part, plain_dir = None, gc.GC_PULL
        if form.startswith("tocab"):
            d = gc.GC_PULL if form == "tocab_pull" else gc.GC_PUSH
            if d not in parts:
                t0 = time.perf_counter()
                parts[d] = gc.tocab_partition(g, d, args.block_width, args.merge_range)
                log(f"tocab_partition {form} {parts[d].info} {time.perf_counter() - t0:.2f} s")
            part = parts[d]
        elif form == "plain_push":
            plain_dir = gc.GC_PUSH
        res = run_form(gc, torch, g, part, plain_dir, n, m, args.steps, args.warmup)
        res["partition"] = part.info if part else None
        results[form] = res
        log(f"{form}: {res['ms_per_step']:.3f} ms/iter, {res['gteps']:.1f} GTEPS, {res['checks']}")

    traversal = None
    if args.bfs_sources > 0:
        if gc.GC_PULL not in parts:
            parts[gc.GC_PULL] = gc.tocab_partition(g, gc.GC_PULL, args.block_width, args.merge_range)
        srcs = gg.sources(gh, args.bfs_sources, seed=2)
        pols = [("plain_pull", gc.GC_POLICY_PULL, False), ("tocab_pull", gc.GC_POLICY_PULL, True),
                ("push", gc.GC_POLICY_PUSH, False), ("heuristic_tocab", gc.GC_POLICY_HEURISTIC, True),
                ("heuristic_plain", gc.GC_POLICY_HEURISTIC, False)]
        traversal = {"bfs": run_traversal(gc, torch, g, gh, parts[gc.GC_PULL], srcs, "bfs", pols),
                     "sources": [int(x) for x in srcs]}

    head = forms[0]
    hres = results[head]
    info = hres["partition"] or {}
    kern = {k: v for k, v in hres["kernels"].items() if k not in ("pr_init", "pr_dangling")}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms = kern[dom][0] / kern[dom][1]
    per_launch = kernel_bytes(dom, n, m, info)
    achieved = per_launch / (dom_ms * 1e-3) / 1e9
    src = os.path.join(ROOT, "paper_1904_02241_amd", "csrc", "gc_pagerank.hip")
    traffic = traffic_from_profiles(dom, src)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "kernel_ms": round(dom_ms, 4), "algorithmic_bytes_per_launch": per_launch}
    step_bytes = sum(kernel_bytes(k, n, m, info) * v[1] for k, v in hres["kernels"].items()) / args.steps
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(gh, args.cpu_seconds)
        log(f"cpu baseline {cpu}")
    forms_out = {}
    for f, r in results.items():
        forms_out[f] = {"gteps": round(r["gteps"], 2), "ms_per_iter": round(r["ms_per_step"], 4),
                        "kernels_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in r["kernels"].items()},
                        "rank_sum": r["checks"]["sum"]}
    if "plain_pull" in results:
        forms_out["tocab_pull_over_plain_pull"] = round(results[head]["gteps"] / results["plain_pull"]["gteps"], 3)
    out = {
        "metric": METRIC, "value": round(hres["gteps"], 2), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(hres["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"pagerank_{head}_rmat{args.scale}", "graph": "rmat", "scale": args.scale,
                   "edge_factor": args.edge_factor, "n": n, "m": m, "block_width": args.block_width,
                   "merge_range": args.merge_range, "damping": 0.85, "dangling": "uniform",
                   "P": info.get("P"), "B": info.get("B")},
        "roofline": roofline,
        "step_algorithmic_GBs": round(step_bytes / (hres["ms_per_step"] * 1e-3) / 1e9, 1),
        "cpu_baseline": cpu,
        "forms": forms_out,
        "traversal": traversal,
    }
    print(json.dumps(out), flush=True)
    for p in parts.values():
        p.free()
    g.free()


if __name__ == "__main__":
    main()
