"""Benchmark of the alpha-CNG hot path on one MI355X.

One step = the whole path on one batch of synthetic input: build the graph
(entry point, exact candidates, pruning, connectivity) over the base set, then
search the query batch at the beam width that reaches recall@10 >= 0.95.
Inputs are resident in HBM before the timed region starts.

Default workload: 1,000,000 x 128 integer-valued vectors in [0, 255] from a
16-dim latent model (SIFT-shaped stand-in), 10,000 queries, R=32, C=128,
alpha=1.2, tau=0, k=10, L swept over 16..256.

Prints ONE JSON line:  value = search QPS (queries / median search-kernel time)
at the chosen L; build seconds, recall, the HBM roofline of the search kernel,
the MFMA roofline of the candidate filter and the CPU-oracle baseline ride
along.
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

HBM_PEAK_GBS = 8000.0
FP32_MFMA_TFLOPS = 157.3
BF16_MFMA_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--L", type=int, default=0, help="fixed beam width (skip the sweep)")
    ap.add_argument("--search-reps", type=int, default=10)
    ap.add_argument("--visited-log2", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--search-only", action="store_true",
                    help="time only the search leg (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (scale for HBM byte counters)")
    return ap.parse_args()


def recall(ids, gt_ids, gt_dist_k, res_dist):
    """strict: |GT_k & Res| / k;  tie-aware: results whose distance is at most the
    k-th true one (both as float32 sqrt of the same fixed-order D, so a point tied
    with the k-th neighbour counts)."""
    k = gt_ids.shape[1]
    strict = np.mean([len(set(a.tolist()) & set(b.tolist())) / k for a, b in zip(ids, gt_ids)])
    tie = np.mean(np.minimum((res_dist <= gt_dist_k[:, None]).sum(1), k) / k)
    return float(strict), float(tie)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import paper_2510_05975_amd as cng
    import workloads

    cfg = workloads.CONFIGS[a.config]
    n = a.n or cfg["n"]
    nq = a.nq or cfg["nq"]
    R, Cc, alpha, tau, k = cfg["R"], cfg["C"], cfg["alpha"], cfg["tau"], cfg["k"]
    dev = "cuda:0"
    t = time.time()
    x, q = workloads.generate(a.config, n=n, nq=nq)
    gen_s = time.time() - t
    d = x.shape[1]
    print(f"# generated {n}x{d} + {nq} queries in {gen_s:.1f}s", file=sys.stderr, flush=True)
    xd = torch.from_numpy(x).to(dev)
    qd = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()

    # exact ground truth on the GPU (the same exact-candidate stage, queries as rows)
    t = time.time()
    gt_ids_t, gt_D_t, _ = cng.knn(qd, xd, k)
    torch.cuda.synchronize()
    gt_ids = cng.u32(gt_ids_t)
    gt_dk = np.sqrt(gt_D_t.cpu().numpy()[:, k - 1]).astype(np.float32)  # IEEE sqrt, as the search
    print(f"# ground truth in {time.time() - t:.1f}s", file=sys.stderr, flush=True)

    def build():
        return cng.build(xd, R, Cc, alpha, tau)

    def search(g, L, vlog2=a.visited_log2, stats=False):
        return cng.search(xd, g.adj, qd, k, L, g.entry, visited_log2=vlog2, stats=stats)

    g = build()
    torch.cuda.synchronize()
    print(f"# build {g.stats}", file=sys.stderr, flush=True)

    # ---- beam sweep: the smallest L with tie-aware recall@10 >= 0.95
    sweep = []
    Ls = [a.L] if a.L else cfg["L"]
    chosen = None
    for L in Ls:
        ids, dists, hops, ndc = search(g, L, vlog2=14, stats=True)
        torch.cuda.synchronize()
        s, tw = recall(cng.u32(ids), gt_ids, gt_dk, dists.cpu().numpy())
        row = dict(L=L, recall_strict=round(s, 4), recall_tie=round(tw, 4),
                   hops=float(hops.float().mean()), ndc=float(ndc.float().mean()))
        sweep.append(row)
        print(f"# sweep {row}", file=sys.stderr, flush=True)
        if chosen is None and tw >= 0.95:
            chosen = row
            if not a.L:
                break
    if chosen is None:
        chosen = sweep[-1]
    L = chosen["L"]
    # algorithmic work of one query batch (no repeated evaluations)
    _, _, hops_t, ndc_t = search(g, L, vlog2=14, stats=True)
    torch.cuda.synchronize()
    ndc_alg = ndc_t.double().sum().item()
    hops_alg = hops_t.double().sum().item()
    W = g.adj.shape[1]
    alg_bytes = ndc_alg * d * 4 + hops_alg * W * 4 + nq * d * 4 + nq * k * 8

    # ---- warmup + timed steps
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def one_step():
        out = {}
        if not a.search_only:
            t0 = time.perf_counter()
            gb = build()
            out["build_s"] = time.perf_counter() - t0
            out["stats"] = gb.stats
        else:
            gb = g
        times = []
        for _ in range(a.search_reps):
            ev0.record(stream)
            search(gb, L)
            ev1.record(stream)
            ev1.synchronize()
            times.append(ev0.elapsed_time(ev1))
        out["search_ms"] = float(np.median(times))
        return out

    if a.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(a.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = [one_step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    search_ms = float(np.median([s["search_ms"] for s in steps]))
    qps = nq / (search_ms / 1e3)
    achieved = alg_bytes / (search_ms / 1e3) / 1e9
    out = {
        "metric": "search QPS at recall@10=0.95 (plain FP32); build secs",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "d": d, "nq": nq, "R": R, "C": Cc,
                   "alpha": alpha, "tau": tau, "k": k, "L": L, "row_width": W},
        "recall@10": chosen["recall_tie"],
        "recall@10_strict": chosen["recall_strict"],
        "search_ms": round(search_ms, 4),
        "hops_mean": hops_alg / nq,
        "ndc_mean": ndc_alg / nq,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "sweep": sweep,
    }
    if not a.search_only:
        bs = [s["build_s"] for s in steps]
        st = steps[-1]["stats"]
        cand_s = float(np.median([s["stats"]["ms_candidates"] for s in steps])) / 1e3
        flops_alg = float(n) * (n - 1) * d        # n(n-1)/2 pairs x 2d
        tflops = flops_alg / cand_s / 1e12
        peak = BF16_MFMA_TFLOPS if st.get("filter_dtype") == 1 else FP32_MFMA_TFLOPS
        out["build_secs"] = round(float(np.median(bs)), 4)
        out["build_stages_ms"] = {kk: round(st[kk], 2) for kk in
                                  ("ms_entry", "ms_candidates", "ms_prune", "ms_connect")}
        out["build_info"] = {kk: st[kk] for kk in ("connect_rounds", "connect_added",
                                                    "overflow_rows", "exact_integer",
                                                    "filter_dtype")}
        out["roofline_build"] = {"bound": "mfma", "achieved": round(tflops, 2), "peak": peak,
                                 "unit": "TFLOP/s", "frac": round(tflops / peak, 4),
                                 "kernel": "candidate stage (filter GEMM + rerank)",
                                 "traffic": None}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x, q, cng.u32(g.adj), g.entry, k, L, a.cpu_seconds)
    print(json.dumps(out))


def cpu_baseline(x, q, adj, entry, k, L, budget_s):
    """The oracle as it stands, on the host cores: search QPS on a bounded
    sample of the same queries and graph."""
    import oracle
    threads = oracle.max_threads()
    m = 64
    t = time.perf_counter()
    oracle.search(x, adj, q[:m], k, L, entry)
    dt = time.perf_counter() - t
    # grow the sample to roughly the time budget
    m2 = int(min(len(q), max(m, m * budget_s / max(dt, 1e-3))))
    if m2 > m:
        t = time.perf_counter()
        oracle.search(x, adj, q[:m2], k, L, entry)
        dt = time.perf_counter() - t
        m = m2
    return {"value": round(m / dt, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} of the {len(q)} queries, same graph and L, FP32 mode, {dt:.1f}s"}


if __name__ == "__main__":
    main()
