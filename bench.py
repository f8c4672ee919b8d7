#!/usr/bin/env python3
"""Throughput benchmark of the QIEO generation on one MI355X.

A step is one generation of the whole loop (CIP of the previous generation,
QIP, Evaluation, DetermineElite, fused in one launch) over the resident
population of the largest single-instance workload: Np = 4096 chromosomes of
Ng = 200,000 items (weights U[1,100], value = weight + 10, capacity =
floor(sum/2), seed 2).  The default K = 200 steps is that workload's whole
generation budget.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 200] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, 8.0 TB/s
BYTES_PER_GENE_UPDATE = 16      # binary32 (alpha, beta) read + write
KERNEL_SOURCES = ["paper_2609_30862_amd/csrc/qieo_kernels.hip",
                  "paper_2609_30862_amd/csrc/qieo_device.hpp",
                  "paper_2609_30862_amd/csrc/qieo_kernels.hpp"]
PROFILE = "profiles/generation_kernel_np4096_ng200000.md"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(n_pop: int, n_items: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on this workload with the current kernel sources; else None."""
    import hashlib
    if (n_pop, n_items) != (4096, 200_000):
        return None
    try:
        text = open(os.path.join(ROOT, PROFILE)).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        fig = dict(line.strip().split(": ", 1) for line in text.splitlines()
                   if line.strip().startswith(("traffic_bytes_per_launch:", "kernel_source_sha256:")))
        if fig.get("kernel_source_sha256") != h.hexdigest():
            return None
        return float(fig["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(inst, rows: int, gens: int):
    """The CPU oracle, untuned and single-threaded, on a bounded sample of the
    same workload: the first `rows` chromosomes of the population over the
    full item list, for `gens` generations."""
    import oracle
    o = oracle.Oracle(inst.values, inst.weights, inst.capacity, rows, inst.seed, threads=1)
    o.run(1)                    # generation 0 observes only; time full generations
    t0 = time.perf_counter()
    o.run(gens)
    dt = time.perf_counter() - t0
    return {"value": rows * inst.n_items * gens / dt, "unit": "gene-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": "first %d of %d chromosomes x %d items, %d generations after "
                      "generation 0, %.1f s" % (rows, inst.n_pop, inst.n_items, gens, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-pop", type=int, default=4096)
    ap.add_argument("--n-items", type=int, default=200_000)
    ap.add_argument("--tile", type=str, default="", help="R,S work shape override")
    ap.add_argument("--kernel-flags", type=int, default=-1, help="generation kernel variant")
    ap.add_argument("--cpu-rows", type=int, default=256)
    ap.add_argument("--cpu-gens", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (to scale HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(instances are independent; see the sharding design). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2609_30862_amd import qieo

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB x 5" % args.copy_calibration)
        return
    inst = workloads.large_instance(args.n_pop, args.n_items)
    log("workload %s, %d steps, %d warmup" % (inst.name, args.steps, args.warmup))
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    if args.tile:
        r, s = (int(x) for x in args.tile.split(","))
        g.set_tile(r, s)
    if args.kernel_flags >= 0:
        g.set_kernel_flags(args.kernel_flags)
    log("work shape rows/block, waves/block = %s" % (g.tile(),))
    g.step(args.warmup)

    g.set_timing(True)
    g.kernel_time(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step_async(args.steps)
    g.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, kern_ms = g.kernel_time(reset=True)
    g.set_timing(False)

    genes = inst.n_pop * inst.n_items
    value = genes * args.steps / wall
    avg_ms = kern_ms / max(launches, 1)
    bytes_per_launch = BYTES_PER_GENE_UPDATE * genes
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    best = g.best()
    log("wall %.3f s, %.3f ms/generation, kernel avg %.3f ms over %d launches, "
        "%.1f GB/s algorithmic, best fitness %d (gen %d)"
        % (wall, wall / args.steps * 1e3, avg_ms, launches, achieved, best.fitness,
           best.generation))
    g.close()

    out = {
        "metric": "gene-updates/s",
        "value": value,
        "unit": "gene-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "qieo-knapsack single instance Np=%d Ng=%d, %d generations"
                               % (inst.n_pop, inst.n_items, args.steps),
                   "n_pop": inst.n_pop, "n_items": inst.n_items, "seed": inst.seed,
                   "generations_per_step": 1},
        "hbm_frac_algorithmic": value * BYTES_PER_GENE_UPDATE / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(inst.n_pop, inst.n_items),
                     "kernel": "generation_kernel", "kernel_avg_ms": avg_ms,
                     "bytes_per_launch": bytes_per_launch},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on %d rows x %d generations" % (args.cpu_rows, args.cpu_gens))
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_rows, args.cpu_gens)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
