#!/usr/bin/env python3
"""Throughput benchmark of the QIEO generation on one MI355X.

A step is one generation of the whole loop (CIP of the previous generation,
QIP, Evaluation, DetermineElite, fused) over the resident population of the
largest single-instance workload: Np = 4096 chromosomes of Ng = 200,000
items (weights U[1,100], value = weight + 10, capacity = floor(sum/2), seed
2), with binary64 amplitudes, the paper's precision (--precision 32 for
binary32).  The default K = 200 steps is that workload's whole generation
budget.  Five timed runs (--repeats), each on a fresh population of the same
seed; the reported figures are the median run's.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 200] [--warmup 3] [--repeats 5] [--precision 64]
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
# (alpha, beta) read and written once per gene-update: 4 amplitudes
AMPLITUDES_PER_GENE_UPDATE = 4
KERNEL_SOURCES = ["paper_2609_30862_amd/csrc/qieo_kernels.hip",
                  "paper_2609_30862_amd/csrc/qieo_device.hpp",
                  "paper_2609_30862_amd/csrc/qieo_elite.hpp",
                  "paper_2609_30862_amd/csrc/qieo_kernels.hpp",
                  "paper_2609_30862_amd/csrc/qieo_layout.hpp"]
PROFILE = "profiles/generation_kernel_np4096_ng200000.md"
# the on-chip loop's sources and its instruction-count summary
ONCHIP_SOURCES = ["paper_2609_30862_amd/csrc/qieo_onchip.hip",
                  "paper_2609_30862_amd/csrc/qieo_onchip.hpp",
                  "paper_2609_30862_amd/csrc/qieo_device.hpp",
                  "paper_2609_30862_amd/csrc/qieo_elite.hpp",
                  "paper_2609_30862_amd/csrc/qieo_host.hpp",
                  "paper_2609_30862_amd/csrc/qieo_layout.hpp"]
ONCHIP_PROFILE = "profiles/onchip_kernel_np1024_ng10000.md"
BATCH_PROFILE = "profiles/batch_512_ragged.md"
# vector ALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one non-packed instruction per lane and cycle), in G lane-instructions/s
VALU_PEAK_G = 256 * 4 * 16 * 2.4
# kernels of the whole-call paths (qieo_get_call_path 1, 2, 3)
PATH_KERNELS = {1: "resident_kernel (one launch per call)",
                2: "persistent_kernel (one launch per call)",
                3: "onchip_kernel (one cooperative launch per call)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_code_digest(read=None, sources=None) -> str:
    """sha256 of the kernel sources' code: each line with its // comment and
    surrounding blanks removed, empty lines dropped (comments do not change
    what the counters measured).  read(path) -> text, default: the tree."""
    import hashlib
    h = hashlib.sha256()
    for f in (sources or KERNEL_SOURCES):
        text = read(f) if read else open(os.path.join(ROOT, f)).read()
        for line in text.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def onchip_valu_per_generation(n_pop: int, n_items: int):
    """Vector ALU instructions (per wave, summed over the grid) of one
    generation of the on-chip loop, from the committed rocprofv3 summary, if
    it was taken on this workload with the current on-chip code; else None."""
    if (n_pop, n_items) != (1024, 10_000):
        return None
    keys = ("valu_insts_per_generation", "onchip_code_sha256")
    try:
        text = open(os.path.join(ROOT, ONCHIP_PROFILE)).read()
        fig = dict(line.strip().split(": ", 1) for line in text.splitlines()
                   if line.strip().startswith(tuple(k + ":" for k in keys)))
        if fig.get("onchip_code_sha256") != kernel_code_digest(sources=ONCHIP_SOURCES):
            return None
        return float(fig["valu_insts_per_generation"])
    except (OSError, KeyError, ValueError):
        return None


def batch_valu_per_call(onchip_launches: int):
    """Vector ALU instructions (per wave, summed over the grids) of the
    512-instance batch's on-chip launches in one 500-generation call, from
    the committed rocprofv3 summary, if it was taken with the current
    on-chip code and the same number of on-chip launches; else None."""
    keys = ("batch_valu_insts_per_call", "batch_onchip_launches", "onchip_code_sha256")
    try:
        text = open(os.path.join(ROOT, BATCH_PROFILE)).read()
        fig = dict(line.strip().split(": ", 1) for line in text.splitlines()
                   if line.strip().startswith(tuple(k + ":" for k in keys)))
        if fig.get("onchip_code_sha256") != kernel_code_digest(sources=ONCHIP_SOURCES):
            return None
        if int(fig["batch_onchip_launches"]) != onchip_launches:
            return None
        return float(fig["batch_valu_insts_per_call"])
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic(n_pop: int, n_items: int, shape=None, precision: int = 64):
    """HBM bytes per generation from the committed rocprofv3 counter summary,
    if it was taken on this workload and amplitude precision with the current
    kernel code and the same work shape (rows, waves, variant bits) when one
    is given; else None.  The summary's machine-readable lines carry a
    precision suffix (_f32, _f64)."""
    if (n_pop, n_items) != (4096, 200_000):
        return None
    sfx = "_f64" if precision == 64 else "_f32"
    keys = ("traffic_bytes_per_launch" + sfx, "kernel_code_sha256", "work_shape" + sfx)
    try:
        text = open(os.path.join(ROOT, PROFILE)).read()
        fig = dict(line.strip().split(": ", 1) for line in text.splitlines()
                   if line.strip().startswith(tuple(k + ":" for k in keys)))
        if fig.get("kernel_code_sha256") != kernel_code_digest():
            return None
        if shape is not None and fig.get("work_shape" + sfx) != "%d %d %d" % tuple(shape):
            return None
        return float(fig["traffic_bytes_per_launch" + sfx])
    except (OSError, KeyError, ValueError):
        return None


def rotating_rows(inst, precision: int, first: int, count: int):
    """Rows that rotate in generations first .. first+count-1 of the run (CIP
    of generation t-1, applied in the launch of t, moves every row whose
    fitness at t-1 is below that generation's elite; the elite and its ties
    only read beta).  The trajectory is deterministic, so a fresh run of the
    same seed stepped one generation at a time sees the timed runs' rows.
    Returns the per-generation counts."""
    from paper_2609_30862_amd import qieo
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      precision=precision)
    counts = []
    prev = None
    for t in range(first + count):
        if t >= first:
            counts.append(0 if prev is None else int((prev[0] < prev[1]).sum()))
        g.step(1)
        st = g.export_rows(0, inst.n_pop, amplitudes=False, alleles=False)
        fit = st["fitness"].astype("int64")
        prev = (fit, fit[int(st["elite"])])
    g.close()
    return counts


def cpu_baseline(inst, rows: int, gens: int, threads: int = 1, run_gens: int = 200,
                 precision: int = 64):
    """The CPU oracle, untuned, on a bounded sample of the same workload: the
    first `rows` chromosomes of the population over the full item list, for
    `gens` generations, on `threads` host threads (rows split among them).
    The whole population's time per generation and per run of `run_gens`
    generations is extrapolated from the sample's rate, and labelled so."""
    import oracle
    # the single-threaded run is pinned to one core of the process's set (the
    # calling thread only; the mask is restored afterwards)
    pinned, mask = None, None
    if threads == 1 and hasattr(os, "sched_setaffinity"):
        try:
            mask = os.sched_getaffinity(0)
            pinned = min(mask)
            os.sched_setaffinity(0, {pinned})
        except OSError:
            pinned = None
    try:
        o = oracle.Oracle(inst.values, inst.weights, inst.capacity, rows, inst.seed,
                          threads=threads, precision=precision)
        o.run(1)                # generation 0 observes only; time full generations
        t0 = time.perf_counter()
        o.run(gens)
        dt = time.perf_counter() - t0
    finally:
        if pinned is not None:
            os.sched_setaffinity(0, mask)
    rate = rows * inst.n_items * gens / dt
    per_gen = inst.n_pop * inst.n_items / rate
    return {"value": rate, "unit": "gene-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d of %d chromosomes x %d items, %d generations after "
                      "generation 0, binary%d amplitudes, %.1f s"
                      % (rows, inst.n_pop, inst.n_items, gens, precision, dt),
            "extrapolated_s_per_generation": per_gen,
            "extrapolated_s_per_run": run_gens * per_gen, "run_generations": run_gens,
            "pinned_cpu": pinned, "host": host_info()}


def host_info():
    """The host the CPU baseline ran on, read at run time."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"cpu": model, "nproc": os.cpu_count(), "usable_cpus": affinity}


def host_threads() -> int:
    """Host threads the process may use (its CPU affinity, at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def bench_batch(args):
    """512 ragged instances, 500 generations each: one batched call (all
    instances in the same launches, graph-replayed) against the per-instance
    loop of qieo_step calls, at identical best-found profit."""
    import numpy as np
    import torch
    import workloads
    from paper_2609_30862_amd import qieo

    insts = workloads.batch_instances()
    gens = insts[0].generations
    genes = sum(i.genes for i in insts)
    probs = [(i.values, i.weights, i.capacity, i.n_pop, i.seed) for i in insts]
    log("batch: %d instances, %.4g genes per generation, %d generations" % (len(insts), genes, gens))
    tuned = None
    if args.autotune:
        # class shapes tuned on the batch itself (its state is restored); the
        # tuning database then gives them to every batch built below
        b = qieo.Batch(probs)
        t0 = time.perf_counter()
        tuned = b.autotune(args.autotune)
        b.close()
        for c in tuned:
            if c["shape_class"] == -1:
                log("tuned on-chip variants: subset 0x%x, %d launches, %.4f ms/generation "
                    "(default subset 0x%x, %d launches: %.4f), %d subsets timed"
                    % (c["flags"], c["rows_per_block"], c["ms_per_generation"], c["default_flags"],
                       c["default_rows_per_block"], c["default_ms_per_generation"],
                       c["candidates"]))
                continue
            log("tuned class %d (%d rows, <= %d chunks): R %d S %d bits %d, %.4f ms/generation "
                "(default R %d S %d bits %d: %.4f)"
                % (c["shape_class"], c["rows"], c["max_chunks"], c["rows_per_block"],
                   c["waves_per_block"], c["flags"], c["ms_per_generation"],
                   c["default_rows_per_block"], c["default_waves_per_block"], c["default_flags"],
                   c["default_ms_per_generation"]))
        log("class tuning took %.1f s" % (time.perf_counter() - t0))
    variants = {}
    onchip_launches = None
    # untimed: two generations of the whole batch load every kernel variant
    # the timed calls use
    b = qieo.Batch(probs)
    b.step(2)
    b.close()
    # one call per variant, each on a fresh batch; "default" is the library's
    # default mode (every member that fits in batched on-chip launches, the
    # others LDS-resident or in per-generation launches, rows of 8+ chunks in
    # segment order)
    all_variants = (("default", True, 1, True),
                    ("no_onchip", True, 1, False),
                    ("no_onchip_no_persistent", False, 1, False),
                    ("no_onchip_segment_order_32_chunk_rows_only", True, 2, False),
                    ("no_onchip_row_order_long_rows", True, 0, False))
    for name, pers, seg, onchip in all_variants:
        if name != "default" and args.batch_variants != "all" and \
                name not in args.batch_variants.split(","):
            continue
        b = qieo.Batch(probs)
        b.set_persistent(pers)
        b.set_segment_order(seg)
        b.set_onchip(onchip)
        n_onchip = b.onchip_launches()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(gens)
        variants[name] = time.perf_counter() - t0
        if name == "default":
            best_batch = [b.best(k) for k in range(len(insts))]
            onchip_launches = n_onchip
        b.close()
        log("batched (%s, %d on-chip launches): %.3f s" % (name, n_onchip, variants[name]))
    wall_batch = variants["default"]

    # the third call of a batch: without the on-chip loop a repeated call is
    # replayed from its captured graph; with it, launched directly
    for name, onchip in (("replay_captured_no_onchip", False), ("third_call_default", True)):
        if args.batch_variants != "all" and name not in args.batch_variants.split(","):
            continue
        b = qieo.Batch(probs)
        b.set_onchip(onchip)
        b.step(gens)
        b.step(gens)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(gens)
        variants[name] = time.perf_counter() - t0
        b.close()
        log("batched, third call (%s): %.3f s" % (name, variants[name]))

    loops = {}
    done_at = {}                # per-instance completion time in the loop, from its start
    same = 0
    # the loop in the library's default mode (whole-call launches where they
    # pay, graph capture on or off), and the plain per-generation launch loop
    for mode in (() if args.skip_loop else ("graph", "launches", "per_generation_launches")):
        wall_loop = 0.0
        done_at[mode] = []
        for k, i in enumerate(insts):
            g = qieo.Instance(i.values, i.weights, i.capacity, i.n_pop, i.seed)
            g.set_graph(mode == "graph")
            if mode == "per_generation_launches":
                g.set_persistent(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(gens)
            wall_loop += time.perf_counter() - t0
            done_at[mode].append(wall_loop)
            if mode == "graph":
                r = g.best()
                same += int((r.fitness, r.profit, r.generation, r.chromosome) ==
                            (best_batch[k].fitness, best_batch[k].profit,
                             best_batch[k].generation, best_batch[k].chromosome))
            g.close()
        loops[mode] = wall_loop
        log("per-instance loop (%s): %.3f s" % (mode, wall_loop))
    # the on-chip launches keep the planes in registers: bound by vector ALU
    # issue, measured by their instruction count (rocprofv3 SQ_INSTS_VALU);
    # the call's whole wall time, the left-out members' launches included
    valu = batch_valu_per_call(onchip_launches or 0) if gens == 500 else None
    valu_rate = None if valu is None else valu * 64 / wall_batch / 1e9
    roofline = {"bound": "alu", "achieved": valu_rate, "peak": VALU_PEAK_G,
                "unit": "G VALU lane-instructions/s",
                "frac": None if valu_rate is None else valu_rate / VALU_PEAK_G,
                "traffic": None,
                "kernel": "onchip_multi_kernel (%s on-chip launches per call)" % onchip_launches,
                "valu_insts_per_call": valu}
    if args.skip_loop:
        out = {"workload": "batch", "batch_variants_seconds": variants, "roofline": roofline,
               "value": genes * gens / wall_batch, "unit": "gene-updates/s",
               "onchip_launches": onchip_launches, "tuned_classes": tuned}
        print(json.dumps(out), flush=True)
        return
    log("identical best records %d/%d" % (same, len(insts)))
    wall_launch_loop = loops.pop("per_generation_launches")
    wall_loop = min(loops.values())
    # per-instance latency from the start: the batched call returns every
    # result when it ends; the loop finishes instance k after the calls of
    # instances 0..k (creation excluded on both sides)
    fastest = min(loops, key=loops.get)
    lat_loop = np.array(done_at[fastest])
    latency = {"batched": {"p50": wall_batch, "p99": wall_batch},
               "per_instance_loop": {"p50": float(np.percentile(lat_loop, 50)),
                                     "p99": float(np.percentile(lat_loop, 99))}}
    log("latency from the start: batched p50 = p99 = %.3f s; loop p50 %.3f s, p99 %.3f s"
        % (wall_batch, latency["per_instance_loop"]["p50"], latency["per_instance_loop"]["p99"]))
    out = {
        "metric": "gene-updates/s", "value": genes * gens / wall_batch, "unit": "gene-updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": wall_batch * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "qieo-knapsack batch of %d ragged instances, %d generations"
                               % (len(insts), gens)},
        "per_instance_loop": {"value": genes * gens / wall_loop, "seconds": wall_loop,
                              "variants_seconds": loops},
        "batch_variants_seconds": variants,
        "onchip_launches": onchip_launches,
        "roofline": roofline,
        "speedup_vs_loop": wall_loop / wall_batch,
        "per_generation_launch_loop": {"value": genes * gens / wall_launch_loop,
                                       "seconds": wall_launch_loop},
        "speedup_vs_per_generation_launch_loop": wall_launch_loop / wall_batch,
        "latency_s": latency,
        "identical_best": "%d/%d" % (same, len(insts)),
        "tuned_classes": tuned,
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Open-loop replay of a Poisson request stream through the server: each
    request is submitted at its arrival time; latency is completion minus
    submission.  The per-instance loop (qieo_create + qieo_step per request,
    one after another) runs a sample of the same requests for comparison."""
    import numpy as np
    import torch
    import workloads
    from paper_2609_30862_amd import qieo

    reqs = workloads.serving_requests(args.requests, args.rate)
    work = [r.instance.genes * r.instance.generations for r in reqs]
    log("serve: %d requests at %.0f/s, %.4g gene-updates, budget %.0f GB, cap %d, G=%d"
        % (len(reqs), args.rate, sum(work), args.budget_gb, args.max_resident,
           args.gens_per_iter))
    srv = qieo.Server(int(args.budget_gb * (1 << 30)), args.max_resident, args.gens_per_iter)
    srv.set_onchip(not args.no_onchip)
    torch.cuda.synchronize()
    tickets = []
    t0 = time.perf_counter()
    for r in reqs:
        delay = t0 + r.arrival_s - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        i = r.instance
        tickets.append(srv.submit(i.values, i.weights, i.capacity, i.n_pop, i.seed,
                                  i.generations))
    t_sub = time.perf_counter() - t0
    log("submitted in %.2f s; waiting" % t_sub)
    res, lat = [], []
    last_log = time.perf_counter()
    for k, t in enumerate(tickets):
        out = srv.wait(t)
        res.append(out[0])
        lat.append(out[1] * 1e-9)
        if time.perf_counter() - last_log > 20:
            st = srv.stats()
            log("  %d/%d done, resident %d, queued %d" % (k + 1, len(tickets), st["resident"],
                                                          st["queued"]))
            last_log = time.perf_counter()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    served = sum(work) / wall
    log("served: %.2f s, %.4g gene-updates/s, latency p50 %.2f s p99 %.2f s, peak resident %d"
        % (wall, served, np.percentile(lat, 50), np.percentile(lat, 99), st["peak_resident"]))

    m = min(args.loop_sample, len(reqs))
    loop_s, same = 0.0, 0
    for k in range(m):
        i = reqs[k].instance
        g = qieo.Instance(i.values, i.weights, i.capacity, i.n_pop, i.seed)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        g.step(i.generations)
        loop_s += time.perf_counter() - ts
        r = g.best()
        same += int((r.fitness, r.generation, r.chromosome) ==
                    (res[k].fitness, res[k].generation, res[k].chromosome) and
                    np.array_equal(r.bits, res[k].bits))
        g.close()
    loop_rate = sum(work[:m]) / loop_s
    log("per-instance loop on %d requests: %.2f s, %.4g gene-updates/s, identical %d/%d"
        % (m, loop_s, loop_rate, same, m))
    # the same requests as a plain per-generation launch loop (mode 0)
    launch_s = 0.0
    for k in range(m):
        i = reqs[k].instance
        g = qieo.Instance(i.values, i.weights, i.capacity, i.n_pop, i.seed)
        g.set_persistent(0)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        g.step(i.generations)
        launch_s += time.perf_counter() - ts
        g.close()
    launch_rate = sum(work[:m]) / launch_s
    log("per-generation launch loop on %d requests: %.2f s, %.4g gene-updates/s"
        % (m, launch_s, launch_rate))
    out = {
        "metric": "gene-updates/s", "value": served, "unit": "gene-updates/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "qieo-knapsack serving, %d Poisson requests at %.0f/s, "
                               "%.0f GB budget" % (len(reqs), args.rate, args.budget_gb),
                   "max_resident": args.max_resident, "gens_per_iter": args.gens_per_iter,
                   "onchip": not args.no_onchip},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean()), "max": float(lat.max())},
        "server": {k: st[k] for k in ("iterations", "peak_resident", "peak_pool_used", "failed")},
        "per_instance_loop": {"requests": m, "value": loop_rate, "seconds": loop_s,
                              "identical_best": "%d/%d" % (same, m)},
        "speedup_vs_loop": served / loop_rate,
        "per_generation_launch_loop": {"requests": m, "value": launch_rate, "seconds": launch_s},
        "speedup_vs_per_generation_launch_loop": served / launch_rate,
    }
    print(json.dumps(out), flush=True)


def bench_stream(args):
    """HBM reference rates on the large workload's two amplitude planes
    (4096 x 200,064 binary32 each, 3.28 GB), with stock torch kernels: an
    in-place read-modify-write of both planes (16 B per gene, as one
    generation), the same read and write into two other planes, a read of
    both (sums) and a write of both (fills)."""
    import torch
    rows, pitch = args.n_pop, (args.n_items + 63) // 64 * 64
    a = torch.zeros(rows * pitch, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    a2 = torch.zeros_like(a)
    b2 = torch.zeros_like(a)
    genes = rows * pitch
    ops = {
        "read+write in place": (lambda: (a.mul_(1.5), b.mul_(1.5)), 16),
        "read+write elsewhere": (lambda: (torch.mul(a, 1.5, out=a2), torch.mul(b, 1.5, out=b2)), 16),
        "read only": (lambda: (a.sum(), b.sum()), 8),
        "write only": (lambda: (a.fill_(0.5), b.fill_(0.5)), 8),
    }
    out = {}
    for name, (fn, per_gene) in ops.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        out[name] = {"ms": ms, "GB/s": per_gene * genes / (ms * 1e-3) / 1e9}
        log("%-20s %.4f ms  %.1f GB/s" % (name, ms, out[name]["GB/s"]))
    print(json.dumps({"workload": "stream", "rows": rows, "pitch": pitch, "rates": out}),
          flush=True)


def bench_fractions(args):
    """Per-step time of the generation over an (Np, Ng) grid, for the fused
    launch, the paper's four-launch pipeline with DetermineElite on the device
    or on the host, and the chromosome-parallel mapping (eq. (3)).  Prints
    one JSON line per cell."""
    import torch
    import workloads
    from paper_2609_30862_amd import qieo

    grid = [(np_, ng) for np_ in (256, 1024, 4096) for ng in (500, 2500, 10_000, 40_000, 200_000)]
    for (np_, ng) in grid:
        inst = workloads.random_instance(ng, np_, seed=ng + np_, wmax=100, offset=10)
        g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
        g.set_timing(True)
        cell = {"n_pop": np_, "n_items": ng}
        for name, pipe, gens in (("fused", 0, 20), ("unfused_device_de", 1, 20),
                                 ("unfused_host_de", 3, 20), ("chromosome", 4, 3)):
            g.set_pipeline(pipe)
            g.step(2)
            g.stage_time(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(gens)
            wall = (time.perf_counter() - t0) / gens * 1e3
            st = g.stage_time(reset=True)
            per = {k: v[1] / gens for k, v in st.items() if v[0]}
            cell[name] = {"t_gen_ms": wall, "stage_ms": per}
        f = cell["unfused_host_de"]["stage_ms"]
        tot = sum(f.values())
        cell["fractions_host_de"] = {k: v / tot for k, v in f.items()}
        cell["rho"] = cell["chromosome"]["t_gen_ms"] / cell["fused"]["t_gen_ms"]
        g.close()
        log("Np=%5d Ng=%6d fused %.3f ms, unfused %.3f ms, host-DE %.3f ms, chromosome %.2f ms"
            % (np_, ng, cell["fused"]["t_gen_ms"], cell["unfused_device_de"]["t_gen_ms"],
               cell["unfused_host_de"]["t_gen_ms"], cell["chromosome"]["t_gen_ms"]))
        print(json.dumps(cell), flush=True)


def bench_launch(args):
    """Small and medium single instances, where launch overhead matters: time
    per generation with one launch per generation, with graph replay of the
    whole call, in the default mode (1), with the single-workgroup loop
    (mode 2: from LDS where the state fits, else from global memory) and
    with the on-chip grid loop (mode 3; per-generation launches where the
    population does not fit it)."""
    import torch
    import workloads
    from paper_2609_30862_amd import qieo

    shapes = [(16, 100), (32, 500), (64, 100), (64, 1000), (128, 500), (24, 5000), (256, 500),
              (64, 4000), (256, 2000), (32, 12_000), (128, 8000), (256, 8000), (512, 5000),
              (1024, 2000), (4096, 1000), (2048, 3000), (1024, 10_000),
              # around the default mode's on-chip threshold: 256 to 2048 (row, chunk) items
              (256, 200), (512, 100), (96, 1300), (128, 1000), (1024, 200), (512, 400),
              (2048, 100), (64, 8000)]
    for (np_, ng) in shapes:
        inst = workloads.random_instance(ng, np_, seed=ng + np_)
        cell = {"n_pop": np_, "n_items": ng}
        for name, graph, pers in (("launches", 0, 0), ("graph", 1, 0), ("persistent", 0, 1),
                                  ("persistent_any", 0, 2), ("onchip", 0, 3)):
            g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
            g.set_graph(graph)
            g.set_persistent(pers)
            g.step(500)                      # warm-up
            g.step(500)                      # a repeated call: graph captured here
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(500)
            cell[name] = (time.perf_counter() - t0) / 500 * 1e6
            g.close()
        log("Np=%5d Ng=%6d  us/generation: launches %.2f  graph %.2f  default mode %.2f  "
            "single workgroup %.2f  on-chip %.2f"
            % (np_, ng, cell["launches"], cell["graph"], cell["persistent"],
               cell["persistent_any"], cell["onchip"]))
        print(json.dumps(cell), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed generations (default: the workload's budget, 200 for large)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-pop", type=int, default=4096)
    ap.add_argument("--n-items", type=int, default=200_000)
    ap.add_argument("--tile", type=str, default="", help="R,S work shape override")
    ap.add_argument("--kernel-flags", type=int, default=-1, help="generation kernel variant")
    ap.add_argument("--precision", type=int, choices=[32, 64], default=None,
                    help="amplitude precision: 64 is the paper's binary64 (default for the "
                         "large workload), 32 binary32 (default for small and medium, whose "
                         "configurations name binary32)")
    ap.add_argument("--autotune", type=int, default=0, metavar="GENS",
                    help="time every work shape for GENS generations first and use the best")
    ap.add_argument("--repeats", type=int, default=5,
                    help="large: timed runs, each on a fresh instance of the same seed "
                         "(identical work); value is the median run")
    ap.add_argument("--cpu-rows", type=int, default=256)
    ap.add_argument("--cpu-gens", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["large", "medium", "small", "batch", "serve",
                                           "fractions", "launch", "stream"],
                    default="large",
                    help="large: the single 4096 x 200,000 instance (default); medium: "
                         "1024 x 10,000, 1000 generations (its planes fit the 256 MB "
                         "last-level cache); small: 16 x 100, 500 generations; batch: 512 "
                         "ragged instances x 500 generations vs a per-instance launch loop; "
                         "serve: Poisson request stream through the continuous-batching server; "
                         "fractions: per-step costs of the fused and unfused pipelines; "
                         "launch: launch-bound small instances; stream: HBM reference rates "
                         "on the large workload's planes")
    ap.add_argument("--config", type=int, choices=[1, 2, 3, 4, 5], default=None,
                    help="the five workloads by number: 1 small, 2 medium, 3 large, 4 batch, "
                         "5 serve (all 20,000 requests unless --requests is given)")
    ap.add_argument("--requests", type=int, default=None,
                    help="serve: number of requests (default 2000; 20,000 with --config 5)")
    ap.add_argument("--rate", type=float, default=500.0, help="serve: offered requests/s")
    ap.add_argument("--budget-gb", type=float, default=128.0, help="serve: HBM budget")
    ap.add_argument("--max-resident", type=int, default=0, help="serve: resident cap (0 = none)")
    ap.add_argument("--gens-per-iter", type=int, default=25, help="serve: generations/iteration")
    ap.add_argument("--loop-sample", type=int, default=200,
                    help="serve: requests re-run one by one for the per-instance loop baseline")
    ap.add_argument("--batch-variants", default="all",
                    help="batch: comma-separated variants to time (default, no_onchip, "
                         "no_onchip_no_persistent, no_onchip_segment_order_32_chunk_rows_only, "
                         "no_onchip_row_order_long_rows, replay_captured_no_onchip, "
                         "third_call_default) or all; default is always timed")
    ap.add_argument("--no-onchip", action="store_true",
                    help="serve: residents in per-generation launches only (no batched on-chip loop)")
    ap.add_argument("--skip-loop", action="store_true",
                    help="batch: time the batched calls only (no per-instance loop)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (to scale HBM counters)")
    args = ap.parse_args()
    if args.config is not None:
        args.workload = {1: "small", 2: "medium", 3: "large", 4: "batch", 5: "serve"}[args.config]
    if args.requests is None:
        args.requests = 20_000 if args.config == 5 else 2000

    if args.gpus != 1:
        print("bench.py measures one GPU only: libqieo runs each population on one GPU "
              "and has no multi-GPU path (independent instances would be routed to GPUs "
              "with no communication). Run with --gpus 1.", file=sys.stderr)
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
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "fractions":
        return bench_fractions(args)
    if args.workload == "stream":
        return bench_stream(args)
    if args.workload == "launch":
        return bench_launch(args)
    if args.workload == "medium":
        inst = workloads.medium_instance()
    elif args.workload == "small":
        inst = workloads.small_instance()
    else:
        inst = workloads.large_instance(args.n_pop, args.n_items)
    if args.steps is None:
        args.steps = inst.generations
    if args.precision is None:
        args.precision = 64 if args.workload == "large" else 32
    elem = 8 if args.precision == 64 else 4
    log("workload %s, binary%d amplitudes, %d steps, %d warmup"
        % (inst.name, args.precision, args.steps, args.warmup))
    if args.autotune:
        r = qieo.qieo_autotune(inst.n_items, inst.n_pop, args.autotune)
        log("autotune: %s" % r)
    genes = inst.n_pop * inst.n_items
    # algorithmic bytes of a generation in which every row rotates: alpha
    # and beta read and written once
    bytes_per_launch = AMPLITUDES_PER_GENE_UPDATE * elem * genes
    runs = []

    def fresh():
        # a fresh population of the same seed: every run does the same work
        h = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=args.precision)
        if args.tile:
            r, s = (int(x) for x in args.tile.split(","))
            h.set_tile(r, s)
        if args.kernel_flags >= 0:
            h.set_kernel_flags(args.kernel_flags)
        h.step(args.warmup)
        return h

    for rep in range(max(1, args.repeats)):
        # wall time of K generations, no timing events in the stream
        g = fresh()
        shape = tuple(g.tile()) + (g.kernel_flags(),)
        if rep == 0:
            log("work shape rows/block, waves/block, variant bits = %s" % (shape,))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step_async(args.steps)
        g.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        best = g.best()
        g.close()
        # kernel time: the same K generations with HIP events around each
        # generation's launches (the event records cost a few microseconds
        # per generation, so they stay out of the wall-time run)
        g = fresh()
        g.set_timing(True)
        g.kernel_time(reset=True)
        torch.cuda.synchronize()
        g.step_async(args.steps)
        g.sync()
        torch.cuda.synchronize()
        launches, kern_ms = g.kernel_time(reset=True)
        path = g.call_path()
        g.set_timing(False)
        g.close()
        # per generation: the events enclose each generation's launches, or
        # the whole call where one single-workgroup launch runs all of them
        avg_ms = kern_ms / args.steps
        log("run %d: wall %.3f s, %.3f ms/generation, kernel avg %.3f ms over %d timed "
            "launches, %.1f GB/s algorithmic, best fitness %d (gen %d)"
            % (rep, wall, wall / args.steps * 1e3, avg_ms, launches,
               bytes_per_launch / (avg_ms * 1e-3) / 1e9, best.fitness, best.generation))
        runs.append((wall, avg_ms))

    # the median run by wall time, and the median kernel average
    wall = sorted(w for w, _ in runs)[len(runs) // 2]
    avg_ms = sorted(a for _, a in runs)[len(runs) // 2]
    value = genes * args.steps / wall
    # the rows that rotated in the timed generations: a row that does not
    # rotate (the elite and its ties, every row at generation 0) reads only
    # beta, so a generation moves elem * Ng * (Np + 3 * rotating rows) bytes
    rot = rotating_rows(inst, args.precision, args.warmup, args.steps)
    rot_frac = sum(rot) / float(inst.n_pop * args.steps)
    bytes_exact = elem * inst.n_items * (inst.n_pop * args.steps + 3 * sum(rot)) / args.steps
    log("rotating rows in the timed generations: %d of %d (%.5f)"
        % (sum(rot), inst.n_pop * args.steps, rot_frac))
    achieved = bytes_exact / (avg_ms * 1e-3) / 1e9
    # the on-chip loop keeps the planes in registers: bound by vector ALU
    # issue, measured by its instruction count (rocprofv3 SQ_INSTS_VALU)
    valu = onchip_valu_per_generation(inst.n_pop, inst.n_items)
    valu_rate = None if valu is None else valu * 64 / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "alu", "achieved": valu_rate, "peak": VALU_PEAK_G,
                "unit": "G VALU lane-instructions/s",
                "frac": None if valu_rate is None else valu_rate / VALU_PEAK_G,
                "traffic": None, "kernel": PATH_KERNELS[3], "kernel_avg_ms": avg_ms,
                "valu_insts_per_generation": valu}

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
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": "qieo-knapsack single instance Np=%d Ng=%d, binary%d "
                               "amplitudes, %d generations"
                               % (inst.n_pop, inst.n_items, args.precision, args.steps),
                   "n_pop": inst.n_pop, "n_items": inst.n_items, "seed": inst.seed,
                   "precision": "binary%d" % args.precision,
                   "generations_per_step": 1,
                   # generation indices the timed region runs (after the
                   # warm-up, on a fresh population of the seed)
                   "timed_generations": [args.warmup, args.warmup + args.steps - 1],
                   # amplitude planes within the 256 MB last-level cache: the
                   # rate is the cache's, not HBM's
                   "cache_resident": genes * 2 * elem <= 256 << 20},
        "repeats": len(runs),
        "ms_per_step_runs": [w / args.steps * 1e3 for w, _ in runs],
        "kernel_avg_ms_runs": [a for _, a in runs],
        "hbm_frac_algorithmic": value * bytes_exact / genes / (HBM_PEAK_GBS * 1e9),
        "rotating_rows": {"fraction": rot_frac, "rows": sum(rot),
                          "of": inst.n_pop * args.steps,
                          "min_per_generation": min(rot), "max_per_generation": max(rot)},
        "roofline": roofline if path == qieo.PATH_ONCHIP else
                    {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     # counters were taken with one work shape and variant
                     "traffic": measured_traffic(inst.n_pop, inst.n_items, shape,
                                                 args.precision),
                     "kernel": PATH_KERNELS.get(path, "generation_kernel")
                               if path != qieo.PATH_LAUNCHES
                               else ("segment_kernel + segment_fe_kernel" if shape[2] & 16
                                     else "generation_kernel"),
                     "kernel_avg_ms": avg_ms,
                     # algorithmic bytes of the timed generations' average
                     # launch (rotating rows 4 amplitudes per gene, others 1)
                     "bytes_per_launch": bytes_exact,
                     "bytes_per_launch_all_rows_rotating": bytes_per_launch},
    }
    if path == qieo.PATH_ONCHIP:
        out["note"] = ("on-chip loop: the planes stay in registers for the call, so "
                       "hbm_frac_algorithmic is what the per-generation path would need")
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on %d rows x %d generations" % (args.cpu_rows, args.cpu_gens))
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_rows, args.cpu_gens,
                                           run_gens=args.steps, precision=args.precision)
        nt = host_threads()
        log("cpu baseline: oracle on %d threads, %d rows x %d generations"
            % (nt, args.cpu_rows * nt, args.cpu_gens))
        out["cpu_baseline_threads"] = cpu_baseline(inst, min(inst.n_pop, args.cpu_rows * nt),
                                                   args.cpu_gens, threads=nt,
                                                   run_gens=args.steps,
                                                   precision=args.precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
