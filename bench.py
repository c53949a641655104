#!/usr/bin/env python3
"""Benchmark: k-variant combinations scored per second on one MI355X.

One step = the whole search on one dataset already resident in device memory
(class partition, bit packing, counting + FP32 scoring + filtering, candidate
selection, FP64 rescoring, final ordering) through fiuncho_scan_batch on a
stream.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
                  [--shard I/P] [--kernel auto|popcount|pairs|mfma|mfma-fp4|triples] [--autotune]

--shard I/P times one GPU's share of a search split across P GPUs (shard I
of the job's work tiles); the rate is that share's combinations per second.

Workloads (seeded synthetic data, see paper_2201_03331_amd/synth.py):
  order3-1000x6400 (default), order2-100x1600, order2-4000x16000,
  order4-200x4000, order5-200x4000, batch64 (64 uneven datasets in one
  persistent launch, replayed from a HIP graph), batch64-plain (the same 64
  datasets, one call each).
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "k-SNP combinations scored/s (×samples) at order 2/3/4, 1 MI355X, batched vs plain"

# gfx950: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 32-bit VALU lane-ops/s
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9


def workloads():
    from paper_2201_03331_amd import synth
    return {
        "order3-1000x6400": lambda: [synth.order3_main()],
        "order2-100x1600": lambda: [synth.order2_small()],
        "order2-4000x16000": lambda: [synth.order2_dense()],
        "order4-200x4000": lambda: [synth.high_order(4)],
        "order5-200x4000": lambda: [synth.high_order(5)],
        "batch64": lambda: synth.batch_jobs(64),
        "batch64-plain": lambda: synth.batch_jobs(64),
    }


def word_ops_per_combination(k: int, m0: int, m1: int, kernel: int) -> int:
    """64-bit AND+popcount operations a popcount kernel executes per
    combination, over W = ceil(m0/64) + ceil(m1/64) words: 4 per word at
    order 2 (rows g=0,1 of both variants); 8 at order 3 on the pair-table
    kernel (only the {0,1}^3 cells are counted, the others follow from
    lower-order tables); 2*3^(k-1) otherwise (rows g=0,1 of the last variant
    against every row of the prefix)."""
    from paper_2201_03331_amd import fiuncho
    W = (m0 + 63) // 64 + (m1 + 63) // 64
    if k == 1:
        return 0
    if k == 2:
        return 4 * W
    if k == 3 and kernel == fiuncho.KERNEL_PAIRS:
        return 8 * W
    if k == 4 and kernel == fiuncho.KERNEL_TRIPLES:
        return 16 * W
    return 2 * 3 ** (k - 1) * W


# gfx950 dense int8 matrix-core peak (ops/s; one multiply-add = 2 ops)
MFMA_I8_PEAK_OPS = 5.0e15
# dense FP4 (E2M1) matrix peak of MI355X, operations per second
MFMA_FP4_PEAK_OPS = 10.1e15


def kernel_sources_sha256() -> str:
    """Hash of every source that defines or launches a kernel (all of csrc
    but the host-side API file, and the public header): any change voids
    counters taken on an earlier build."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2201_03331_amd", "csrc")
    files = sorted(f for f in glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))
                   if os.path.basename(f) != "api.hip") + [os.path.join(ROOT, "include", "fiuncho.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the counter table in
    profiles/hbm_traffic.md (rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a
    copy of known size), or None when no row was taken on these sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    sha = kernel_sources_sha256()
    for line in open(path):
        cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
        if len(cells) >= 8 and cells[0] == kernel and cells[1] == workload and cells[2] == sha:
            try:
                return float(cells[7])
            except ValueError:
                return None
    return None


def cpu_baseline(d, budget_s: float = 20.0):
    """The oracle (plain per-sample counting, FP64 MI) timed on the host cores
    over a contiguous sample of ranks of the same workload."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    total = math.comb(d.n, d.order)
    probe = min(total, 20000)
    t0 = time.perf_counter()
    oracle.scan_range(d.genotypes, d.phenotype, d.order, d.top_n, 0, probe, nthreads=threads)
    dt = max(time.perf_counter() - t0, 1e-6)
    count = min(total, max(probe, int(probe * budget_s / dt)))
    t0 = time.perf_counter()
    oracle.scan_range(d.genotypes, d.phenotype, d.order, d.top_n, 0, count, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "combinations/s", "cores": threads, "kind": "oracle",
            "sample": f"lexicographic ranks [0, {count}) of the same dataset "
                      f"({count / total:.3g} of C({d.n},{d.order})), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="order3-1000x6400", choices=sorted(workloads().keys()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", default="auto", choices=("auto", "popcount", "pairs", "mfma", "mfma-fp4", "triples"),
                    help="force this counting kernel for every dataset shape it handles")
    ap.add_argument("--autotune", action="store_true",
                    help="time the kernels for every dataset shape first (fiuncho_autotune)")
    ap.add_argument("--shard", default=None, metavar="I/P",
                    help="search only shard I of P of every dataset's work tiles")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of this many MiB (for counter scaling)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the scan would shard by (k-1)-prefix; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_03331_amd import fiuncho

    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 5}))
        return

    datasets = workloads()[args.workload]()
    plain = args.workload.endswith("-plain")
    if args.kernel != "auto":
        forced = {"popcount": fiuncho.KERNEL_POPCOUNT, "pairs": fiuncho.KERNEL_PAIRS,
                  "mfma": fiuncho.KERNEL_MFMA, "mfma-fp4": fiuncho.KERNEL_MFMA_FP4,
                  "triples": fiuncho.KERNEL_TRIPLES}[args.kernel]
        for d in datasets:
            if fiuncho.lib().fiuncho_set_kernel(d.n, d.m, d.order, forced) != fiuncho.OK:
                ap.error(f"kernel {args.kernel} does not handle order {d.order}")
    tuned = {}
    if args.autotune:
        for d in datasets:
            key = (d.order, d.n.bit_length(), ((d.m + 63) // 64).bit_length())
            if key not in tuned:
                tuned[key] = fiuncho.autotune(d.n, d.m, d.order)
    shard = None
    if args.shard:
        si, sp = (int(v) for v in args.shard.split("/"))
        if not 0 <= si < sp:
            ap.error("--shard I/P needs 0 <= I < P")
        shard = (si, sp)
    sh = None if shard is None else [shard] * len(datasets)
    batches = ([fiuncho.DeviceBatch([d], shards=None if sh is None else [shard]) for d in datasets]
               if plain else [fiuncho.DeviceBatch(datasets, shards=sh)])
    stream = torch.cuda.current_stream()
    graph = args.workload == "batch64"
    if graph:
        batches[0].capture()

    def step():
        if graph:
            batches[0].replay()
            return
        for b in batches:
            b.run(stream)

    # warm-up calls run profiled too: a profiled call's first use of a job
    # shape does host-side bookkeeping (a sharded job's combination count)
    fiuncho.set_profiling(not graph)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.warmup and not graph:
        fiuncho.get_profile()  # averages restart after the warm-up calls
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    fiuncho.set_profiling(False)
    ms = start.elapsed_time(end) / args.steps
    if graph:
        # events recorded by graph replays cannot be timed: the phase times of
        # a graph step come from one eager call right after the timed replays
        fiuncho.set_profiling(True)
        batches[0].run(stream)
        torch.cuda.synchronize()
        fiuncho.set_profiling(False)
    prof = fiuncho.get_profile()

    # results of the last step: status and the top hit
    res = [r for b in batches for r in b.results()]
    ok = all(s == 0 for s, _ in res)
    def share(d):
        if shard is None:
            return math.comb(d.n, d.order)
        return int(fiuncho.shard_counts(d.n, d.m, d.order, shard[1], fiuncho.TILE_ROUND_ROBIN)[shard[0]])

    combos = sum(share(d) for d in datasets)
    combos_m = sum(share(d) * d.m for d in datasets)
    value = combos / (ms / 1e3)

    # roofline of the dominant counting kernel: algorithmic work per launch
    # over that kernel's measured time.  Popcount kernels: 32-bit VALU
    # lane-ops (4 per 64-bit AND+popcount).  Matrix-core kernels: operations
    # of the one-hot contraction, 2 x (4 or 8) cells x m samples per
    # combination, against the int8 or the FP4 peak (a batch with both: the
    # time both parts would take at their peaks).
    lane_ops = 0
    mfma_ops = 0
    mfma_peak_s = 0.0
    # the counter table's workload key (a shard launches fewer tiles)
    traffic_key = args.workload + ("" if shard is None else f" shard {shard[0]}/{shard[1]}")
    kernels = set()
    for d in datasets:
        m1 = int(d.phenotype.sum())
        kern = fiuncho.get_kernel(d.n, d.m, d.order)
        kernels.add(kern)
        if kern in (fiuncho.KERNEL_MFMA, fiuncho.KERNEL_MFMA_FP4) and (d.order <= 3 or d.m <= 20447):
            # cells counted on the matrix cores for every combination over
            # every sample: the {0,1}^k cells at orders 2 and 3 (4 and 8; the
            # others come from class counts and pair tables), at orders 4 and
            # 5 every prefix row against rows 0, 1 of the last variant
            # (2 * 3^(k-1))
            cells = 4 if d.order == 2 else 8 if d.order == 3 else 2 * 3 ** (d.order - 1)
            ops = 2 * cells * d.m * share(d)
            mfma_ops += ops
            mfma_peak_s += ops / (MFMA_FP4_PEAK_OPS if kern == fiuncho.KERNEL_MFMA_FP4 else MFMA_I8_PEAK_OPS)
        else:
            lane_ops += 4 * word_ops_per_combination(d.order, d.m - m1, m1, kern) * share(d)
    calls = len(batches) if plain else 1
    scan_ms = prof["scan_ms"] * calls
    mfma_ms = prof["mfma_ms"] * calls
    if mfma_ms > scan_ms:
        achieved = mfma_ops / (mfma_ms / 1e3) / 1e12
        peak = mfma_ops / mfma_peak_s / 1e12
        fp4 = fiuncho.KERNEL_MFMA_FP4 in kernels
        i8 = fiuncho.KERNEL_MFMA in kernels
        fmt = "int8 and FP4" if fp4 and i8 else "FP4" if fp4 else "int8"
        roofline = {"bound": "mfma", "kernel": f"mfma_kernel (one-hot {fmt} contraction + FP32 MI + filter)",
                    "achieved": achieved, "peak": peak, "unit": f"T {fmt} op/s", "frac": achieved / peak,
                    # the counter table holds the FP4 kernels' launches
                    "traffic": measured_traffic("mfma_kernel", traffic_key) if fmt == "FP4" else None}
    else:
        achieved = lane_ops / (scan_ms / 1e3) / 1e12
        peak = VALU_PEAK_LANE_OPS / 1e12
        roofline = {"bound": "alu", "kernel": "scan_kernel (AND+popcount counting + FP32 MI + filter)",
                    "achieved": achieved, "peak": peak, "unit": "T int32 lane-op/s", "frac": achieved / peak,
                    # the counter table holds the pair-table (order 3) and
                    # triple-table (order 4) kernels' launches
                    "traffic": measured_traffic("scan_kernel", traffic_key)
                    if kernels <= {fiuncho.KERNEL_PAIRS, fiuncho.KERNEL_TRIPLES} else None}
    names = {fiuncho.KERNEL_POPCOUNT: "popcount", fiuncho.KERNEL_PAIRS: "pairs", fiuncho.KERNEL_MFMA: "mfma",
             fiuncho.KERNEL_TRIPLES: "triples", fiuncho.KERNEL_MFMA_FP4: "mfma-fp4"}

    d0 = datasets[0]
    planted_first = None
    if len(datasets) == 1 and shard is None and res[0][1].size:
        planted = [p for p in d0.planted if len(p) == d0.order]
        if planted:
            planted_first = tuple(int(v) for v in res[0][1][0]["snp"][: d0.order]) == planted[0]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "combinations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "datasets": len(datasets),
            "snps": d0.n if len(datasets) == 1 else None,
            "samples": d0.m if len(datasets) == 1 else None,
            "order": d0.order if len(datasets) == 1 else "2+3",
            "top_n": d0.top_n,
            "combinations": combos,
            "calls_per_step": len(batches),
            "shard": None if shard is None else f"{shard[0]}/{shard[1]}",
        },
        "combinations_x_samples_per_s": combos_m / (ms / 1e3),
        "arithmetic": "u64 bitsets, u32 popcount counts, plain f32 MI estimate with a rigorous "
                      "rounding bound for filtering, compensated f32 and f64 MI of the kept",
        "phases_ms": {k: round(prof[k], 4) for k in ("pack_ms", "pilot_ms", "scan_ms", "mfma_ms",
                                                     "select_ms", "total_ms")},
        "kernels": sorted(names[k] for k in kernels),
        "autotuned": {f"order {k[0]}, snps < 2^{k[1]}, words < 2^{k[2]}": names[v]
                      for k, v in sorted(tuned.items())} if args.autotune else None,
        "candidates": prof["candidates"],
        "rescored": prof["kept"],
        "status_ok": ok,
        "planted_first": planted_first,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and len(datasets) == 1 and shard is None:
        out["cpu_baseline"] = cpu_baseline(d0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
