#!/usr/bin/env python3
"""Benchmark: k-variant combinations scored per second on one MI355X.

One step = the whole search on one dataset already resident in device memory
(class partition, bit packing, counting + FP32 scoring + filtering, candidate
selection, FP64 rescoring, final ordering) through fiuncho_scan_batch on a
stream.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
                  [--shard I/P] [--kernel auto|popcount|pairs|mfma|mfma-fp4|triples|mfma-fp4-tables] [--autotune]

--shard I/P times one GPU's share of a search split across P GPUs (shard I
of the job's work tiles); the rate is that share's combinations per second.

A default run (order3-1000x6400, automatic kernels, no shard) also measures
the other workloads of the metric in the same process and adds them as
"configs": each with its step time, rate, kernels, dominant kernel and its
roofline fraction; batch64 (one graph replay) carries its speed-up over
batch64-plain (64 calls).  --no-configs skips them.  Besides combinations/s
the line gives combinations x samples/s and table cells x samples/s
(combinations x 3^k x samples), the unit of the paper's own figures.

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


def host_cpus() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def io_read_rate(d):
    """The input stage (Fig. 1) on the workload's dataset: its genotypes and
    classes written as text files (one line of digits per variant), then read
    back by the library's reader on the host.  Not part of the timed step."""
    import tempfile
    from paper_2201_03331_amd import fiuncho
    G = np.ascontiguousarray(d.genotypes, dtype=np.uint8)
    y = np.ascontiguousarray(d.phenotype, dtype=np.uint8)
    with tempfile.TemporaryDirectory() as tmp:
        gp, yp = os.path.join(tmp, "genotypes.txt"), os.path.join(tmp, "phenotype.txt")
        text = np.empty((G.shape[0], G.shape[1] + 1), dtype=np.uint8)
        text[:, :-1] = G + ord("0")
        text[:, -1] = ord("\n")
        with open(gp, "wb") as f:
            f.write(text.tobytes())
        with open(yp, "wb") as f:
            f.write((y + ord("0")).tobytes() + b"\n")
        nbytes = os.path.getsize(gp) + os.path.getsize(yp)
        fiuncho.lib()  # loaded before the clock starts
        t0 = time.perf_counter()
        G2, y2 = fiuncho.read_dataset(gp, yp)
        dt = time.perf_counter() - t0
    assert np.array_equal(G2, G) and np.array_equal(y2, y), "the reader changed the dataset"
    return {"read_s": round(dt, 4), "bytes": nbytes, "MB_per_s": round(nbytes / dt / 1e6, 1),
            "format": "text, one line of genotype digits per variant"}


def cpu_baseline(d, budget_s: float = 15.0):
    """The oracle (plain per-sample counting, FP64 MI) timed on every host CPU
    this process may use, over a contiguous sample of ranks of the same
    workload."""
    import oracle
    threads = host_cpus()
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
            "nproc": os.cpu_count(), "sample": f"lexicographic ranks [0, {count}) of the same dataset "
                                              f"({count / total:.3g} of C({d.n},{d.order})), {dt:.1f} s "
                                              f"on {threads} threads"}


KERNEL_NAMES = {1: "popcount", 2: "pairs", 3: "mfma", 4: "triples", 5: "mfma-fp4", 6: "mfma-fp4-tables"}


def arithmetic_of(kernels) -> str:
    """What the launched counting kernels compute in."""
    from paper_2201_03331_amd import fiuncho
    parts = []
    if kernels & {fiuncho.KERNEL_MFMA_FP4, fiuncho.KERNEL_MFMA_FP4_TABLES}:
        parts.append("{0,1}^k cells (or every prefix row, orders 4-5) as a one-hot FP4 (E2M1) "
                     "contraction on the matrix cores with FP32 accumulation (exact integer counts below 2^24)")
    if fiuncho.KERNEL_MFMA in kernels:
        parts.append("{0,1}^k cells as a one-hot int8 contraction on the matrix cores with int32 accumulation")
    if kernels & {fiuncho.KERNEL_POPCOUNT, fiuncho.KERNEL_PAIRS, fiuncho.KERNEL_TRIPLES}:
        parts.append("u64 bitset AND + u32 popcount counts")
    return ("; ".join(parts) + "; remaining cells by inclusion-exclusion from u32 class counts and lower-order "
            "tables; plain f32 MI estimate with a proven rounding bound for filtering; compensated f32 and "
            "f64 MI of the kept")


def measure(datasets, steps, warmup, graph=False, plain=False, shard=None):
    """Times `steps` steps (one search of every dataset each) after `warmup`
    untimed ones; returns the step time, the phase profile, the results and
    the roofline of the dominant counting kernel."""
    import torch
    from paper_2201_03331_amd import fiuncho

    sh = None if shard is None else [shard] * len(datasets)
    batches = ([fiuncho.DeviceBatch([d], shards=None if sh is None else [shard]) for d in datasets]
               if plain else [fiuncho.DeviceBatch(datasets, shards=sh)])
    stream = torch.cuda.current_stream()
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
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if warmup and not graph:
        fiuncho.get_profile()  # averages restart after the warm-up calls
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    fiuncho.set_profiling(False)
    ms = start.elapsed_time(end) / steps
    if graph:
        # events recorded by graph replays cannot be timed: the phase times of
        # a graph step come from one eager call right after the timed replays
        fiuncho.set_profiling(True)
        batches[0].run(stream)
        torch.cuda.synchronize()
        fiuncho.set_profiling(False)
    prof = fiuncho.get_profile()
    res = [r for b in batches for r in b.results()]
    ok = all(s == 0 for s, _ in res)

    def share(d):
        if shard is None:
            return math.comb(d.n, d.order)
        return int(fiuncho.shard_counts(d.n, d.m, d.order, shard[1], fiuncho.TILE_ROUND_ROBIN)[shard[0]])

    combos = sum(share(d) for d in datasets)
    combos_m = sum(share(d) * d.m for d in datasets)
    # table cells times samples: the unit of the paper's own throughput figures
    cells_m = sum(share(d) * 3 ** d.order * d.m for d in datasets)

    # roofline of the dominant counting kernel: algorithmic work per launch
    # over that kernel's measured time.  Popcount kernels: 32-bit VALU
    # lane-ops (4 per 64-bit AND+popcount).  Matrix-core kernels: operations
    # of the one-hot contraction, 2 x (4 or 8) cells x m samples per
    # combination, against the int8 or the FP4 peak (a batch with both: the
    # time both parts would take at their peaks).
    lane_ops = 0
    mfma_ops = 0
    mfma_peak_s = 0.0
    kernels = set()
    for d in datasets:
        m1 = int(d.phenotype.sum())
        kern = fiuncho.get_kernel(d.n, d.m, d.order)
        if kern == fiuncho.KERNEL_MFMA_FP4 and d.order >= 4 and d.m > 20447:
            kern = fiuncho.KERNEL_POPCOUNT  # the matrix cores take orders 4-5 up to 20,447 samples
        if kern == fiuncho.KERNEL_MFMA_FP4_TABLES and d.m >= 16384:
            # packed tables: fewer than 16,384 samples
            kern = (fiuncho.KERNEL_TRIPLES if d.order == 4 else
                    fiuncho.KERNEL_MFMA_FP4 if d.m <= 20447 else fiuncho.KERNEL_POPCOUNT)
        kernels.add(kern)
        if kern in (fiuncho.KERNEL_MFMA, fiuncho.KERNEL_MFMA_FP4, fiuncho.KERNEL_MFMA_FP4_TABLES):
            # cells counted on the matrix cores for every combination over
            # every sample: the {0,1}^k cells (2^k; the others come from class
            # counts and lower-order tables), on the rows kernel of orders 4
            # and 5 every prefix row against rows 0, 1 of the last variant
            # (2 * 3^(k-1))
            cells = (4 if d.order == 2 else 8 if d.order == 3 else 2 ** d.order if kern == fiuncho.KERNEL_MFMA_FP4_TABLES
                     else 2 * 3 ** (d.order - 1))
            ops = 2 * cells * d.m * share(d)
            mfma_ops += ops
            mfma_peak_s += ops / (MFMA_I8_PEAK_OPS if kern == fiuncho.KERNEL_MFMA else MFMA_FP4_PEAK_OPS)
        else:
            lane_ops += 4 * word_ops_per_combination(d.order, d.m - m1, m1, kern) * share(d)
    calls = len(batches) if plain else 1
    scan_ms = prof["scan_ms"] * calls
    mfma_ms = prof["mfma_ms"] * calls
    if mfma_ms > scan_ms:
        achieved = mfma_ops / (mfma_ms / 1e3) / 1e12
        peak = mfma_ops / mfma_peak_s / 1e12
        fp4 = bool(kernels & {fiuncho.KERNEL_MFMA_FP4, fiuncho.KERNEL_MFMA_FP4_TABLES})
        i8 = fiuncho.KERNEL_MFMA in kernels
        fmt = "int8 and FP4" if fp4 and i8 else "FP4" if fp4 else "int8"
        name = ("mfma_sub_kernel (one-hot FP4 contraction of the {0,1}^k cells + lower-order tables + FP32 MI "
                "+ filter)" if kernels == {fiuncho.KERNEL_MFMA_FP4_TABLES}
                else f"mfma_kernel (one-hot {fmt} contraction + FP32 MI + filter)")
        roofline = {"bound": "mfma", "kernel": name,
                    "achieved": achieved, "peak": peak, "unit": f"T {fmt} op/s", "frac": achieved / peak,
                    "kernel_ms": mfma_ms, "fmt": fmt}
    else:
        achieved = lane_ops / (scan_ms / 1e3) / 1e12
        peak = VALU_PEAK_LANE_OPS / 1e12
        roofline = {"bound": "alu", "kernel": "scan_kernel (AND+popcount counting + FP32 MI + filter)",
                    "achieved": achieved, "peak": peak, "unit": "T int32 lane-op/s", "frac": achieved / peak,
                    "kernel_ms": scan_ms, "fmt": None}
    planted_first = None
    if len(datasets) == 1 and shard is None and res[0][1].size:
        d0 = datasets[0]
        planted = [p for p in d0.planted if len(p) == d0.order]
        if planted:
            planted_first = tuple(int(v) for v in res[0][1][0]["snp"][: d0.order]) == planted[0]
    elif len(datasets) > 1 and shard is None:
        planted_first = all(h.size and tuple(int(v) for v in h[0]["snp"][: d.order]) == d.planted[0]
                            for d, (_, h) in zip(datasets, res))
    del batches
    torch.cuda.synchronize()
    return {"ms": ms, "prof": prof, "ok": ok, "combos": combos, "combos_m": combos_m, "cells_m": cells_m,
            "roofline": roofline,
            "kernels": kernels, "planted_first": planted_first}


# the per-workload block of a default run: (workload, steps, warm-up)
CONFIG_BLOCK = [("order2-100x1600", 50, 5), ("order2-4000x16000", 20, 3), ("batch64", 3, 1),
                ("batch64-plain", 3, 1), ("order4-200x4000", 10, 2), ("order5-200x4000", 2, 1)]


def launch_config(datasets):
    """The counting kernel and the waves per SIMD its launch asks for
    ("max": as many as fit) of each dataset shape, as the library chose them
    (its heuristic, or fiuncho_autotune / fiuncho_set_config)."""
    from paper_2201_03331_amd import fiuncho
    out = {}
    for d in datasets:
        key = f"order {d.order}, {d.n} x {d.m}"
        if key not in out and len(out) < 4:
            k, w = fiuncho.get_config(d.n, d.m, d.order)
            out[key] = {"kernel": KERNEL_NAMES[k], "waves_per_simd": w or "max"}
    return out


def summary(name, r, steps, warmup):
    rf = r["roofline"]
    return {"ms_per_step": round(r["ms"], 4), "steps": steps, "warmup": warmup,
            "combinations": r["combos"], "combinations_per_s": r["combos"] / (r["ms"] / 1e3),
            "combinations_x_samples_per_s": r["combos_m"] / (r["ms"] / 1e3),
            "cells_x_samples_per_s": r["cells_m"] / (r["ms"] / 1e3),
            "kernels": sorted(KERNEL_NAMES[k] for k in r["kernels"]),
            "dominant_kernel": rf["kernel"], "kernel_ms": round(rf["kernel_ms"], 4),
            "roofline_bound": rf["bound"], "roofline_frac": round(rf["frac"], 4),
            "status_ok": r["ok"], "planted_first": r["planted_first"],
            "phases_ms": {k: round(r["prof"][k], 4) for k in ("pack_ms", "pilot_ms", "scan_ms", "mfma_ms",
                                                               "select_ms", "total_ms")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the order-3 launch still shortens over its first ~10 back-to-back calls
    # (4.8 -> 4.1 ms while the clocks rise), so the default warms up longer
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="order3-1000x6400", choices=sorted(workloads().keys()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-workload block (the other workloads of the metric)")
    ap.add_argument("--kernel", default="auto", choices=("auto", "popcount", "pairs", "mfma", "mfma-fp4", "triples",
                                                         "mfma-fp4-tables"),
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
        print("bench.py runs on one GPU only: a search splits into per-GPU shares of its work "
              "tiles (fiuncho_job.shard_index / shard_count, timed here with --shard I/P), but "
              "no multi-GPU run is built", file=sys.stderr)
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
    if args.kernel != "auto":
        forced = {"popcount": fiuncho.KERNEL_POPCOUNT, "pairs": fiuncho.KERNEL_PAIRS,
                  "mfma": fiuncho.KERNEL_MFMA, "mfma-fp4": fiuncho.KERNEL_MFMA_FP4,
                  "triples": fiuncho.KERNEL_TRIPLES,
                  "mfma-fp4-tables": fiuncho.KERNEL_MFMA_FP4_TABLES}[args.kernel]
        for d in datasets:
            if fiuncho.lib().fiuncho_set_kernel(d.n, d.m, d.order, forced) != fiuncho.OK:
                ap.error(f"kernel {args.kernel} does not handle order {d.order}")
    tuned = {}
    if args.autotune:
        for d in datasets:
            key = (d.order, d.n.bit_length(), ((d.m + 63) // 64).bit_length())
            if key not in tuned:
                fiuncho.autotune(d.n, d.m, d.order)
                tuned[key] = fiuncho.get_config(d.n, d.m, d.order)
    shard = None
    if args.shard:
        si, sp = (int(v) for v in args.shard.split("/"))
        if not 0 <= si < sp:
            ap.error("--shard I/P needs 0 <= I < P")
        shard = (si, sp)
    r = measure(datasets, args.steps, args.warmup, graph=args.workload == "batch64",
                plain=args.workload.endswith("-plain"), shard=shard)
    ms, prof, kernels = r["ms"], r["prof"], r["kernels"]
    rf = dict(r["roofline"])
    # the counter table's workload key (a shard launches fewer tiles); it holds
    # the FP4 matrix-core kernels' and the pair- and triple-table kernels' launches
    traffic_key = args.workload + ("" if shard is None else f" shard {shard[0]}/{shard[1]}")
    if rf["bound"] == "mfma":
        rf["traffic"] = (measured_traffic(rf["kernel"].split()[0], traffic_key) if rf["fmt"] == "FP4" else None)
    else:
        rf["traffic"] = (measured_traffic("scan_kernel", traffic_key)
                         if kernels <= {fiuncho.KERNEL_PAIRS, fiuncho.KERNEL_TRIPLES} else None)
    rf["kernel_ms"] = round(rf["kernel_ms"], 4)
    del rf["fmt"]
    d0 = datasets[0]
    out = {
        "metric": METRIC,
        "value": r["combos"] / (ms / 1e3),
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
            "combinations": r["combos"],
            "calls_per_step": len(datasets) if args.workload.endswith("-plain") else 1,
            "shard": None if shard is None else f"{shard[0]}/{shard[1]}",
        },
        "combinations_x_samples_per_s": r["combos_m"] / (ms / 1e3),
        "cells_x_samples_per_s": r["cells_m"] / (ms / 1e3),
        "arithmetic": arithmetic_of(kernels),
        "phases_ms": {k: round(prof[k], 4) for k in ("pack_ms", "pilot_ms", "scan_ms", "mfma_ms",
                                                     "select_ms", "total_ms")},
        "kernels": sorted(KERNEL_NAMES[k] for k in kernels),
        "launch_config": launch_config(datasets),
        "autotuned": {f"order {k[0]}, snps < 2^{k[1]}, words < 2^{k[2]}":
                      {"kernel": KERNEL_NAMES[v[0]], "waves_per_simd": v[1] or "max"}
                      for k, v in sorted(tuned.items())} if args.autotune else None,
        "candidates": prof["candidates"],
        "rescored": prof["kept"],
        "status_ok": r["ok"],
        "planted_first": r["planted_first"],
        "roofline": rf,
    }
    del datasets
    if not args.no_configs and args.workload == "order3-1000x6400" and shard is None and args.kernel == "auto":
        block = {}
        for name, steps, warm in CONFIG_BLOCK:
            ds = workloads()[name]()
            rc = measure(ds, steps, warm, graph=name == "batch64", plain=name.endswith("-plain"))
            block[name] = summary(name, rc, steps, warm)
            del ds
            torch.cuda.empty_cache()
            print(f"bench: {name} {rc['ms']:.3f} ms/step", file=sys.stderr, flush=True)
        block["batch64"]["speedup_vs_plain"] = round(block["batch64-plain"]["ms_per_step"] /
                                                     block["batch64"]["ms_per_step"], 4)
        out["configs"] = block
    if not args.no_cpu_baseline and len(d0.genotypes) and args.workload != "batch64" and \
            not args.workload.endswith("-plain") and shard is None:
        out["cpu_baseline"] = cpu_baseline(d0)
    if len(d0.genotypes) and args.workload != "batch64" and not args.workload.endswith("-plain") and \
            shard is None:
        out["io"] = io_read_rate(d0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
