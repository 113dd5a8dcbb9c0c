"""Benchmark of the ES-BGK stream-collide step on one MI355X.

Prints one JSON line.  The headline workload is a 4096 x 4096 periodic D2Q37
domain with both populations stored in FP32 (N_f = 3, Pr = 0.71, tau = 0.6,
superposed shear and thermal waves plus seeded noise); a step is one fused
stream-collide launch over the whole grid with inputs resident in HBM, in the
two-copy pull streaming scheme.  `value` is million lattice-cell updates per
second (MLUPS) over exactly --steps timed steps.  Variants (the same workload
with A-A in-place streaming, FP16/BF16 deviation storage, D3Q39 at 256^3,
the batched 256-domain workload in its execution modes) are reported beside
it, each with its HBM-roofline fraction.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--variants aa,f16,bf16,d3q39,batch]
                    [--no-variants] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % of HBM peak, FP32 vs FP16-storage vs batched, at stated error vs FP64"
HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_step_d2q37_f32_4096_traffic.json")


def kernel_source_hash() -> str:
    """Hash of the step kernels' source with comments and blank space
    removed, so that a traffic summary stays valid across comment edits and
    is dropped when the code changes."""
    import re
    h = hashlib.sha256()
    for f in ("kernels.hpp", "ops_impl.hpp"):
        with open(os.path.join(ROOT, "paper_1611_02409_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_cell(Q, npop, storage):
    return 2 * Q * npop * (4 if storage == "f32" else 2)


def time_single(esb, torch, D, Q, Nf, Pr, tau, dims, storage, fields, steps, warmup, tune_cache, streaming="pull"):
    log(f"D{D}Q{Q} {dims} {storage} {streaming}: init")
    lat = esb.Lattice(D, Q, Nf, Pr, tau, dims, storage=storage, streaming=streaming)
    lat.init_fields(*fields)
    tile = lat.autotune(cache_path=tune_cache)
    log(f"D{D}Q{Q} {dims} {storage} {streaming}: tile {tile}, timing {steps} steps")
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_ms, per = lat.step_timed(steps)       # HIP events around every launch, on the lattice's stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ncell = int(np.prod(dims))
    # after `warmup` steps the first timed launch has parity warmup % 2
    first_odd = warmup % 2 == 1
    odd = per[0::2] if first_odd else per[1::2]
    even = per[1::2] if first_odd else per[0::2]
    return dict(lat=lat, tile=tile, total_ms=total_ms, wall_s=wall, ncell=ncell,
                mlups=ncell * steps / (total_ms * 1e-3) / 1e6, odd_ms=float(np.mean(odd)),
                even_ms=float(np.mean(even)), launch_ms=float(np.mean(per)))


def roofline(bytes_per_launch, launch_ms, peak=HBM_PEAK_GBS, traffic=None):
    ach = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": peak, "unit": "GB/s", "frac": round(ach / peak, 4),
            "traffic": traffic}


def measured_traffic(kernel):
    """HBM bytes per launch of one FP32 D2Q37 4096^2 step kernel ("pull",
    "aa_even" or "aa_odd") from the committed rocprofv3 counter summary, if it
    was taken from the current kernel source; otherwise None."""
    try:
        with open(PROFILE_TRAFFIC) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


def _counter_rows(d):
    """Counter records of every rocprofv3 output under directory d: the
    SQLite (rocpd) databases rocprofv3 writes by default, or CSV files."""
    import csv
    import glob
    import sqlite3
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
        db = sqlite3.connect(path)
        for name, counter, value, disp, grid in db.execute(
                "select kernel_name, counter_name, value, dispatch_id, grid_size from counters_collection"):
            rows.append({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value,
                         "Dispatch_Id": f"{path}:{disp}", "Grid_Size": grid})
        db.close()
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter, match, grid=None):
    """Sum of `counter` (KiB) per dispatch of kernels whose name contains all
    of `match` (and, if given, whose grid has `grid` work-items)."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter or not all(m in r.get("Kernel_Name", "") for m in match):
            continue
        if grid is not None and int(r.get("Grid_Size", grid)) != grid:
            continue
        k = r.get("Dispatch_Id") or r.get("Correlation_Id")
        out[k] = out.get(k, 0.0) + float(r["Counter_Value"])
    return list(out.values())


# demangled-name prefixes of the FP32 (storage 0) D2Q37 step kernels with
# both populations, by layout (0 A-A even, 1 A-A odd, 2 pull)
STEP_KERNELS = {"pull": "k_step<esbgk::LatD2Q37, 0, 2, true,", "aa_even": "k_step<esbgk::LatD2Q37, 0, 0, true,",
                "aa_odd": "k_step<esbgk::LatD2Q37, 0, 1, true,"}


def ingest_counters(fetch_dir, write_dir, ncell=4096 * 4096):
    """Turn two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) into HBM bytes per launch of the FP32
    D2Q37 step kernels, each counter scaled by what it reads for the
    arithmetic-free stream kernel of known size (74 FP32 planes read and
    written once), and store them with the kernel source hash."""
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    ref = ("k_stream_rw",)
    known = 74 * ncell * 4
    sf = np.median(_per_dispatch(fr, "FETCH_SIZE", ref)) * 1024 / known
    sw = np.median(_per_dispatch(wr, "WRITE_SIZE", ref)) * 1024 / known
    bpl = bytes_per_cell(37, 2, "f32") * ncell
    kernels = {}
    for name, prefix in STEP_KERNELS.items():
        fd = _per_dispatch(fr, "FETCH_SIZE", (prefix,), ncell)
        wd = _per_dispatch(wr, "WRITE_SIZE", (prefix,), ncell)
        if not fd or not wd:
            continue
        f, w = np.median(fd) * 1024, np.median(wd) * 1024
        kernels[name] = {"fetch_bytes_raw": f, "write_bytes_raw": w, "dispatches": [len(fd), len(wd)],
                         "hbm_bytes_per_launch": f / sf + w / sw,
                         "traffic_over_algorithmic": (f / sf + w / sw) / bpl}
    res = {"workload": "D2Q37 4096x4096 FP32 f+g", "algorithmic_bytes_per_launch": bpl,
           "stream_kernel_fetch_factor": sf, "stream_kernel_write_factor": sw, "kernels": kernels,
           "kernel_source_hash": kernel_source_hash(),
           "commands": [f"rocprofv3 --pmc FETCH_SIZE -d {fetch_dir} -- python3 bench.py --steps 6 --warmup 2 "
                        "--variants aa --no-cpu",
                        f"rocprofv3 --pmc WRITE_SIZE -d {write_dir} -- python3 bench.py --steps 6 --warmup 2 "
                        "--variants aa --no-cpu",
                        f"python bench.py --ingest-counters {fetch_dir} {write_dir}"]}
    with open(PROFILE_TRAFFIC, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def _oracle_rate(n, threads, seconds, max_steps):
    import oracle
    import workloads
    oracle.set_threads(threads)
    sim = oracle.Sim(2, 37, 3, 0.71, 0.6, (n, n))
    sim.init(*workloads.waves_noise_2d(n))
    steps = 0
    t0 = time.perf_counter()
    while True:
        sim.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds or steps >= max_steps:
            break
    return n * n * steps / el / 1e6, steps, el


def cpu_baseline(seconds=12.0):
    """The FP64 oracle on the host: D2Q37, N_f = 3, 1024^2 periodic, same
    initial recipe, as many whole steps as fit in about `seconds`, on the
    host's cores (at most 16, the share of one GPU), and on one thread for a
    third of that time."""
    threads = min(16, os.cpu_count() or 1)
    v, steps, el = _oracle_rate(1024, threads, seconds, 200)
    v1, steps1, el1 = _oracle_rate(1024, 1, seconds / 3, 200)
    return {"value": round(v, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, D2Q37 1024x1024 periodic, N_f=3, Pr=0.71, tau=0.6, {steps} steps in {el:.1f} s "
                      f"on {threads} threads; {steps1} steps in {el1:.1f} s on 1 thread",
            "single_thread_value": round(v1, 3)}


VARIANTS = ("aa", "pr", "f16", "bf16", "d3q39", "d2q33", "batch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variants", default=",".join(VARIANTS),
                    help="comma list of variants to time beside the headline: " + ",".join(VARIANTS))
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the HBM-traffic summary from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (the batched and single-domain paths have no "
              "multi-GPU mode); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    variants = set() if args.no_variants else {v for v in args.variants.split(",") if v}
    unknown = variants - set(VARIANTS)
    if unknown:
        ap.error(f"unknown variants {sorted(unknown)}")

    import torch
    import paper_1611_02409_amd as esb
    import workloads

    tune_cache = None   # tune afresh each run (about a second per workload)
    N = 4096
    D, Q, Nf, Pr, tau = 2, 37, 3, 0.71, 0.6
    fields = workloads.waves_noise_2d(N)
    bpl = bytes_per_cell(Q, 2, "f32") * N * N

    # headline: two-copy pull streaming, FP32
    main_run = time_single(esb, torch, D, Q, Nf, Pr, tau, (N, N), "f32", fields, args.steps, args.warmup, tune_cache)
    roof = roofline(bpl, main_run["launch_ms"], traffic=measured_traffic("pull"))
    roof["kernel"] = "k_step<D2Q37, FP32, pull layout> (the one kernel of every step)"
    roof["bytes_per_launch"] = bpl
    roof["avg_launch_ms"] = round(main_run["launch_ms"], 4)
    step_ms = main_run["total_ms"] / args.steps
    out = {
        "metric": METRIC,
        "value": round(main_run["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D2Q37 4096x4096 periodic, f and g populations FP32 SoA, N_f=3 (gamma=1.4), "
                               "Pr=0.71, tau=0.6, kappa=0.2, shear+thermal waves (amplitude 1e-3) + N(0,1e-5^2) "
                               "noise seed 1611",
                   "lattice": "D2Q37", "grid": [N, N], "storage": "f32", "N_f": Nf, "Pr": Pr, "tau": tau,
                   "streaming": "two-copy pull (reads x - c_i, aligned writes; bitwise equal to A-A in place)",
                   "tile": {p: dict(zip(("block", "order", "policy", "cells_per_item"), t))
                            for p, t in zip(("even_step", "odd_step"), main_run["tile"])},
                   "algorithmic_bytes_per_cell_step": bytes_per_cell(Q, 2, "f32"),
                   "hbm_GBs_per_step_avg": round(bpl / (step_ms * 1e-3) / 1e9, 1)},
        "roofline": roof,
    }
    del main_run
    torch.cuda.empty_cache()

    var = {}
    if "aa" in variants:
        r = time_single(esb, torch, D, Q, Nf, Pr, tau, (N, N), "f32", fields, args.steps, args.warmup, tune_cache,
                        streaming="aa")
        var["d2q37_4096_f32_aa_in_place"] = {
            "mlups": round(r["mlups"], 1), "ms_per_step": round(r["total_ms"] / args.steps, 4),
            "even_kernel": {"avg_launch_ms": round(r["even_ms"], 4),
                            "frac_of_hbm_peak": round(bpl / (r["even_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "traffic": measured_traffic("aa_even")},
            "odd_kernel": {"avg_launch_ms": round(r["odd_ms"], 4),
                           "frac_of_hbm_peak": round(bpl / (r["odd_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "traffic": measured_traffic("aa_odd")},
            "tile": r["tile"]}
        del r
        torch.cuda.empty_cache()
    if "pr" in variants:
        # the same workload at the other two Prandtl numbers (same kernel,
        # other omega and nu)
        for pr in (0.5, 2.0):
            r = time_single(esb, torch, D, Q, Nf, pr, tau, (N, N), "f32", fields, args.steps, args.warmup,
                            tune_cache)
            var[f"d2q37_4096_f32_pr{pr:g}"] = {"mlups": round(r["mlups"], 1),
                                               "roofline_frac": round(bpl / (r["launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                               "streaming": "pull", "tile": r["tile"]}
            del r
            torch.cuda.empty_cache()
    for storage in ("f16", "bf16"):
        if storage not in variants:
            continue
        r = time_single(esb, torch, D, Q, Nf, Pr, tau, (N, N), storage, fields, args.steps, args.warmup, tune_cache)
        b = bytes_per_cell(Q, 2, storage) * N * N
        var[f"d2q37_4096_{storage}_dev"] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["total_ms"] / args.steps, 4),
                                            "roofline_frac": round(b / (r["launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                            "GBs_per_step": round(b / (r["total_ms"] / args.steps * 1e-3) / 1e9, 1),
                                            "streaming": "pull", "tile": r["tile"]}
        del r
        torch.cuda.empty_cache()
    del fields
    if "d3q39" in variants:
        # D3Q39 256^3 thermal Taylor-Green vortex, FP32
        n3 = 256
        f3 = workloads.taylor_green_3d(n3)
        s3 = max(50, args.steps // 2)
        r = time_single(esb, torch, 3, 39, 2, 0.71, 0.7, (n3, n3, n3), "f32", f3, s3, args.warmup, tune_cache)
        b = bytes_per_cell(39, 2, "f32") * n3 ** 3
        var["d3q39_256cube_f32"] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["total_ms"] / s3, 4),
                                    "roofline_frac": round(b / (r["launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                    "GBs_per_step": round(b / (r["total_ms"] / s3 * 1e-3) / 1e9, 1),
                                    "streaming": "pull", "tile": r["tile"]}
        del r
        torch.cuda.empty_cache()
        # the same vortex with BF16 deviation storage (f and g paired)
        r = time_single(esb, torch, 3, 39, 2, 0.71, 0.7, (n3, n3, n3), "bf16", f3, s3, args.warmup, tune_cache)
        b = bytes_per_cell(39, 2, "bf16") * n3 ** 3
        var["d3q39_256cube_bf16"] = {"mlups": round(r["mlups"], 1),
                                     "roofline_frac": round(b / (r["launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                     "streaming": "pull", "tile": r["tile"]}
        del r, f3
        torch.cuda.empty_cache()
    if "d2q33" in variants:
        # the shock-tube lattice (|c| up to 4) on the 4096^2 wave workload, FP32
        n2 = 4096
        f2 = workloads.waves_noise_2d(n2)
        r = time_single(esb, torch, 2, 33, 3, 0.71, 0.6, (n2, n2), "f32", f2, max(50, args.steps // 2), args.warmup,
                        tune_cache)
        b = bytes_per_cell(33, 2, "f32") * n2 * n2
        var["d2q33_4096_f32"] = {"mlups": round(r["mlups"], 1),
                                 "roofline_frac": round(b / (r["launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "streaming": "pull", "tile": r["tile"]}
        del r, f2
        torch.cuda.empty_cache()
    if "batch" in variants:
        var["batched_256_d2q37_f32"] = time_batch(esb, torch, workloads, args.batch_steps, tune_cache)
        torch.cuda.empty_cache()
    if var:
        out["variants"] = var

    # the arithmetic-free copy kernel of the same pattern, last: its buffer is
    # allocated and freed outside the timed lattices
    log("stream ceiling")
    ceiling = esb.stream_ceiling(N * N, 10)
    roof["measured_stream_ceiling_GBs"] = round(ceiling, 1)
    roof["frac_of_measured_ceiling"] = round(roof["achieved"] / ceiling, 4)

    if not args.no_cpu:
        log("cpu baseline (FP64 oracle on the host)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def time_batch(esb, torch, workloads, batch_steps, tune_cache):
    """256 independent domains (A-A in place) in the three execution modes
    with the autotuned launch shape, plus the persistent launch advancing
    MALL-sized domain groups."""
    doms = workloads.batch_domains(256)
    bt = esb.Batch(2, 37, [dict(dims=(d["nx"], d["ny"]), Nf=d["Nf"], Pr=d["Pr"], tau=d["tau"]) for d in doms])
    for k, d in enumerate(doms):
        bt.init_fields(k, *workloads.batch_fields(d))
    cells, bps = bt.info()
    block, policy = bt.autotune(cache_path=tune_cache)
    log(f"batch autotune: block {block}, policy {policy}")
    res = {"tile": {"block": block, "policy": policy}}

    def run(name, mode, n):
        bt.step(n if mode != 2 else 20, mode)          # warm-up (captures the graph of n steps)
        torch.cuda.synchronize()
        ms = bt.step_timed(n, mode)
        if bt.status() != 0:
            raise RuntimeError("persistent batch kernel reported a timed-out wait")
        res[name] = {"mlups": round(cells * n / (ms * 1e-3) / 1e6, 1), "steps": n,
                     "GBs": round(bps * n / (ms * 1e-3) / 1e9, 1),
                     "frac_of_hbm_peak": round(bps * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    for mode, name in ((0, "persistent_graph"), (1, "graph_per_step")):
        log(f"batch {len(doms)} domains, {cells} cells: mode {name}, {batch_steps} steps")
        run(name, mode, batch_steps)
    # the per-domain loop at its own best work-group size (the tuned shape of
    # the persistent launch need not suit one launch per domain)
    best = None
    for blk, pol in sorted({(256, 0), (512, 0), (block, policy)}):
        bt.set_tile(blk, pol)
        log(f"batch {len(doms)} domains: mode per_domain_loop, block {blk} policy {pol}, {batch_steps} steps")
        run("per_domain_loop", 2, batch_steps)
        r = res.pop("per_domain_loop")
        if best is None or r["mlups"] > best["mlups"]:
            best = dict(r, tile={"block": blk, "policy": pol})
    res["per_domain_loop"] = best
    # the same persistent launch, advancing groups of domains (about 128 MB
    # of storage each) eight steps at a time while they sit in the MALL
    bt.set_tile(block, policy, 8, 128e6)
    ng = max(8, batch_steps // 5)
    log(f"batch: persistent, domain groups of 128 MB advanced 8 steps at a time, {ng} steps")
    run("persistent_graph_grouped", 0, ng)
    res["persistent_graph_grouped"].update(window=8, group_bytes=128e6)
    res["cells"] = cells
    res["domains"] = len(doms)
    res["speedup_vs_per_domain_loop"] = round(res["persistent_graph"]["mlups"] / res["per_domain_loop"]["mlups"], 3)
    del bt
    return res


if __name__ == "__main__":
    main()
