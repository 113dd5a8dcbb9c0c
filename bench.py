"""Benchmark of the ES-BGK stream-collide step on one MI355X.

Prints one JSON line.  The headline workload is a 4096 x 4096 periodic D2Q37
domain with both populations stored in FP32 (N_f = 3, Pr = 0.71, tau = 0.6,
superposed shear and thermal waves plus seeded noise); a step is one fused
stream-collide launch over the whole grid with inputs resident in HBM, in the
two-copy pull streaming scheme.  `value` is million lattice-cell updates per
second (MLUPS) over exactly --steps timed steps.  Variants (the same workload
with A-A in-place streaming, FP16/BF16 deviation storage, D3Q39 at 256^3,
D2Q33, the batched 256-domain workload in its execution modes and both
streaming schemes) are reported beside it, each with its HBM-roofline
fraction.

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
PROFILE_DIR = os.path.join(ROOT, "profiles")


def traffic_path(lattice):
    """Committed HBM-traffic summary of the FP32 step kernels of one
    benchmark workload (D2Q37 4096^2 or D3Q39 256^3, 2^24 cells each)."""
    size = "4096" if lattice == "D2Q37" else "256cube"
    return os.path.join(PROFILE_DIR, f"k_step_{lattice.lower()}_f32_{size}_traffic.json")


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


PAD_CANDIDATES = (0, 16384, 24576, 49152)   # plane padding, bytes


def time_single(esb, torch, D, Q, Nf, Pr, tau, dims, storage, fields, steps, warmup, tune_cache, streaming="pull"):
    """Autotune the launch shape, pick the plane padding (the candidate
    layout with the highest rate over a short run, keeping the allocation
    that was measured), tune the launch shape again on it, then time `steps`
    steps after `warmup` from the initial state."""
    log(f"D{D}Q{Q} {dims} {storage} {streaming}: init")
    ncell = int(np.prod(dims))
    best, tile, pad_rates = None, None, {}
    for pad in PAD_CANDIDATES:
        lat = esb.Lattice(D, Q, Nf, Pr, tau, dims, storage=storage, streaming=streaming, plane_pad=pad)
        lat.init_fields(*fields)
        if tile is None:
            tile = lat.autotune(cache_path=tune_cache)
        else:
            lat.set_tile(*tile[0], parity=0)
            lat.set_tile(*tile[1], parity=1)
        lat.step(4)
        ms, _ = lat.step_timed(40)
        pad_rates[pad] = round(ncell * 40 / (ms * 1e-3) / 1e6, 1)
        if best is None or pad_rates[pad] > pad_rates[best[0]]:
            best = (pad, lat)
        del lat
        torch.cuda.empty_cache()
    pad, lat = best
    lat.init_fields(*fields)
    if pad != PAD_CANDIDATES[0]:
        tile = lat.autotune(cache_path=tune_cache)     # launch shape again, on the chosen allocation
    log(f"D{D}Q{Q} {dims} {storage} {streaming}: tile {tile}, plane pad {pad} ({pad_rates}), timing {steps} steps")
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_ms, per = lat.step_timed(steps)       # HIP events around every launch, on the lattice's stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # after `warmup` steps the first timed launch has parity warmup % 2
    first_odd = warmup % 2 == 1
    odd = per[0::2] if first_odd else per[1::2]
    even = per[1::2] if first_odd else per[0::2]
    return dict(lat=lat, tile=tile, plane_pad=pad, pad_rates=pad_rates, total_ms=total_ms, wall_s=wall, ncell=ncell,
                mlups=ncell * steps / (total_ms * 1e-3) / 1e6, odd_ms=float(np.mean(odd)),
                even_ms=float(np.mean(even)), launch_ms=float(np.mean(per)))


GOLDEN_4096 = os.path.join(ROOT, "tests", "golden", "ref_waves4096_pr0.71.npz")


def error_vs_fp64(lat, fields, steps=1000):
    """The stated error of a 4096^2 D2Q37 waves run (N_f = 3, Pr = 0.71,
    tau = 0.6): relative L2 of rho, u and T, as 512^2 block means, after
    `steps` steps from the initial state, against the stored FP64 oracle run
    of the same workload (tests/golden, written by a script that calls only
    the oracle), and the relative drift of the FP64 totals of mass and
    energy.  None if the reference is missing."""
    import workloads
    if not os.path.exists(GOLDEN_4096):
        return None
    ref = np.load(GOLDEN_4096)
    if f"rho_{steps}" not in ref.files:
        return None
    out_n = int(ref["out_n"])

    def rel_l2(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    lat.init_fields(*fields)
    t0 = lat.totals()
    lat.step(steps)
    t1 = lat.totals()
    m = lat.read_moments()
    bm = lambda a: workloads.block_mean(a, out_n)
    e_rho = rel_l2(1.0 + bm(m["rho"] - 1.0), 1.0 + ref[f"rho_{steps}"].astype(np.float64))
    e_T = rel_l2(1.0 + bm(m["T"] - 1.0), 1.0 + ref[f"T_{steps}"].astype(np.float64))
    e_u = rel_l2(np.stack([bm(m["u"][0]), bm(m["u"][1])]),
                 np.stack([ref[f"ux_{steps}"], ref[f"uy_{steps}"]]).astype(np.float64))
    return {"steps": steps, "reference": "FP64 oracle, 512^2 block means", "rho": float(f"{e_rho:.3g}"),
            "u": float(f"{e_u:.3g}"), "T": float(f"{e_T:.3g}"),
            "mass_drift": float(f"{abs(t1[0] - t0[0]) / t0[0]:.3g}"),
            "energy_drift": float(f"{abs(t1[-1] - t0[-1]) / t0[-1]:.3g}")}


def roofline(bytes_per_launch, launch_ms, peak=HBM_PEAK_GBS, traffic=None):
    ach = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": peak, "unit": "GB/s", "frac": round(ach / peak, 4),
            "traffic": traffic}


# kernel cache-policy template argument of each ABI cache policy (1 default,
# 2 non-temporal loads and stores, 3 non-temporal stores)
CP_OF_POLICY = {1: 0, 2: 2, 3: 3}
LAYOUT_NAMES = {0: "aa_even", 1: "aa_odd", 2: "pull"}


def traffic_key(layout, cp, block, cpi):
    return f"{layout} cp{cp} wg{block} cpi{cpi}"


def measured_traffic(layout, tile, lattice="D2Q37"):
    """HBM bytes per launch of one FP32 step kernel (layout "pull",
    "aa_even" or "aa_odd"; tile = (block, order, policy, cells_per_item) as
    the autotuner reports it) from the committed rocprofv3 counter summary,
    if that summary holds this launch shape and was taken from the current
    kernel source; otherwise None."""
    try:
        with open(traffic_path(lattice)) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    block, _, policy, cpi = tile
    key = traffic_key(layout, CP_OF_POLICY.get(policy, -1), block, cpi)
    return d.get("kernels", {}).get(key, {}).get("hbm_bytes_per_launch")


def pull_traffic(tiles, lattice="D2Q37"):
    """Mean HBM bytes per launch of the pull kernel over the even- and
    odd-step launch shapes (None unless both were measured)."""
    t = [measured_traffic("pull", tuple(x), lattice) for x in tiles]
    return None if None in t else round(float(np.mean(t)))


def _counter_rows(d):
    """Counter records of every rocprofv3 output under directory d: the
    SQLite (rocpd) databases rocprofv3 writes by default, or CSV files."""
    import csv
    import glob
    import sqlite3
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
        db = sqlite3.connect(path)
        for name, counter, value, disp, grid, wg in db.execute(
                "select kernel_name, counter_name, value, dispatch_id, grid_size, workgroup_size "
                "from counters_collection"):
            rows.append({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value,
                         "Dispatch_Id": f"{path}:{disp}", "Grid_Size": grid, "Workgroup_Size": wg})
        db.close()
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter, match):
    """Sum of `counter` (KiB) per dispatch of kernels whose name contains all
    of `match`, grouped by (kernel name, grid size, work-group size)."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter or not all(m in r.get("Kernel_Name", "") for m in match):
            continue
        g = (r["Kernel_Name"], int(r.get("Grid_Size", 0)), int(r.get("Workgroup_Size", 0)))
        k = r.get("Dispatch_Id") or r.get("Correlation_Id")
        out.setdefault(g, {})
        out[g][k] = out[g].get(k, 0.0) + float(r["Counter_Value"])
    return {g: list(v.values()) for g, v in out.items()}


def ingest_counters(fetch_dir, write_dir, lattice="D2Q37", ncell=4096 * 4096):
    """Turn two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) into HBM bytes per launch of the FP32 step
    kernels of one lattice, per launch shape (layout, cache policy,
    work-group size, cells per work-item), each counter scaled by what it
    reads for the arithmetic-free stream kernel of known size (74 FP32 planes
    of 2^24 cells read and written once), and store them with the kernel
    source hash."""
    import re
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    known = 74 * ncell * 4

    def median_all(groups):
        return np.median([v for vals in groups.values() for v in vals])

    sf = median_all(_per_dispatch(fr, "FETCH_SIZE", ("k_stream_rw",))) * 1024 / known
    sw = median_all(_per_dispatch(wr, "WRITE_SIZE", ("k_stream_rw",))) * 1024 / known
    Q = int(lattice.split("Q")[1])
    bpl = bytes_per_cell(Q, 2, "f32") * ncell
    pat = re.compile(r"k_step<esbgk::Lat" + lattice + r", 0, (\d), true, (\d),")
    fd = _per_dispatch(fr, "FETCH_SIZE", (f"k_step<esbgk::Lat{lattice}, 0, ",))
    wd = _per_dispatch(wr, "WRITE_SIZE", (f"k_step<esbgk::Lat{lattice}, 0, ",))
    kernels = {}
    for g in sorted(set(fd) & set(wd), key=str):
        m = pat.search(g[0])
        if not m or ncell % g[1]:
            continue
        key = traffic_key(LAYOUT_NAMES[int(m.group(1))], int(m.group(2)), g[2], ncell // g[1])
        f, w = np.median(fd[g]) * 1024, np.median(wd[g]) * 1024
        kernels[key] = {"fetch_bytes_raw": f, "write_bytes_raw": w, "dispatches": [len(fd[g]), len(wd[g])],
                        "hbm_bytes_per_launch": f / sf + w / sw,
                        "traffic_over_algorithmic": (f / sf + w / sw) / bpl}
    variant = "aa" if lattice == "D2Q37" else "d3q39"
    workload = "D2Q37 4096x4096" if lattice == "D2Q37" else "D3Q39 256x256x256"
    res = {"workload": f"{workload} FP32 f+g", "algorithmic_bytes_per_launch": bpl,
           "key": "layout, cache-policy template argument (0 default, 2 non-temporal loads and stores, "
                  "3 non-temporal stores), work-group size, cells per work-item",
           "stream_kernel_fetch_factor": sf, "stream_kernel_write_factor": sw, "kernels": kernels,
           "kernel_source_hash": kernel_source_hash(),
           "commands": [f"rocprofv3 --pmc FETCH_SIZE -d {fetch_dir} -- python3 bench.py --steps 6 --warmup 2 "
                        f"--variants {variant} --no-cpu",
                        f"rocprofv3 --pmc WRITE_SIZE -d {write_dir} -- python3 bench.py --steps 6 --warmup 2 "
                        f"--variants {variant} --no-cpu",
                        f"python bench.py --ingest-counters {fetch_dir} {write_dir} --lattice {lattice}"]}
    with open(traffic_path(lattice), "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps({k: round(v["traffic_over_algorithmic"], 4) for k, v in kernels.items()}, indent=1))


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
    ap.add_argument("--lattice", default="D2Q37", choices=("D2Q37", "D3Q39"),
                    help="lattice whose step kernels --ingest-counters summarises")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters, lattice=args.lattice)
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
    roof = roofline(bpl, main_run["launch_ms"], traffic=pull_traffic(main_run["tile"]))
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
                   "plane_pad": main_run["plane_pad"],
                   "plane_pad_MLUPS_40_steps": main_run["pad_rates"],
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
                            "traffic": measured_traffic("aa_even", r["tile"][0])},
            "odd_kernel": {"avg_launch_ms": round(r["odd_ms"], 4),
                           "frac_of_hbm_peak": round(bpl / (r["odd_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "traffic": measured_traffic("aa_odd", r["tile"][1])},
            "tile": r["tile"], "plane_pad": r["plane_pad"],
            "plane_pad_MLUPS_40_steps": r["pad_rates"]}
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
                                               "streaming": "pull", "tile": r["tile"], "plane_pad": r["plane_pad"],
            "plane_pad_MLUPS_40_steps": r["pad_rates"]}
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
                                            "streaming": "pull", "tile": r["tile"], "plane_pad": r["plane_pad"],
            "plane_pad_MLUPS_40_steps": r["pad_rates"]}
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
                                    "traffic": pull_traffic(r["tile"], "D3Q39"),
                                    "streaming": "pull", "tile": r["tile"], "plane_pad": r["plane_pad"],
            "plane_pad_MLUPS_40_steps": r["pad_rates"]}
        del r
        torch.cuda.empty_cache()
        # the same vortex with BF16 deviation storage (f and g paired)
        r = time_single(esb, torch, 3, 39, 2, 0.71, 0.7, (n3, n3, n3), "bf16", f3, s3, args.warmup, tune_cache)
        b = bytes_per_cell(39, 2, "bf16") * n3 ** 3
        var["d3q39_256cube_bf16"] = {"mlups": round(r["mlups"], 1),
                                     "roofline_frac": round(b / (r["launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                     "streaming": "pull", "tile": r["tile"], "plane_pad": r["plane_pad"],
            "plane_pad_MLUPS_40_steps": r["pad_rates"]}
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
                                 "streaming": "pull", "tile": r["tile"], "plane_pad": r["plane_pad"],
            "plane_pad_MLUPS_40_steps": r["pad_rates"]}
        del r, f2
        torch.cuda.empty_cache()
    if "batch" in variants:
        var["batched_256_d2q37_f32"] = time_batch(esb, torch, workloads, args.batch_steps, tune_cache, "pull")
        torch.cuda.empty_cache()
        var["batched_256_d2q37_f32_aa"] = time_batch(esb, torch, workloads, args.batch_steps, tune_cache, "aa",
                                                     grouped=True)
        torch.cuda.empty_cache()
    if var:
        out["variants"] = var

    # the stated error of the 4096^2 runs against the FP64 oracle, after the
    # timed work (fresh lattices: results do not depend on the launch shape
    # or the plane padding)
    fields = workloads.waves_noise_2d(N)
    for storage in ("f32", "f16", "bf16"):
        if storage != "f32" and storage not in variants:
            continue
        log(f"error of the {storage} run against the FP64 oracle (1000 steps)")
        lat = esb.Lattice(D, Q, Nf, Pr, tau, (N, N), storage=storage, streaming="pull")
        err = error_vs_fp64(lat, fields)
        if storage == "f32":
            out["error_vs_fp64"] = err
        else:
            var[f"d2q37_4096_{storage}_dev"]["error_vs_fp64"] = err
        del lat
        torch.cuda.empty_cache()
    del fields

    # the arithmetic-free copy kernel of the same pattern, last: its buffer is
    # allocated and freed outside the timed lattices
    log("stream ceiling")
    ceiling = esb.stream_ceiling(N * N, 10)
    roof["measured_stream_ceiling_GBs"] = round(ceiling, 1)
    roof["frac_of_measured_ceiling"] = round(roof["achieved"] / ceiling, 4)
    # the same probe for the variants' own stream patterns (4-byte planes in
    # one or two sets; 2^24 cells each): their HBM rate as a fraction of it
    patterns = {"d2q37_4096_f32_pr0.5": None, "d2q37_4096_f32_pr2": None,
                "d2q37_4096_f16_dev": (37, 1), "d2q37_4096_bf16_dev": (37, 1), "d3q39_256cube_f32": (78, 2),
                "d3q39_256cube_bf16": (39, 1), "d2q33_4096_f32": (66, 2)}
    probed = {(74, 2): ceiling}
    aa = var.get("d2q37_4096_f32_aa_in_place")
    if aa is not None:
        for kern in ("even_kernel", "odd_kernel"):
            aa[kern]["frac_of_measured_ceiling"] = round(aa[kern]["frac_of_hbm_peak"] * HBM_PEAK_GBS / ceiling, 4)
    for name, pat in patterns.items():
        v = var.get(name)
        if v is None or "roofline_frac" not in v:
            continue
        pat = pat or (74, 2)
        if pat not in probed:
            log(f"stream ceiling, {pat[0]} planes in {pat[1]} set(s)")
            probed[pat] = esb.stream_ceiling(N * N, 10, planes=pat[0], sets=pat[1])
        v["measured_stream_ceiling_GBs"] = round(probed[pat], 1)
        v["frac_of_measured_ceiling"] = round(v["roofline_frac"] * HBM_PEAK_GBS / probed[pat], 4)

    if not args.no_cpu:
        log("cpu baseline (FP64 oracle on the host)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def time_batch(esb, torch, workloads, batch_steps, tune_cache, streaming="pull", grouped=False):
    """256 independent domains (two-copy pull or A-A in place) in the three
    execution modes with the autotuned launch shape, and optionally the
    persistent launch advancing MALL-sized domain groups."""
    doms = workloads.batch_domains(256)
    bt = esb.Batch(2, 37, [dict(dims=(d["nx"], d["ny"]), Nf=d["Nf"], Pr=d["Pr"], tau=d["tau"]) for d in doms],
                   streaming=streaming)
    for k, d in enumerate(doms):
        bt.init_fields(k, *workloads.batch_fields(d))
    cells, bps = bt.info()
    block, policy = bt.autotune(cache_path=tune_cache)
    log(f"batch ({streaming}) autotune: block {block}, policy {policy}")
    res = {"streaming": streaming, "tile": {"block": block, "policy": policy}}

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
        log(f"batch ({streaming}) {len(doms)} domains, {cells} cells: mode {name}, {batch_steps} steps")
        run(name, mode, batch_steps)
    # the per-domain loop at its own best work-group size (the tuned shape of
    # the persistent launch need not suit one launch per domain)
    best = None
    for blk, pol in sorted({(256, 0), (512, 0), (block, policy)}):
        bt.set_tile(blk, pol)
        log(f"batch ({streaming}) {len(doms)} domains: mode per_domain_loop, block {blk} policy {pol}, "
            f"{batch_steps} steps")
        run("per_domain_loop", 2, batch_steps)
        r = res.pop("per_domain_loop")
        if best is None or r["mlups"] > best["mlups"]:
            best = dict(r, tile={"block": blk, "policy": pol})
    res["per_domain_loop"] = best
    if grouped:
        # the same persistent launch, advancing groups of domains (about 128
        # MB of storage each) eight steps at a time while they sit in the MALL
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
