"""Write stored reference outputs of the FP64 oracle for the large workloads.

Calls only `oracle/` and the seeded input generators in `workloads.py`;
nothing here touches the GPU library.  Usage (from the repository root):

    python tests/golden/make_references.py waves --n 4096 --Pr 0.71 \
        --steps 1000 --threads 7
    python tests/golden/make_references.py waves --n 1024 --Pr 0.71 \
        --steps 1000 5000 --threads 7 --out-n 256

For each requested step count the file `ref_waves{n}_pr{Pr}.npz` gains, as
float32 deviations block-averaged to an out_n^2 grid: rho - 1, u_x, u_y and
T - 1; plus the FP64 domain totals (mass, momentum, energy) at step 0 and at
each snapshot.  The run is the D2Q37, N_f = 3, tau = 0.6, kappa = 0.2
configuration with superposed shear/thermal waves and seeded noise.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def waves(n: int, Pr: float, steps: list[int], threads: int, out_n: int = 512, tau: float = 0.6):
    oracle.set_threads(threads)
    path = os.path.join(HERE, f"ref_waves{n}_pr{Pr:g}.npz")
    rho, u, T = workloads.waves_noise_2d(n)
    sim = oracle.Sim(2, 37, 3, Pr, tau, (n, n), kappa=0.2)
    sim.init(rho, u, T)
    del rho, u, T
    data = dict(n=n, Pr=Pr, tau=tau, Nf=3, kappa=0.2, out_n=out_n, totals0=sim.totals())
    t0 = time.time()
    done = 0
    for target in sorted(steps):
        while done < target:
            chunk = min(50, target - done)
            sim.step(chunk)
            done += chunk
            el = time.time() - t0
            print(f"[waves n={n} Pr={Pr}] step {done}/{max(steps)}  {el:.0f}s  "
                  f"{n * n * done / el / 1e6:.2f} MLUPS", flush=True)
        m = sim.moments()
        data[f"rho_{target}"] = workloads.block_mean(m["rho"] - 1.0, out_n).astype(np.float32)
        data[f"ux_{target}"] = workloads.block_mean(m["u"][0], out_n).astype(np.float32)
        data[f"uy_{target}"] = workloads.block_mean(m["u"][1], out_n).astype(np.float32)
        data[f"T_{target}"] = workloads.block_mean(m["T"] - 1.0, out_n).astype(np.float32)
        data[f"totals_{target}"] = sim.totals()
        data["steps"] = np.array(sorted(s for s in steps if s <= target))
        np.savez_compressed(path + ".tmp.npz", **data)
        os.replace(path + ".tmp.npz", path)
        print(f"[waves] wrote snapshot {target} to {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    w = sub.add_parser("waves")
    w.add_argument("--n", type=int, default=4096)
    w.add_argument("--Pr", type=float, default=0.71)
    w.add_argument("--tau", type=float, default=0.6)
    w.add_argument("--steps", type=int, nargs="+", default=[1000, 5000])
    w.add_argument("--threads", type=int, default=0)
    w.add_argument("--out-n", type=int, default=512, help="side of the block-averaged output grid")
    a = ap.parse_args()
    if a.cmd == "waves":
        waves(a.n, a.Pr, a.steps, a.threads, out_n=a.out_n, tau=a.tau)


if __name__ == "__main__":
    main()
