"""CPU checks of bench.py's host logic: the one-GPU guard and the
HBM-traffic arithmetic that turns rocprofv3 counter databases into bytes
per launch."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import numpy as np  # noqa: E402

NCELL = 4096 * 4096


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _fake_db(path, counter, rows):
    """rows: (kernel name, grid, work-group, KiB) per dispatch."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (kernel_name text, counter_name text, value real, "
               "dispatch_id integer, grid_size integer, workgroup_size integer)")
    for k, (name, grid, wg, kib) in enumerate(rows):
        # split each dispatch's value over two records, as per-XCD counters are
        db.execute("insert into counters_collection values (?,?,?,?,?,?)", (name, counter, kib / 2, k, grid, wg))
        db.execute("insert into counters_collection values (?,?,?,?,?,?)", (name, counter, kib / 2, k, grid, wg))
    db.commit()
    db.close()


def test_ingest_scales_by_the_copy_kernel(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    known_kib = 74 * NCELL * 4 / 1024
    alg_half_kib = 2 * 37 * 4 * NCELL / 1024          # read (or written) bytes of one launch
    stream = "void esbgk::(anonymous namespace)::k_stream_rw<74, 2>(char*)"
    pull3 = "void esbgk::k_step<esbgk::LatD2Q37, 0, 2, true, 3, true>(char*)"
    odd0 = "void esbgk::k_step<esbgk::LatD2Q37, 0, 1, true, 0, true>(char*)"
    # the fetch counter reads half of the true bytes, the write counter all
    fetch = [(stream, NCELL, 256, known_kib / 2)] * 3 + [(pull3, NCELL, 512, alg_half_kib / 2 * 1.1)] * 5 + \
            [(odd0, NCELL // 4, 256, alg_half_kib / 2)] * 3
    write = [(stream, NCELL, 256, known_kib)] * 3 + [(pull3, NCELL, 512, alg_half_kib)] * 5 + \
            [(odd0, NCELL // 4, 256, alg_half_kib * 1.2)] * 3
    _fake_db(str(tmp_path / "f" / "a_results.db"), "FETCH_SIZE", fetch)
    _fake_db(str(tmp_path / "w" / "a_results.db"), "WRITE_SIZE", write)
    bench.ingest_counters(str(tmp_path / "f"), str(tmp_path / "w"))
    with open(bench.traffic_path("D2Q37")) as fh:
        d = json.load(fh)
    assert d["stream_kernel_fetch_factor"] == pytest.approx(0.5)
    assert d["stream_kernel_write_factor"] == pytest.approx(1.0)
    k = d["kernels"]
    assert set(k) == {"pull cp3 wg512 cpi1", "aa_odd cp0 wg256 cpi4"}
    assert k["pull cp3 wg512 cpi1"]["traffic_over_algorithmic"] == pytest.approx(1.05)
    assert k["aa_odd cp0 wg256 cpi4"]["traffic_over_algorithmic"] == pytest.approx(1.1)
    # the bench line looks entries up by the autotuner's (block, order, policy, cells per item)
    bpl = 592 * NCELL
    assert bench.measured_traffic("pull", (512, 1, 3, 1)) == pytest.approx(1.05 * bpl)
    assert bench.measured_traffic("aa_odd", (256, 2, 1, 4)) == pytest.approx(1.1 * bpl)
    assert bench.measured_traffic("pull", (256, 1, 3, 1)) is None
    assert bench.pull_traffic([(512, 1, 3, 1), (512, 2, 3, 1)]) == pytest.approx(1.05 * bpl)
    assert bench.pull_traffic([(512, 1, 3, 1), (128, 1, 3, 1)]) is None
    # a summary from other kernel source is ignored
    d["kernel_source_hash"] = "0" * 16
    with open(bench.traffic_path("D2Q37"), "w") as fh:
        json.dump(d, fh)
    assert bench.measured_traffic("pull", (512, 1, 3, 1)) is None


class _FakeLattice:
    """Stands in for a 4096^2 lattice: its moments after `steps` are the
    stored FP64 reference's block means repeated over 8 x 8 cells, plus a
    chosen relative perturbation of u; its totals drift by a chosen amount."""

    def __init__(self, ref, du=0.0, drift=0.0):
        self.ref, self.du, self.drift = ref, du, drift

    def init_fields(self, *fields):
        self.t = np.array([4096.0 ** 2, 0.0, 0.0, 3.0 * 4096 ** 2])

    def totals(self):
        return self.t.copy()

    def step(self, n):
        self.t = self.t * (1.0 + self.drift)

    def read_moments(self):
        up = lambda a: np.repeat(np.repeat(a.astype(np.float64), 8, axis=0), 8, axis=1)
        r = self.ref
        return {"rho": 1.0 + up(r["rho_1000"]), "T": 1.0 + up(r["T_1000"]),
                "u": (1.0 + self.du) * np.stack([up(r["ux_1000"]), up(r["uy_1000"])])}


@pytest.mark.skipif(not os.path.exists(bench.GOLDEN_4096), reason="reference not generated")
def test_error_vs_fp64_arithmetic():
    """The bench's error report against the stored FP64 oracle run: zero for
    the reference itself, the chosen relative error of u and the chosen
    drift otherwise (block means of repeated values are exact)."""
    ref = np.load(bench.GOLDEN_4096)
    e = bench.error_vs_fp64(_FakeLattice(ref), ())
    assert e["rho"] == 0 and e["u"] == 0 and e["T"] == 0 and e["mass_drift"] == 0
    e = bench.error_vs_fp64(_FakeLattice(ref, du=1e-3, drift=2e-9), ())
    assert e["u"] == pytest.approx(1e-3, rel=1e-6)
    assert e["rho"] < 1e-15 and e["T"] < 1e-15
    assert e["mass_drift"] == pytest.approx(2e-9, rel=1e-3) and e["energy_drift"] == pytest.approx(2e-9, rel=1e-3)
