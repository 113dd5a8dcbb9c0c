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
