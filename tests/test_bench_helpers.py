"""CPU checks of bench.py's bookkeeping: the kernel names it reports, the
traffic entry it accepts only for the kernel source and instantiation the
counters were taken on, the algorithmic byte count, and the refusal of more
than one GPU."""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_kernel_names(bench):
    assert bench.sssp_kernel_name(3, 4) == "k_sssp_wg<2, 4, false>"
    assert bench.sssp_kernel_name(0, 0) == "k_sssp_wg<2, 4, false>"      # default shape of the node queue
    assert bench.sssp_kernel_name(5, 4) == "k_sssp_wg<2, 2, false>"
    assert bench.sssp_kernel_name(3, 1) == "k_sssp_ds<4, 4>"
    assert bench.sssp_kernel_name(6, 1) == "k_sssp_ds<1, 1>"
    # chain-contracted search, then the fill of the nodes it leaves out
    assert bench.sssp_kernel_name(3, 4, 4) == "k_sssp_wg<2, 4, true, 7> + k_chain_fill"
    assert bench.sssp_kernel_name(0, 1, 4) == "k_sssp_wg<2, 4, true, 7> + k_chain_fill"   # one workgroup per tree
    assert bench.sssp_kernel_name(2, 4, 4) == "k_sssp_wg<1, 4, true> + k_chain_fill"
    assert bench.sssp_kernel_name(2, 4, 3) == "k_sssp_wn<2, 4>"


def test_traffic_entry_matches_source_and_kernel(bench, tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    entry = {"kernel": "k_sssp_wg<2, 4, false>", "kernel_sha256": "abc", "bytes_per_launch": 123.0}
    (tmp_path / "profiles" / "sssp_traffic.json").write_text(json.dumps(entry))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_entry("abc", "k_sssp_wg<2, 4, false>") == 123.0
    assert bench.traffic_entry("abd", "k_sssp_wg<2, 4, false>") is None       # kernel source changed
    assert bench.traffic_entry("abc", "k_sssp_wg<4, 4, false>") is None       # another instantiation


def test_committed_traffic_entry_is_used_only_for_its_kernel(bench):
    """The committed counter entry feeds the JSON line only while the kernel
    source it was measured on is the current one; otherwise traffic is null."""
    src = open(os.path.join(ROOT, "paper_2104_12911_amd", "csrc", "qdta_kernels.hip"), "rb").read()
    t = json.load(open(os.path.join(ROOT, "profiles", "sssp_traffic.json")))
    cur = hashlib.sha256(src).hexdigest()
    got = bench.traffic_entry(cur, t["kernel"])
    if t["kernel_sha256"] == cur:
        assert got == t["bytes_per_launch"]
    else:
        assert got is None


def test_algorithmic_bytes(bench):
    assert bench.sssp_bytes_per_tree(550_000, 1_000_000) == 12.4e6


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_reduce_traffic_scales_by_the_calibration_kernel(tmp_path):
    """Per-launch HBM bytes: the kernel's mean FETCH_SIZE / WRITE_SIZE (KiB
    per dispatch) times the factor that makes the calibration add kernel read
    and write its known size."""
    import sqlite3
    import bench

    def db(path, counter, rows):
        con = sqlite3.connect(path)
        con.execute("create table pmc_events (dispatch_id int, name text, counter_name text, counter_value real)")
        con.executemany("insert into pmc_events values (?, ?, ?, ?)", [(d, n, counter, v) for d, n, v in rows])
        con.commit()
        con.close()

    k = "void qdta::k_sssp_wg<2, 4, true>(qdta::NetDev)"
    add = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<float>>()"
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    # FETCH_SIZE of the 1 MiB calibration reads half the true size; two launches of the kernel
    db(fdb, "FETCH_SIZE", [(1, add, 512.0), (2, k, 1000.0), (3, k, 3000.0), (4, "other", 9.0)])
    db(wdb, "WRITE_SIZE", [(1, add, 1024.0), (2, k, 10.0), (3, k, 30.0)])
    out = bench.reduce_traffic(fdb, wdb, "k_sssp_wg<2, 4, true>", 1, str(tmp_path / "t.json"), ["a", "b"])
    assert out["fetch_kib_per_launch"] == 2000.0 and out["write_kib_per_launch"] == 20.0
    assert out["calibration"]["fetch_scale"] == 2.0 and out["calibration"]["write_scale"] == 1.0
    assert out["bytes_per_launch"] == 1024.0 * (2000.0 * 2.0 + 20.0)
    assert out["fetch_launches"] == 2


def test_reduce_traffic_adds_the_parts_of_a_two_kernel_launch(tmp_path):
    """A launch named "A + B" (the contracted search and its chain fill) is
    one dispatch of each: their per-launch means add up."""
    import sqlite3
    import bench

    def db(path, counter, rows):
        con = sqlite3.connect(path)
        con.execute("create table pmc_events (dispatch_id int, name text, counter_name text, counter_value real)")
        con.executemany("insert into pmc_events values (?, ?, ?, ?)", [(d, n, counter, v) for d, n, v in rows])
        con.commit()
        con.close()

    a = "void qdta::k_sssp_wg<2, 4, true, 7>(qdta::NetDev)"
    b = "qdta::k_chain_fill(qdta::NetDev, qdta::DemDev)"
    add = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<float>>()"
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    db(fdb, "FETCH_SIZE", [(1, add, 1024.0), (2, a, 100.0), (3, b, 7.0), (4, a, 300.0), (5, b, 9.0)])
    db(wdb, "WRITE_SIZE", [(1, add, 1024.0), (2, a, 10.0), (3, b, 1.0), (4, a, 30.0), (5, b, 3.0)])
    out = bench.reduce_traffic(fdb, wdb, "k_sssp_wg<2, 4, true, 7> + k_chain_fill", 1, str(tmp_path / "t.json"),
                               [], last=2)
    assert out["fetch_kib_per_launch"] == 200.0 + 8.0 and out["write_kib_per_launch"] == 20.0 + 2.0
    assert out["fetch_launches"] == [2, 2]
    assert out["bytes_per_launch"] == 1024.0 * (208.0 + 22.0)


def test_trace_summary_adds_the_parts_of_a_two_kernel_launch(tmp_path):
    import sqlite3
    import bench
    path = str(tmp_path / "k.db")
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, dispatch_id int, duration int)")
    con.executemany("insert into kernels values (?, ?, ?)", [
        ("void qdta::k_sssp_wg<2, 4, true, 7>(qdta::NetDev)", 1, 80_000_000),
        ("qdta::k_chain_fill(qdta::NetDev)", 2, 4_000_000),
        ("void qdta::k_sssp_wg<2, 4, true, 7>(qdta::NetDev)", 3, 90_000_000),
        ("qdta::k_chain_fill(qdta::NetDev)", 4, 6_000_000)])
    con.commit()
    con.close()
    text = bench.trace_summary(path, "k_sssp_wg<2, 4, true, 7> + k_chain_fill", 2)
    assert "mean 85.00 ms" in text and "mean 5.00 ms" in text
    assert "mean 90.00 ms per launch of both" in text
