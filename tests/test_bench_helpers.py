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
    assert bench.sssp_kernel_name(3, 4, 4) == "k_sssp_wg<2, 4, true>"   # chain-contracted search
    assert bench.sssp_kernel_name(0, 1, 4) == "k_sssp_wg<2, 4, true>"   # one workgroup per tree whatever asked
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
