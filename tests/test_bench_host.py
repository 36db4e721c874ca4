"""Host-side behaviour of bench.py (no GPU): the one-GPU guard, the traffic
figure taken from the committed counter summary only while the kernel source
is unchanged, and the host description that goes with the oracle baseline."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout + r.stderr
    assert not any(line.startswith("{") for line in r.stdout.splitlines())  # no bench line


def test_traffic_comes_from_the_summary_of_the_same_kernel_source(monkeypatch):
    p = os.path.join(ROOT, "profiles", "force_kernel_traffic_drum1m.json")
    d = json.load(open(p))
    P = d["pairs_per_particle"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: d["kernel_source_hash"])
    assert bench.load_traffic("fp64", P) == float(d["per_launch_bytes"]["fp64"])
    # read + written bytes make up the total
    tot = d["per_launch_read_bytes"]["fp64"] + d["per_launch_write_bytes"]["fp64"]
    assert abs(tot - d["per_launch_bytes"]["fp64"]) <= 1e-6 * tot
    # a bed with other candidate pairs per particle is not the profiled one
    assert bench.load_traffic("fp64", 0.8 * P) is None
    assert bench.load_traffic("fp64", 1.2 * P) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("fp64", P) is None


def test_algorithmic_bytes_per_unit():
    # particle: 72 B state read + 72 B written + 8 B radius/material;
    # unordered candidate pair: 8 B identity + 24 B history read + 24 B written
    assert bench.BYTES_PER_PARTICLE == 72 + 72 + 8
    assert bench.BYTES_PER_PAIR == 8 + 24 + 24


def test_host_cpu_description():
    h = bench.host_cpu()
    assert isinstance(h["model"], str) and h["model"]
    assert h["cpus_usable"] >= 1 and h["cpus_online"] >= h["cpus_usable"]
