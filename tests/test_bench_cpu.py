"""Host logic of bench.py and the roofline accounting it reports (no GPU)."""

import json
import os
import subprocess
import sys

import numpy as np

from paper_2008_08483_amd import roofline, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_method_slots_of_one_reaction():
    # A + A <=> B: per species ln C (4), C from Y (3), Gibbs layer (7), mu (1);
    # per cell ln T and 1/T (8), T^2..T^4 and ln C0 (4); the reaction: Arrhenius
    # (2), ln k_r (1), q_f - q_r (1), nu'.lnC (1 nonzero), nu.Gt (2), nu''.lnC
    # (1), two exponentials (8), production (2)
    nu_f = np.array([[2, 0]], np.int8)
    nu_r = np.array([[0, 1]], np.int8)
    assert roofline.method_slots(nu_f, nu_r) == 2 * 15 + 12 + 18


def test_method_slots_of_the_benchmark_mechanism():
    src = synth.make_mechanism(53, 325)
    assert roofline.method_slots(src.nu_f, src.nu_r) == 8292.0


def test_compulsory_bytes_match_the_traffic_record():
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    n = 1 << 20
    alg = t["algorithmic_bytes_per_launch"]
    assert roofline.hbm_bytes(53, 4) == 432
    assert alg["read"] == 4 * (53 + 2) * n and alg["write"] == 4 * 53 * n
    assert alg["total"] == roofline.hbm_bytes(53, 4) * n


def test_traffic_is_reported_only_for_the_same_kernel_source(monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: t["kernel_source_hash"])
    assert bench.measured_traffic() == t["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None
