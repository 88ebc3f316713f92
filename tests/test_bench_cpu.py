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


def test_method_counts_of_one_reaction():
    # A + A <=> B (2 species, 1 reaction), by the formulas of the method:
    # transcendentals 2 NR + NS + 3 = 7; FP64 7 NS + 3 NR = 17; FP32-class
    # Arrhenius 3 + nu'.lnC 1 nonzero + rate 1 + production 2 nonzeros = 7;
    # slots 4 * 7 + 7 + 17 = 52
    nu_f = np.array([[2, 0]], np.int8)
    nu_r = np.array([[0, 1]], np.int8)
    assert roofline.method_counts(nu_f, nu_r) == (7, 7, 17)
    assert roofline.method_slots(nu_f, nu_r) == 52.0


def test_roofline_of_the_benchmark_mechanism():
    # 53 species / 325 reactions x 2^20 cells: 706 transcendentals, 2,868
    # FP32-class and 1,346 FP64 operations per cell -> 4 * 706 + 2868 + 1346
    # = 7,038 slots, 187.7 us at 39.32 T slots/s; with the microbenchmarked
    # rates 706/21 + 2868/82 + 1346/46 = 97.9 CU-clocks per cell, 167.0 us
    src = synth.make_mechanism(53, 325)
    assert roofline.method_slots(src.nu_f, src.nu_r) == 7038.0
    n = 1 << 20
    assert abs(roofline.t_valu(src.nu_f, src.nu_r, n) - 7038 * n / 39.3216e12) < 1e-12
    clocks = 706 / 21 + 2868 / 82 + 1346 / 46
    assert abs(roofline.t_valu(src.nu_f, src.nu_r, n, "measured") - clocks * n / (256 * 2.4e9)) \
        < 1e-12
    r = roofline.roofline(src.nu_f, src.nu_r, n, 4, 0.7e-3)
    assert abs(r["frac"] - 187.68e-6 / 0.7e-3) < 1e-3
    assert r["t_hbm_s"] < r["t_valu_slots_s"]


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
