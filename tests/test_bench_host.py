"""Host-side logic of bench.py: the one-GPU guard, the algorithmic counts the
roofline uses, and the HBM-traffic record (it must describe the kernel source
as it stands, since bench.py reports it as the kernel's traffic)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_flops_is_the_sum_of_its_parts():
    # basis 5FN, Gram FN(N+1), right-hand side 2FN, column sums FN,
    # residuals 4FN + F, cost 4F, dense solve N^3/3 + 2N^2
    for F, N in ((1000, 8), (2000, 12), (4096, 20), (50, 5), (1, 1)):
        parts = 5 * F * N + F * N * (N + 1) + 2 * F * N + F * N + 4 * F * N + F + 4 * F + N ** 3 / 3 + 2 * N * N
        assert np.isclose(bench.algorithmic_flops(F, N), parts, rtol=0, atol=1e-9)
    assert round(bench.algorithmic_flops(4096, 20)) == 2727307
    assert round(bench.algorithmic_flops(1000, 8)) == 173299


def test_algorithmic_bytes():
    # the log10 tau row, the cost, and the candidate's share of three spectra
    assert bench.algorithmic_bytes(4096, 20, 128) == 936
    assert bench.algorithmic_bytes(1000, 8, 256) == 8 * 8 + 8 + 24 * 1000 / 256


def test_traffic_record_matches_the_kernel_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "fit_eval_traffic.json")))["records"][0]
    assert rec["source_sha256_16"] == bench.kernel_source_hash(), \
        "the kernel changed since its HBM traffic was measured: re-take the rocprofv3 FETCH/WRITE_SIZE profile"
    assert np.isclose(rec["bytes_per_launch"],
                      1024 * (rec["fetch_kib_per_dispatch"] * rec["copy_scale_fetch"] +
                              rec["write_kib_per_dispatch"] * rec["copy_scale_write"]), rtol=1e-6)

    class WL:
        name = rec["workload"] + " I400 polish50"

    sched = [{"freq_split": rec["freq_split"]}]
    assert bench.measured_traffic(WL, rec["kernel"], sched) == rec["bytes_per_launch"]
    assert bench.measured_traffic(WL, rec["kernel"], [{"freq_split": rec["freq_split"] * 2}]) is None
    assert bench.measured_traffic(WL, "fit_kernel<8,1,false,1>", sched) is None
