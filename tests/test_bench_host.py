"""Host-side pieces of the benchmark (no GPU): the byte model, the counter
records it reads, the roofline arithmetic and the refusal of several GPUs."""
import hashlib
import os
import subprocess
import sys
import types

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_byte_model():
    # binary32 state: 28 B read + 24 B written; tile of (E+2)^3 cells x 3
    # binary32 values; the chunk's 3 E^3 binary64 sources read and written
    b, per_p, per_item = bench.algorithmic_bytes("fp32_local", 1000, 10)
    assert per_p == 52 and per_item == 12000 + 24576 and b == 52000 + 365760
    b, per_p, per_item = bench.algorithmic_bytes("fp64", 1000, 10)
    assert per_p == 104 and per_item == 24000 + 24576
    _, per_p, per_item = bench.algorithmic_bytes("fp32", 1, 1)
    assert per_p == 52 and per_item == 12000 + 12288
    _, _, per_item = bench.algorithmic_bytes("fp32_local", 1, 1, E=4)
    assert per_item == 3 * 6 ** 3 * 4 + 2 * 3 * 64 * 8


def test_counter_records_match_the_kernel_source():
    """Every committed step-kernel counter record carries the hash of the
    kernel source it was taken on; the benchmark reads its traffic only while
    the hash matches, and the record's bytes are its counters scaled by its
    calibration factors."""
    digest = hashlib.sha256(open(bench.KERNEL_SOURCE, "rb").read()).hexdigest()
    for wl in ("plume512", "plume256", "tg128"):
        path = os.path.join(ROOT, "profiles", f"k_step_{wl}_fp32_local_counters.txt")
        rec = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        hbm = (float(rec["fetch_kib_per_dispatch"]) * 1024 * float(rec["fetch_factor"]) +
               float(rec["write_kib_per_dispatch"]) * 1024 * float(rec["write_factor"]))
        # (the factors are printed to four decimals)
        assert abs(hbm - float(rec["hbm_bytes_per_launch"])) <= 1e-4 * hbm
        alg = float(rec["algorithmic_bytes_per_launch"])
        assert 1.0 <= hbm / alg < 1.1, wl            # nothing re-read
        got = bench.measured_traffic(wl, "fp32_local")
        if rec["kernel_source_sha256"] == digest:
            assert got == float(rec["hbm_bytes_per_launch"])
        else:
            assert got is None
    assert bench.measured_traffic("no_such_workload", "fp32_local") is None


def test_roofline_arithmetic():
    w = types.SimpleNamespace(P=1_000_000, name="no_such_workload", chunk_edge=8)
    r = bench.roofline("fp32_local", w, kernel_ms=2.0, launches=2, items=100, ms_per_step=1.25)
    bytes_launch = 52 * 1_000_000 + 100 * 36576
    assert r["bytes_per_launch"] == bytes_launch
    assert abs(r["achieved"] - bytes_launch / 1e-3 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    assert abs(r["whole_step"]["achieved"] - bytes_launch / 1.25e-3 / 1e9) < 1e-6
    assert r["traffic"] is None and r["bound"] == "hbm" and r["unit"] == "GB/s"


def test_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
