"""The benchmark's command-line contract: one JSON line with the metric, the roofline and the
launch; a request for more than one GPU is refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and r.stdout == ""


@pytest.mark.gpu
def test_bench_line():
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--only", "--steps", "3",
                        "--warmup", "1"], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["dtype"] == "f64"
    assert d["value"] > 0 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert "workload" in d["config"] and d["config"]["crossings_per_step"] > 0
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-4
    assert 0.0 < rf["kernel_ms"] <= rf["call_ms"] <= d["ms_per_step"] * 1.05
    assert d["rounding"]["recheck_tracks"] >= 0 and d["rounding"]["cr_ambiguous"] == 0


def test_oracle_full_command():
    """bench.py --oracle-full: the oracle over every particle of a workload, one JSON line."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-full", "--workload", "C1"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["kind"] == "oracle" and d["particles"] == 1000 and d["crossings"] == 40000   # 40 cells per row
    assert d["threads"] == 1 and d["value"] > 0


def test_path_accuracy_report():
    """The mixed-precision accuracy figures of the benchmark line: path agreement counts the
    particles whose path hash and crossing count both match; travel times are compared for the
    particles both runs brought to a boundary face or a sink cell, relative to the FP64 travel
    time."""
    sys.path.insert(0, ROOT)
    import numpy as np
    from paper_2302_13590_amd import accuracy as ACC
    n = 8
    ref = {"status": np.array([1, 1, 1, 1, 2, 1, 1, 3], np.int32), "t": np.arange(1.0, 9.0) + 10.0,
           "ncross": np.full(n, 4, np.int32), "path_hash": np.arange(n, dtype=np.uint64)}
    mix = {k: v.copy() for k, v in ref.items()}
    mix["path_hash"][1] += np.uint64(1)          # different path
    mix["ncross"][2] += 1                         # same hash, different count
    mix["status"][5] = 3                          # did not terminate
    mix["t"][0] += 1e-3                           # travel time 1 -> 1.001
    mix["t"][4] += 5e-3                           # sink particle: travel time 5 -> 5.005
    acc = ACC.path_agreement(mix, ref, t0=np.full(n, 10.0))
    assert acc["particles"] == n and abs(acc["path_agreement"] - 6 / 8) < 1e-12
    assert abs(acc["status_agreement"] - 7 / 8) < 1e-12
    tr = acc["travel_time_rel_err"]
    assert tr["particles"] == 6                   # boundary or sink in both: 0, 1, 2, 3, 4, 6
    assert abs(tr["max"] - 1e-3) < 1e-9 and tr["p50"] == 0.0


def test_trajectory_error_report():
    """Snapshot position error over the entries both runs define, and NaN-pattern agreement."""
    import numpy as np
    from paper_2302_13590_amd import accuracy as ACC
    ref = np.zeros((3, 4, 3))
    ref[2, 3] = np.nan                            # particle 2 left before the last snapshot
    mix = ref.copy()
    mix[0, 1, 0] = 3.0                            # |d| = 5 at one entry
    mix[0, 1, 1] = 4.0
    mix[1, 2] = np.nan                            # mixed run left earlier
    tr = ACC.trajectory_error(mix, ref)
    assert tr["position_err_m"]["entries"] == 10 and tr["position_err_m"]["max"] == 5.0
    assert tr["position_err_m"]["p50"] == 0.0
    assert abs(tr["nan_pattern_agreement"] - 11 / 12) < 1e-6      # reported to 6 digits
