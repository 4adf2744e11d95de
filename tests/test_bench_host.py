"""Host logic of bench.py (CPU only): the one-GPU guard, the algorithmic byte counts the
roofline divides by, and the reduction of rocprofv3 counter CSVs to HBM bytes per launch."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_step_kernels():
    """N = M = L = 2^22, K = 10, complex64: the first pass reads c once and writes the K-wide
    intermediate once; the second reads it once with 12 bytes of plan data per sample and
    writes f; the derivative pass also writes an FP64 gradient; the sort moves g once."""
    n, K, cs = 1 << 22, 10, 8
    inter = K * n * cs
    kb = lambda name, **kw: bench.kernel_bytes(name, K, n, n, n, cs, **kw)
    assert kb("fwd_passA") == n * cs + inter == 369098752
    assert kb("fwd_passB") == inter + 12 * n + cs * n
    assert kb("gradx_passB") == kb("fwd_passB") + 8 * n
    assert kb("bwd_sort") == (2 * cs + 4) * n
    assert kb("adj_passB") == cs * n + 8 * n + (n + 1) * 4 + inter
    assert kb("adj_passA") == kb("fwd_passA")
    assert kb("fwd_passA", ys=4) == n * cs + K * n * 4          # the half-precision exchange
    assert kb("no_such_kernel") is None


def _write_counters(d, counter, values, calib):
    """One fake rocprofv3 counter CSV: the step kernels in launch order, three steps,
    then the calibration copy."""
    os.makedirs(d, exist_ok=True)
    rows, i = [], 0
    for _ in range(3):
        for k in bench.COUNTER_ORDER:
            rows.append({"Dispatch_Id": i, "Kernel_Name": "void nufft::k_pass_%s<float>(...)" % k,
                         "Counter_Name": counter, "Counter_Value": values[k]})
            i += 1
    rows.append({"Dispatch_Id": i, "Kernel_Name": "at::native::MulFunctor<float>", "Counter_Name": counter,
                 "Counter_Value": calib})
    with open(os.path.join(d, "1_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        w.writerows(rows)


def test_counter_reduction(tmp_path):
    fetch = {k: 1000.0 * (i + 1) for i, k in enumerate(bench.COUNTER_ORDER)}
    write = {k: 300.0 * (i + 1) for i, k in enumerate(bench.COUNTER_ORDER)}
    copy_kib = bench.CALIB_BYTES / 1024.0
    _write_counters(str(tmp_path / "F"), "FETCH_SIZE", fetch, copy_kib / 2)   # the copy's reads count half
    _write_counters(str(tmp_path / "W"), "WRITE_SIZE", write, copy_kib)
    out = str(tmp_path / "traffic.json")
    bench.traffic_summary(str(tmp_path / "F"), str(tmp_path / "W"), out, ["test"])
    rec = json.load(open(out))
    assert rec["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["calibration"]["write_scale"] == pytest.approx(1.0)
    for k in bench.COUNTER_ORDER:
        assert rec["kernels"][k]["bytes_per_launch"] == int(fetch[k] * 1024 * 2 + write[k] * 1024)
    # the backward sort's two kernels are also reported together
    assert rec["kernels"]["bwd_sort"]["bytes_per_launch"] == (rec["kernels"]["bwd_sort.1"]["bytes_per_launch"]
                                                             + rec["kernels"]["bwd_sort.2"]["bytes_per_launch"])
    assert rec["source_sha256_16"] == bench.kernel_source_hash()


def test_counter_reduction_rejects_a_mismatched_run(tmp_path):
    fetch = {k: 1.0 for k in bench.COUNTER_ORDER}
    _write_counters(str(tmp_path / "F"), "FETCH_SIZE", fetch, 1.0)
    with open(os.path.join(str(tmp_path / "F"), "1_counter_collection.csv"), "a") as fh:
        fh.write('99,"void nufft::k_passA<float>(...)",FETCH_SIZE,1.0\n')       # one kernel too many
    _write_counters(str(tmp_path / "W"), "WRITE_SIZE", fetch, 1.0)
    with pytest.raises(SystemExit):
        bench.traffic_summary(str(tmp_path / "F"), str(tmp_path / "W"), str(tmp_path / "t.json"), ["test"])


def test_oversampling_grid_list():
    """The grids the bench plans explicitly: every supported length N <= L <= 2 L0."""
    assert bench.oversampling_grids(1 << 14) == [16384, 24576, 32768]
    assert bench.oversampling_grids(20000) == [24576, 32768, 40960, 49152, 65536]
    assert bench.oversampling_grids(1 << 22) == [4194304, 5242880, 6291456, 8388608]
    assert bench.oversampling_grids(3000) == [4096, 8192]
