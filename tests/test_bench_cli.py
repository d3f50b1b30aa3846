"""Host logic of bench.py, no GPU: the single-GPU contract and the conversion
of rocprofv3 counter files into HBM bytes per launch."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Counter_Name", "Kernel_Name", "Grid_Size", "Counter_Value"])
        w.writeheader()
        for kernel, grid, kib in rows:
            w.writerow(dict(Counter_Name=counter, Kernel_Name=kernel, Grid_Size=grid, Counter_Value=kib))


def test_traffic_from_scales_by_the_copy(tmp_path, monkeypatch):
    # the copy of COPY_BYTES reads back as half its bytes on FETCH_SIZE and all
    # of them on WRITE_SIZE; a kernel's counters scale by the same factors
    copy = "__amd_rocclr_copyBuffer"
    k = "void paco::(anonymous namespace)::local_fft_fast_kernel<12, 2, 1, 2, 16, 0>(paco::LocalPass)"
    half, full = bench.COPY_BYTES / 2 / 1024, bench.COPY_BYTES / 1024
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", [(copy, 1 << 20, half), (copy, 64, 1.0), (k, 524288, 70000.0), (k, 524288, 70002.0)])
    _counter_csv(w, "WRITE_SIZE", [(copy, 1 << 20, full), (k, 524288, 131072.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(out))
    bench.traffic_from(str(f), str(w))
    rec = json.load(open(out))
    assert abs(rec["fetch_scale"] - 2.0) < 1e-9 and abs(rec["write_scale"] - 1.0) < 1e-9
    t = rec["kernels"]["local_fft_fast_kernel<12,2,1,2,16,0>"]
    assert t["fetch_bytes"] == round(70001.0 * 1024 * 2)
    assert t["write_bytes"] == 131072 * 1024
    assert t["hbm_bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"]
    assert rec["kernel_hash"] == bench.kernel_hash()
    # looked up by the same short name, and only while the kernel sources are unchanged
    assert bench.load_traffic("local_fft_fast_kernel<12,2,1,2,16,0>") == t["hbm_bytes_per_launch"]
    rec["kernel_hash"] = "0" * 16
    json.dump(rec, open(out, "w"))
    assert bench.load_traffic("local_fft_fast_kernel<12,2,1,2,16,0>") is None


def test_committed_traffic_covers_the_default_plans_kernels():
    # the roofline's traffic field looks each pass up by its kernel's name:
    # the committed counter summary must hold all three under those names
    with open(bench.TRAFFIC_PATH) as f:
        kernels = json.load(f)["kernels"]
    for name in bench.SYM_KERNELS:
        assert name.split()[1] in kernels, name


def test_short_kernel_names():
    n = "void paco::(anonymous namespace)::middle_packed2_kernel<false, true>(paco::MiddlePass)"
    assert bench.short_kernel_name(n) == "middle_packed2_kernel<false,true>"


def test_cpu_baseline_record():
    # one thread and all cores, the same output bits, the host named
    import numpy as np

    x = (np.random.default_rng(3).standard_normal((1 << 14, 2)) @ [1, 1j]).astype(np.complex64)
    ref, rec = bench.cpu_baseline(x, 1 << 14, budget_s=0.2)
    assert rec["kind"] == "oracle" and rec["unit"] == "GFLOP/s"
    assert rec["cores"] == rec["threads_all"]["threads"] >= 1
    assert rec["threads_1"]["threads"] == 1 and rec["threads_1"]["runs"] >= 3
    assert rec["value"] == rec["threads_all"]["value"] > 0
    assert rec["nproc"] >= 1 and rec["cpu_model"]
    assert ref.dtype == np.complex128 and ref.shape == (1 << 14,)
