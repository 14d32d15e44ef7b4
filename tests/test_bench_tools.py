"""Host-side checks of bench.py's profiler post-processing (no GPU)."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_mfma_util_arithmetic(tmp_path):
    b = load_bench()
    k = "void tnt::packed_gemm_kernel<0, float, 64, 64>(tnt::GemmTask const*)"
    rows = []
    # two dispatches: 8 XCDs x 1000 cycles each, MFMA busy 1024 SIMDs x 500 and x 250
    for d, busy in (("1", 1024 * 500.0), ("2", 1024 * 250.0)):
        rows += [{"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": "GRBM_GUI_ACTIVE",
                  "Counter_Value": 8000.0},
                 {"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": "SQ_VALU_MFMA_BUSY_CYCLES",
                  "Counter_Value": busy},
                 {"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": "SQ_INSTS_MFMA",
                  "Counter_Value": 10.0}]
    # a kernel without MFMA work is left out
    rows += [{"Dispatch_Id": "3", "Kernel_Name": "void copy()", "Counter_Name": "GRBM_GUI_ACTIVE",
              "Counter_Value": 80.0},
             {"Dispatch_Id": "3", "Kernel_Name": "void copy()",
              "Counter_Name": "SQ_VALU_MFMA_BUSY_CYCLES", "Counter_Value": 0.0}]
    write_counters(str(tmp_path / "pmc"), rows)
    out = b.mfma_util(str(tmp_path / "pmc"))
    assert list(out) == ["tnt::packed_gemm_kernel<0, float, 64, 64>"]
    r = out["tnt::packed_gemm_kernel<0, float, 64, 64>"]
    assert r["dispatches"] == 2
    assert r["avg_gpu_cycles"] == pytest.approx(1000.0)
    assert r["mfma_busy_frac"] == pytest.approx(0.375)
    assert r["avg_mfma_insts"] == pytest.approx(10.0)
