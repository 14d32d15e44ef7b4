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


@pytest.mark.parametrize("cfg", ["cfg1", "cfg2", "cfg3", "cfg5"])
def test_reference_schedule_flops(cfg):
    """The unpruned count against the oracle's pruned one at the middle bond:
    step 4 is the same (every produced Bose-Hubbard slab reaches an allowed
    output), step 1 and the MPO passes can only count more, and the total
    stays within a few percent."""
    import synth
    from oracle import flops as oflops
    from oracle import model
    b = load_bench()
    s = synth.CONFIGS[cfg]
    bonds = synth.chain_bonds(s.L, s.N, s.nmax, s.chi)
    left, right = bonds[s.L // 2 - 1], bonds[s.L // 2 + 1]
    W, qw = model.bh_mpo(s.nmax, s.J, s.U, s.mu)
    ref = b.reference_schedule_flops(left, right, s.d, W, qw)
    pruned = oflops.heff2_flops(left, right, s.d, qw, W, W)
    assert ref["step4"] == pruned["step4"]
    assert ref["step1"] >= pruned["step1"] and ref["mpo"] >= pruned["mpo"]
    assert pruned["total"] <= ref["total"] <= 1.15 * pruned["total"]
    if cfg == "cfg3":
        # the sector recipe's own estimate of the reference-schedule count
        assert ref["total"] == pytest.approx(3.656e10, rel=5e-3)
