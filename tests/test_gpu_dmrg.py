"""GPU two-site sweeps against the oracle's reference sweeps.

The GPU path gets the seeded random MPS (synth) and does everything else on
the device: right-canonicalisation, environments, theta formation, Lanczos,
truncated SVD and environment updates.  The oracle's per-bond energies for
the same inputs are stored in tests/golden/sweep_*.json (written by
tests/golden/make_golden.py, oracle only).  Bars: FP64 |dE/E| <= 1e-10 per
bond; FP32-MFMA and BF16x3 matvecs |dE/E| <= 1e-9 at the end of the last
sweep (the refinement matvec and everything outside Lanczos are FP64).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import model

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# Truncation errors at which the kept states of two runs can differ: the
# states of two correct runs after a few sweeps agree only to ~1e-7 (their
# energies to ~1e-14: E is quadratic in the state's error), so where a bond's
# cut falls among Schmidt values near the 1e-12 relative cut (a dense tail)
# which of them survive is decided by that difference.  Reduced-precision
# matvecs add a floor of spurious Schmidt weight of their own (rounding noise
# in the Lanczos vectors, spread over the thousands of discarded directions):
# after four chi = 1024 sweeps the FP32 path discards 1.5e-8 at the middle
# bond where the FP64 oracle discards 1.45e-9, with energies 3e-13 apart.
EPS_NOISE = {"fp64": 1e-10, "fp32": 1e-8, "bf16x3": 1e-7}


def check_kept(got_chi, got_eps, ref_chi, ref_eps, chi_max, precision):
    """Kept dims equal wherever the oracle fills chi_max with a truncation error
    above the noise level.  Truncation errors are compared for magnitude only
    (within a factor 10 above ten times the noise level, within ten times the
    level below it): the first sweep from a random state is far from
    converged, GPU and oracle leave it ~1e-3 apart in the state (2e-6 in the
    energy at chi = 1024, both FP64), and after the second sweep runs whose
    energies agree to 1e-11 still differ in the discarded tail by up to a
    factor 5 (measured).  Their exact parity is checked on converged
    sweeps (the chi = 256 chain) and on given thetas (the SVD tests)."""
    noise = EPS_NOISE[precision]
    for b, (x, y, ex, ey) in enumerate(zip(got_chi, ref_chi, got_eps, ref_eps)):
        if y == chi_max and ey > noise:
            assert x == y, (b, x, y, ex, ey)
        if max(ex, ey) > 10 * noise:
            assert min(ex, ey) * 10 >= max(ex, ey), (b, x, y, ex, ey)
        else:
            assert abs(ex - ey) <= 10 * noise, (b, x, y, ex, ey)


def golden(case):
    with open(os.path.join(GOLD, f"sweep_{case}.json")) as f:
        return json.load(f)


def gpu_sweeps(tnt, g, precision, sweeps=None):
    from paper_1610_02244_amd import binding as B
    s = synth.CONFIGS[g["config"]]
    W, qw = tnt.bose_hubbard_mpo(g["nmax"], g["J"], g["U"], g["mu"])
    bonds, sites = synth.random_mps(g["L"], g["N"], g["nmax"], g["chi"], g["seed"])
    mps = tnt.mps(bonds, sites, g["nmax"] + 1)
    mps.right_canonicalize()
    env = B.Env(tnt, mps, [W] * g["L"], qw, B.MPO_LEFT, B.MPO_RIGHT)
    out = []
    for _ in range(sweeps or len(g["sweeps"])):
        out.append(tnt.sweep(mps, env, g["chi"], kmax=g["lanczos_steps"], precision=precision,
                             rel_tol=g["rel_cutoff"]))
    return out, mps, (W, qw, s)


@pytest.mark.parametrize("case", ["cfg1", "cfg1_exact"])
def test_sweep_fp64_matches_oracle(tnt, case):
    g = golden(case)
    print(f"[sweep fp64] {case}", flush=True)
    res, mps, _ = gpu_sweeps(tnt, g, "fp64")
    for k, (r, ref) in enumerate(zip(res, g["sweeps"])):
        e = np.array(r["bond_E"])
        er = np.array(ref["E"])
        rel = np.max(np.abs(e - er) / np.abs(er))
        print(f"  sweep {k + 1}: E {e[-1]:.15f} oracle {er[-1]:.15f} max|dE/E| {rel:.2e}")
        assert rel <= 1e-10
        # kept dims at every bond, also at exact chi (cfg1_exact: the relative
        # cut 1e-12 decides, 81 at the middle bond)
        assert list(r["bond_chi"]) == ref["chi"]
        # truncation errors to the FP64 backward error of the SVD
        np.testing.assert_allclose(r["bond_eps"], ref["eps"], rtol=1e-6, atol=1e-13)


def test_sweep_cfg1_exact_reaches_ed(tnt):
    g = golden("cfg1_exact")
    res, mps, _ = gpu_sweeps(tnt, g, "fp64")
    e_ed = model.ed_ground_energy(g["L"], g["N"], g["nmax"], g["J"], g["U"])
    assert res[-1]["energy"] == pytest.approx(e_ed, abs=1e-10)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_sweep_fp32_cfg1(tnt, precision):
    g = golden("cfg1")
    res, mps, _ = gpu_sweeps(tnt, g, precision)
    e = res[-1]["bond_E"][-1]
    er = g["sweeps"][-1]["E"][-1]
    rel = abs(e - er) / abs(er)
    print(f"  [sweep {precision} cfg1] |dE/E| = {rel:.2e}")
    assert rel <= 1e-9


def test_sweep_graph_mode_matches_eager(tnt):
    """Sweeps with the Lanczos recurrence replayed from HIP graphs reproduce
    the eager sweeps bitwise (cfg1, FP32 matvecs)."""
    g = golden("cfg1")
    ref, _, _ = gpu_sweeps(tnt, g, "fp32")
    try:
        tnt.set_graphs(True)
        got, _, _ = gpu_sweeps(tnt, g, "fp32")
    finally:
        tnt.set_graphs(False)
    for a, b in zip(ref, got):
        assert list(a["bond_E"]) == list(b["bond_E"])
        assert list(a["bond_chi"]) == list(b["bond_chi"])


def test_canonical_state_norm_and_density(tnt):
    """After a sweep the returned MPS is normalised and holds N bosons."""
    from oracle import dmrg as odmrg
    g = golden("cfg1")
    res, mps, _ = gpu_sweeps(tnt, g, "fp64", sweeps=1)
    W, qw = model.bh_mpo(g["nmax"], g["J"], g["U"], g["mu"])
    bonds, sites = mps.bonds(), mps.sites()
    d = g["nmax"] + 1
    assert odmrg.norm2(bonds, sites, d) == pytest.approx(1.0, abs=1e-12)
    dens = odmrg.site_densities(bonds, sites, d)
    assert sum(dens) == pytest.approx(g["N"], abs=1e-10)
    assert odmrg.expectation(bonds, sites, [W] * g["L"], qw, d) == pytest.approx(
        res[-1]["energy"], abs=1e-10)


def test_sweep_cfg2_first_bonds(tnt):
    """The first sweep from a random state is far from converged (Lanczos
    residuals O(1), truncation errors 1e-3): rounding differences are
    amplified bond by bond, so only its first bond updates are compared
    tightly; converged energies are compared after four sweeps below."""
    g = golden("cfg2")
    res, mps, _ = gpu_sweeps(tnt, g, "fp64")
    e = np.array(res[0]["bond_E"][:12])
    er = np.array(g["sweeps"][0]["E"][:12])
    rel = np.max(np.abs(e - er) / np.abs(er))
    print(f"  [cfg2 first 12 bonds] max|dE/E| {rel:.2e}")
    assert rel <= 1e-11
    assert list(res[0]["bond_chi"][:12]) == g["sweeps"][0]["chi"][:12]


def test_pool_memory_accounting(tnt):
    """tnt_ctx_memory after a chi = 256 sweep: in-use bytes never exceed what
    the pool holds, the peak covers the sweep's largest operand (the Krylov
    basis of the middle bond, 21 FP64 vectors), and the pool's bound holds."""
    g = golden("cfg2")
    gpu_sweeps(tnt, g, "fp32", sweeps=1)
    m = tnt.memory()
    print(f"  pool {m}")
    s = synth.CONFIGS["cfg2"]
    b = synth.chain_bonds(s.L, s.N, s.nmax, s.chi)
    left, right = b[s.L // 2 - 1], b[s.L // 2 + 1]
    n = sum(left[qa] * right[qa + s1 + s2] for qa in left for s1 in range(s.d)
            for s2 in range(s.d) if qa + s1 + s2 in right)
    assert 0 <= m["pool_in_use"] <= m["pool_held"]
    assert m["pool_peak_in_use"] >= 21 * 16 * n
    assert m["pool_held"] <= 2 * m["pool_peak_in_use"] + (4 << 30) + (64 << 20)
    assert m["blas_workspace"] >= 0


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_sweep_cfg2_converged(tnt, precision):
    g = golden("cfg2_4sweeps")
    print(f"[sweep cfg2 x4 {precision}]", flush=True)
    res, mps, _ = gpu_sweeps(tnt, g, precision)
    e = res[-1]["bond_E"][-1]
    er = g["sweeps"][-1]["E"][-1]
    rel_last = abs(e - er) / abs(er)
    print(f"  E {e:.15f} oracle {er:.15f} |dE/E| {rel_last:.2e} "
          f"sweep {res[-1]['seconds_total']:.2f}s")
    assert rel_last <= 1e-9
    # the last (converged) sweep bond by bond: energies, kept dims, errors
    eb = np.array(res[-1]["bond_E"])
    ebr = np.array(g["sweeps"][-1]["E"])
    rel = np.max(np.abs(eb - ebr) / np.abs(ebr))
    print(f"  last sweep max|dE/E| over bonds {rel:.2e}")
    assert rel <= 1e-9
    got_chi, ref_chi = list(res[-1]["bond_chi"]), g["sweeps"][-1]["chi"]
    diff = [(b, int(x), y, float(e), f) for b, (x, y, e, f) in
            enumerate(zip(got_chi, ref_chi, res[-1]["bond_eps"], g["sweeps"][-1]["eps"]))
            if x != y]
    print(f"  kept-dim differences (bond, gpu, oracle, eps gpu, eps oracle): {diff}")
    if precision == "fp64":
        assert got_chi == ref_chi
        np.testing.assert_allclose(res[-1]["bond_eps"], g["sweeps"][-1]["eps"], rtol=1e-3,
                                   atol=1e-10)
    else:
        # A ground vector from reduced-precision matvecs carries rounding noise
        # (~1e-9 lambda_0 for FP32, ~1e-8 for BF16x3) in directions where the
        # FP64 state has exactly nothing; at bonds the oracle does not fill
        # (its 1e-12 relative cut keeps fewer than chi_max states) that noise
        # is kept as extra states.  Where the oracle fills chi_max the kept
        # dims must agree; elsewhere the GPU keeps at least the oracle's states.
        chi_max = g["chi"]
        for x, y in zip(got_chi, ref_chi):
            assert (x == y) if y == chi_max else (x >= y)


@pytest.mark.parametrize("precision,case", [
    ("fp32", "cfg3"), ("bf16x3", "cfg3"), ("fp64", "cfg3"),
    # the same seeded MPS at the other two couplings: the headline path and FP64
    ("fp32", "cfg3_U2"), ("fp64", "cfg3_U2"), ("fp32", "cfg3_U6"), ("fp64", "cfg3_U6")])
def test_sweep_cfg3_vs_oracle(tnt, precision, case):
    """The chi = 1024 chain (L = 64, N = 64, d = 5; U = 3.3, and the same seeded
    MPS at U = 2 and U = 6): the oracle's stored sweeps (written sweep by
    sweep; the first from a random state is not converged and not compared)
    against the GPU's at the same sweep index: energy to 1e-9 relative; kept
    dims equal wherever the oracle fills chi with a truncation error above the
    noise level, errors within it elsewhere."""
    if not os.path.exists(os.path.join(GOLD, f"sweep_{case}.json")):
        pytest.skip(f"no stored oracle run for {case}")
    g = golden(case)
    k = len(g["sweeps"])
    if not g.get("complete", False):
        # the configuration's bar holds after its four sweeps; earlier sweeps of
        # the deep superfluid (U = 2) still differ by ~1e-9 between two
        # correct runs (GPU FP32 vs oracle after two sweeps: 1.2e-9)
        pytest.skip(f"the oracle's chi = 1024 run for {case} is incomplete ({k} sweeps stored)")
    print(f"[sweep {case} (U = {g['U']}) {precision}] {k} sweeps", flush=True)
    res, mps, _ = gpu_sweeps(tnt, g, precision, sweeps=k)
    # the first bond updates, before the unconverged first sweep amplifies
    # rounding differences (they reach chi = 1024 from the fifth bond on)
    e1 = np.array(res[0]["bond_E"][:12])
    r1 = np.array(g["sweeps"][0]["E"][:12])
    rel1 = float(np.max(np.abs(e1 - r1) / np.abs(r1)))
    print(f"  first 12 bond updates of sweep 1: max|dE/E| {rel1:.2e}", flush=True)
    assert rel1 <= {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-5}[precision]
    e = res[-1]["bond_E"][-1]
    er = g["sweeps"][-1]["E"][-1]
    rel = abs(e - er) / abs(er)
    got, ref = list(res[-1]["bond_chi"]), g["sweeps"][-1]["chi"]
    ndiff = sum(a != b for a, b in zip(got, ref))
    print(f"  E {e:.12f} oracle {er:.12f} |dE/E| {rel:.2e} (sweep {k}); kept dims differ at "
          f"{ndiff} bonds; last sweep {res[-1]['seconds_total']:.1f}s; eigenproblems redone "
          f"{[r['eig_retries'] for r in res]}", flush=True)
    assert rel <= 1e-9
    check_kept(got, res[-1]["bond_eps"], ref, g["sweeps"][-1]["eps"], g["chi"], precision)


def test_sweep_own_eig_reduction(tnt):
    """The converged chi = 256 FP64 sweeps (kept dims and errors equal the
    oracle's at every bond) with the SVD's eigenproblems of padded order >= 48
    reduced to tridiagonal form by the library's own panel kernels (divide and
    conquer and back-transformation from rocSOLVER), against the same stored
    oracle run and bars."""
    tnt.set_eig_reduction(48)
    try:
        test_sweep_cfg2_converged(tnt, "fp64")
    finally:
        tnt.set_eig_reduction(-1)
