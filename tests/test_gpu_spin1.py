"""GPU two-site sweeps on the spin-1 Heisenberg chain (the DMRG timing workload
of Sec. 3, Table tab:dmrgtimes) against exact diagonalisation.

The product MPO (tnt_mpo_spin1_heisenberg) drives the same sweep as the
Bose-Hubbard runs; the U(1) charge is s = S^z + 1, so the S^z = 0 sector of L
sites is total charge L with d = 3.  At chi = 3^(L/2) the two-site sweep is
exact, so its energy must reach the oracle's ED ground energy (which is pinned
to a Kronecker-product Hamiltonian).  Bars: FP64 |dE| <= 1e-9; FP32-MFMA and
BF16x3 matvecs |dE/E| <= 1e-9 (FP64 refinement, FP64 SVD and environments).
At the timing-table size (L = 101, chi = 200) the checks are properties: the
energy per bond lies at the Haldane-chain value within the open-boundary
correction, does not rise from sweep to sweep, and the middle bond keeps
exactly chi = 200 states.
"""
import numpy as np
import pytest

import synth
from oracle import spin1 as ospin1

pytestmark = pytest.mark.gpu


def run(tnt, L, chi, sweeps, precision, seed, kmax=24, rel_tol=1e-12):
    from paper_1610_02244_amd import binding as B
    W, qw = tnt.spin1_heisenberg_mpo(1.0)
    bonds, sites = synth.random_mps(L, L, 2, chi, seed)
    mps = tnt.mps(bonds, sites, 3)
    mps.right_canonicalize()
    env = B.Env(tnt, mps, [W] * L, qw, B.SPIN1_LEFT, B.SPIN1_RIGHT)
    return [tnt.sweep(mps, env, chi, kmax=kmax, precision=precision, rel_tol=rel_tol)
            for _ in range(sweeps)]


@pytest.mark.parametrize("L", [6, 8])
def test_spin1_exact_sweep_reaches_ed(tnt, L):
    print(f"[spin1 fp64] L={L}", flush=True)
    res = run(tnt, L, 3 ** (L // 2), 3, "fp64", seed=11 + L)
    e_ed = ospin1.ed_ground_energy(L)
    print(f"  E {res[-1]['energy']:.15f} ED {e_ed:.15f}")
    assert res[-1]["energy"] == pytest.approx(e_ed, abs=1e-9)
    # every bond of the last sweep sees the converged energy
    assert max(abs(e - e_ed) for e in res[-1]["bond_E"]) <= 1e-8


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_spin1_exact_sweep_reduced_precision(tnt, precision):
    print(f"[spin1 {precision}] L=8", flush=True)
    res = run(tnt, 8, 81, 3, precision, seed=19)
    e_ed = ospin1.ed_ground_energy(8)
    rel = abs(res[-1]["energy"] - e_ed) / abs(e_ed)
    print(f"  |dE/E| = {rel:.2e}")
    assert rel <= 1e-9


def test_spin1_timing_size_properties(tnt):
    # L = 101, chi = 200: the workload of the paper's timing table
    L, chi = 101, 200
    print(f"[spin1 fp32] L={L} chi={chi}", flush=True)
    res = run(tnt, L, chi, 2, "fp32", seed=3, kmax=12)
    e1, e2 = res[0]["energy"], res[1]["energy"]
    print(f"  E1 {e1:.12f} E2 {e2:.12f} E/(L-1) {e2 / (L - 1):.8f}")
    assert e2 <= e1 + 1e-9
    # bulk energy per bond of the spin-1 Heisenberg chain is -1.401484...;
    # the two open ends change the total by O(1)
    assert -1.4015 * (L - 1) - 2.0 < e2 < -1.4015 * (L - 1) + 2.0
    assert max(res[1]["bond_chi"]) <= chi
    # the middle bonds fill chi (the Schmidt values there reach far below the
    # relative cut 1e-12); right pass, bond L/2
    mid = res[1]["bond_chi"][L // 2 - 1]
    print(f"  kept chi at the middle bond {mid}, max {max(res[1]['bond_chi'])}")
    assert mid == chi
