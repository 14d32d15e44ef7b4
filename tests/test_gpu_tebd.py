"""GPU TEBD step (tnt_tebd_step) against the TEBD oracle and free fermions.

* Same product state, same bond Hamiltonians, same truncation: the GPU steps
  keep the oracle's dimension at every gate and report its truncation error
  (to 1e-9 relative, or 1e-13 absolute), and the evolved states agree (every
  entry of rho_ij of the GPU state, computed by the oracle's network
  contraction, against the oracle state's).  FP64 throughout.  Cases: chi
  only (rel_tol = -1), chi = 6 (discarded values of 1e-8), and the binding's
  default relative cut 1e-12 (the states' tails then decide the kept dims).
* The paper's second example (Sec. 5): hard-core bosons on L = 51 sites from
  a charge-density wave of 25 bosons, dt = 0.01, chi = 200: the densities
  follow free fermions (Jordan-Wigner) to the Trotter error.
* A bond Hamiltonian that mixes charges is refused.
"""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import observables as oobs
from oracle import tebd as otebd

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("chi,steps,bar,rel_tol", [(64, 3, 1e-9, -1.0), (6, 3, 1e-6, -1.0),
                                                   (64, 3, 1e-9, 1e-12)])
def test_tebd_matches_oracle(tnt, chi, steps, bar, rel_tol):
    L, nmax, J, U, mu, dt = 8, 2, 1.0, 2.0, 0.1, 0.05
    config = (2, 0, 1, 0, 2, 0, 1, 0)
    print(f"[tebd] L={L} chi={chi} steps={steps} rel_tol={rel_tol}", flush=True)
    h = tnt.bond_hamiltonians_bose_hubbard(L, nmax, J, U, mu)
    bonds, sites = synth.product_mps(config)
    mps = tnt.mps(bonds, sites, nmax + 1)
    ob, os_ = bonds, sites
    hs = otebd.bond_hamiltonians_bh(L, nmax, J, U, mu)
    for k in range(steps):
        r = tnt.tebd_step(mps, h, dt, chi, rel_tol=rel_tol)
        ob, os_, rec = otebd.tebd_step(ob, os_, hs, dt, nmax + 1, chi,
                                       trunc=dict(r=rel_tol) if rel_tol > 0 else None)
        assert r["bond_chi"] == [x["chi"] for x in rec], k
        for got_e, x in zip(r["bond_eps"], rec):
            assert got_e == pytest.approx(x["eps"], rel=1e-9, abs=1e-13)
    b = oobs.annihilator(nmax)
    got = oobs.correlation_matrix(mps.bonds(), mps.sites(), nmax + 1, b)
    ref = oobs.correlation_matrix(ob, os_, nmax + 1, b)
    err = np.max(np.abs(got - ref))
    print(f"  max|d rho| = {err:.2e}, max chi {r['max_chi']}")
    assert err <= bar
    # the device correlation pass on the evolved state agrees as well
    dev = mps.correlation(b, -1)
    assert np.max(np.abs(dev - got)) <= 1e-12


def test_hardcore_cdw_melting_free_fermions(tnt):
    L, dt, steps, chi = 51, 0.01, 60, 200
    config = tuple(j % 2 for j in range(L))  # empty, filled, ..., empty: 25 bosons
    assert sum(config) == 25
    print(f"[tebd] hard-core CDW L={L} dt={dt} steps={steps}", flush=True)
    h = tnt.bond_hamiltonians_bose_hubbard(L, 1, 1.0, 0.0)
    bonds, sites = synth.product_mps(config)
    mps = tnt.mps(bonds, sites, 2)
    for _ in range(steps):
        r = tnt.tebd_step(mps, h, dt, chi, renormalise=False)
    dens = np.diag(mps.correlation(oobs.annihilator(1), -1)).real
    hsp = np.zeros((L, L))
    for j in range(L - 1):
        hsp[j, j + 1] = hsp[j + 1, j] = -1.0
    Ut = scipy.linalg.expm(-1j * dt * steps * hsp)
    ref = (np.abs(Ut) ** 2) @ np.asarray(config, dtype=float)
    err = np.max(np.abs(dens - ref))
    print(f"  t = {dt * steps}: max|n_j - n_j(free fermions)| = {err:.2e}, max chi {r['max_chi']}")
    assert err < 1e-4
    assert abs(dens.sum() - 25) < 1e-9


def test_tebd_rejects_charge_mixing(tnt):
    from paper_1610_02244_amd import binding as B
    bonds, sites = synth.product_mps((1, 0, 1))
    mps = tnt.mps(bonds, sites, 2)
    h = tnt.bond_hamiltonians_bose_hubbard(3, 1, 1.0, 0.0)
    h[0, 0, 1] = h[0, 1, 0] = 0.3  # couples (0,0) with (0,1)
    with pytest.raises(B.TntError) as ei:
        tnt.tebd_step(mps, h, 0.01, 4)
    assert ei.value.code == -3  # TNT_E_CHARGE


def test_tebd_two_site_chain(tnt):
    # L = 2: one bond, gated twice with dt/2 = one exact gate of dt
    print("[tebd] L=2", flush=True)
    h = tnt.bond_hamiltonians_bose_hubbard(2, 2, 1.0, 1.5, 0.2)
    bonds, sites = synth.product_mps((2, 0))
    mps = tnt.mps(bonds, sites, 3)
    tnt.tebd_step(mps, h, 0.3, 9)
    hs = otebd.bond_hamiltonians_bh(2, 2, 1.0, 1.5, 0.2)
    G = otebd.gate(hs[0], 0.3)
    # the state of two sites as a 3 x 3 matrix psi[s1, s2]
    psi0 = np.zeros(9, complex)
    psi0[2 * 3 + 0] = 1.0
    want = (G @ psi0).reshape(3, 3)
    got = np.zeros((3, 3), complex)
    hb, hsites = mps.bonds(), mps.sites()
    for (q, s1), A in hsites[0].items():
        for (q2, s2), Bm in hsites[1].items():
            if q2 == q + s1:
                got[s1, s2] += (A @ Bm)[0, 0]
    np.testing.assert_allclose(got, want, atol=1e-12)
