"""Pins of the oracle's two-site sweep.

* With chi at least the exact bond dimension the sweep reaches the exact
  ground energy: cfg1's chain against exact diagonalisation, hard-core bosons
  against free fermions, U = 0 against the single-orbital closed form.
* At chi below that it stays variational (E >= E_exact).
* The energy reported by the last bond equals <psi|H|psi>/<psi|psi> of the
  returned MPS contracted as a whole network; the density sums to N and is
  reflection symmetric (V = 0).
"""
import numpy as np
import pytest

import synth
from oracle import dmrg, model


def run(L, N, nmax, U, chi, seed, sweeps, r=1e-12):
    return dmrg.run_dmrg(L, N, nmax, 1.0, U, 0.0, chi, seed, sweeps, trunc=dict(r=r),
                         random_mps=synth.random_mps)


def test_cfg1_exact_chi_reaches_ed():
    s = synth.CONFIGS["cfg1"]
    e_ed = model.ed_ground_energy(s.L, s.N, s.nmax, s.J, s.U)
    bonds, sites, recs = run(s.L, s.N, s.nmax, s.U, 81, s.seed, 2)
    assert recs[-1][-1]["E"] == pytest.approx(e_ed, abs=1e-10)
    assert max(sum(b.values()) for b in bonds) <= 81


def test_cfg1_chi16_variational_and_consistent():
    s = synth.CONFIGS["cfg1"]
    e_ed = model.ed_ground_energy(s.L, s.N, s.nmax, s.J, s.U)
    bonds, sites, recs = run(s.L, s.N, s.nmax, s.U, s.chi, s.seed, s.sweeps)
    e = recs[-1][-1]["E"]
    assert e >= e_ed - 1e-12
    assert e - e_ed < 1e-3
    W, qw = model.bh_mpo(s.nmax, s.J, s.U)
    assert dmrg.expectation(bonds, sites, [W] * s.L, qw, s.d) == pytest.approx(e, abs=1e-10)
    dens = dmrg.site_densities(bonds, sites, s.d)
    assert sum(dens) == pytest.approx(s.N, abs=1e-10)
    np.testing.assert_allclose(dens, dens[::-1], atol=1e-4)
    # a later sweep ends no higher than an earlier one (bond energies inside a
    # sweep may rise by the truncation error, so compare sweep ends)
    ends = [sw[-1]["E"] for sw in recs]
    assert max(np.diff(ends)) < 1e-9


def test_hardcore_free_fermions():
    L, N = 12, 6
    bonds, sites, recs = run(L, N, 1, 0.0, 64, 7, 3)
    assert recs[-1][-1]["E"] == pytest.approx(model.e0_hardcore(L, N, 1.0), abs=1e-10)
    dens = dmrg.site_densities(bonds, sites, 2)
    np.testing.assert_allclose(dens, dens[::-1], atol=1e-9)


@pytest.mark.slow
def test_free_bosons_single_orbital():
    # U = 0, nmax >= N: the exact state has one Schmidt value per sector, chi = N + 1
    L, N = 16, 4
    bonds, sites, recs = run(L, N, 4, 0.0, N + 1, 8, 6)
    assert recs[-1][-1]["E"] == pytest.approx(model.e0_free_bosons(L, N, 1.0), abs=1e-9)
