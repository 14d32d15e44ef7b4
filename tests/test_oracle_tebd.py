"""Pins of the TEBD oracle (second-order two-site step).

* The bond Hamiltonians sum to Eq. 2's H (Kronecker products projected on the
  fixed-N sector, against the oracle's configuration-by-configuration ED).
* Exact evolution: at exact chi the step's state approaches exp(-iHt) psi_0
  (scipy expm on the sector) with error O(dt^2): halving dt divides it by 4.
  A wrong sign in the exponent, a dropped on-site share or a first-order
  ordering fails this.
* Hard-core bosons (n_max = 1) melting from a charge-density wave have the
  densities of free fermions: n_j(t) = sum_k |[exp(-i h t)]_jk|^2 n_k(0),
  h the single-particle hopping matrix (the paper's second example).
* With renormalisation off and no truncation the norm stays 1.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import model
from oracle import observables as oobs
from oracle import tebd as otebd


def dense_sector_state(bonds, sites, d, basis):
    index = {c: i for i, c in enumerate(basis)}
    v = np.zeros(len(basis), dtype=complex)
    L = len(sites)
    for conf in itertools.product(range(d), repeat=L):
        q = next(iter(bonds[0]))
        M = np.ones((1, 1), dtype=complex)
        for j, s in enumerate(conf):
            A = sites[j].get((q, s))
            if A is None:
                M = None
                break
            M = M @ A
            q += s
        if M is not None:
            v[index[conf]] = M[0, 0]
    return v


def test_bond_hamiltonians_sum_to_H():
    L, N, nmax, J, U, mu = 5, 3, 2, 0.8, 2.5, 0.3
    d = nmax + 1
    hs = otebd.bond_hamiltonians_bh(L, nmax, J, U, mu)
    H = np.zeros((d ** L, d ** L))
    for j, h in enumerate(hs):
        H += np.kron(np.kron(np.eye(d ** j), h), np.eye(d ** (L - j - 2)))
    P = model.fixed_n_projector(L, N, nmax)
    Hed, _ = model.ed_hamiltonian(L, N, nmax, J, U, mu)
    np.testing.assert_allclose(P.T @ H @ P, Hed, atol=1e-12)


def evolve(config, nmax, hs, dt, steps, chi=256, renormalise=True):
    d = nmax + 1
    bonds, sites = synth.product_mps(config)
    for _ in range(steps):
        bonds, sites, rec = otebd.tebd_step(bonds, sites, hs, dt, d, chi,
                                            trunc={"renormalise": renormalise})
    return bonds, sites


def test_second_order_convergence_to_exact_evolution():
    L, nmax, J, U, mu = 5, 2, 1.0, 2.0, 0.3
    config = (1, 0, 2, 0, 1)
    N = sum(config)
    basis = model.fixed_n_basis(L, N, nmax)
    Hed, _ = model.ed_hamiltonian(L, N, nmax, J, U, mu)
    psi0 = np.zeros(len(basis), dtype=complex)
    psi0[basis.index(config)] = 1.0
    t = 0.4
    exact = scipy.linalg.expm(-1j * t * Hed) @ psi0
    hs = otebd.bond_hamiltonians_bh(L, nmax, J, U, mu)
    errs = []
    for steps in (4, 8):
        bonds, sites = evolve(config, nmax, hs, t / steps, steps)
        v = dense_sector_state(bonds, sites, nmax + 1, basis)
        errs.append(np.linalg.norm(v - exact))
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, (errs, ratio)
    assert errs[1] < 2e-3


def free_fermion_densities(L, config, t, J=1.0):
    h = np.zeros((L, L))
    for j in range(L - 1):
        h[j, j + 1] = h[j + 1, j] = -J
    Ut = scipy.linalg.expm(-1j * t * h)
    return (np.abs(Ut) ** 2) @ np.asarray(config, dtype=float)


def test_hardcore_cdw_matches_free_fermions():
    L, dt, steps = 8, 0.02, 25
    config = tuple(1 - (j % 2) for j in range(L))
    hs = otebd.bond_hamiltonians_bh(L, 1, 1.0, 0.0)
    bonds, sites = evolve(config, 1, hs, dt, steps, chi=16)
    dens = np.diag(oobs.correlation_matrix(bonds, sites, 2, oobs.annihilator(1))).real
    ref = free_fermion_densities(L, config, dt * steps)
    assert np.max(np.abs(dens - ref)) < 5e-5  # Trotter error O(dt^2 t), 1.4e-5 here
    # and the densities really moved
    assert np.max(np.abs(dens - np.asarray(config))) > 0.1


def test_norm_conserved_without_truncation():
    hs = otebd.bond_hamiltonians_spin1(6)
    bonds, sites = evolve((2, 0, 1, 1, 2, 0), 2, hs, 0.05, 3, renormalise=False)
    from oracle import dmrg as odmrg
    assert odmrg.norm2(bonds, sites, 3) == pytest.approx(1.0, abs=1e-12)
