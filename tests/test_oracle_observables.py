"""Pins of the observables oracle (rho_ij = <b^dagger_i b_j>, <n_j>).

* Brute force: the MPS expanded into its full state vector configuration by
  configuration (a plain product of site matrices, written here), and rho_ij
  applied on the occupation basis from the definition of b.
* Closed form: at U = 0 with n_max >= N the ground state puts all N bosons in
  the lowest single-particle orbital of the open chain,
  phi(j) = sqrt(2/(L+1)) sin(pi j/(L+1)), so rho_ij = N phi(i) phi(j).
* Invariants: Hermitian; trace = N; <n_j> equals the oracle's densities.
"""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import dmrg as odmrg
from oracle import observables as oobs
from oracle import spin1 as ospin1


def dense_state(bonds, sites, d):
    """psi[config] for every configuration (n_1..n_L) with the MPS charges."""
    L = len(sites)
    psi = {}
    for conf in itertools.product(range(d), repeat=L):
        q = next(iter(bonds[0]))
        M = np.ones((1, 1), dtype=complex)
        ok = True
        for j, s in enumerate(conf):
            A = sites[j].get((q, s))
            if A is None:
                ok = False
                break
            M = M @ A
            q += s
        if ok:
            psi[conf] = M[0, 0]
    return psi


def brute_correlation(psi, L, op):
    """<O^dagger_i O_j> on the configuration basis, O applied entry by entry."""
    nrm = sum(abs(v) ** 2 for v in psi.values())
    C = np.zeros((L, L), dtype=complex)
    d = op.shape[0]

    def apply(site, mat, vec):
        out = {}
        for conf, amp in vec.items():
            for sp in range(d):
                c = mat[sp, conf[site]]
                if c != 0.0:
                    new = conf[:site] + (sp,) + conf[site + 1:]
                    out[new] = out.get(new, 0.0) + c * amp
        return out

    for i in range(L):
        for j in range(L):
            phi = apply(j, op, psi)           # O_j |psi>
            phi = apply(i, op.T, phi)          # O^dagger_i O_j |psi>
            C[i, j] = sum(np.conj(psi.get(k, 0.0)) * v for k, v in phi.items()) / nrm
    return C


@pytest.mark.parametrize("L,N,nmax,chi,seed", [(4, 3, 2, 4, 1), (5, 4, 2, 6, 2), (5, 2, 3, 5, 3)])
def test_density_matrix_equals_brute_force(L, N, nmax, chi, seed):
    bonds, sites = synth.random_mps(L, N, nmax, chi, seed)
    d = nmax + 1
    b = oobs.annihilator(nmax)
    C = oobs.correlation_matrix(bonds, sites, d, b)
    ref = brute_correlation(dense_state(bonds, sites, d), L, b)
    np.testing.assert_allclose(C, ref, atol=1e-12, rtol=0)
    np.testing.assert_allclose(C, C.conj().T, atol=1e-12)
    assert np.trace(C).real == pytest.approx(N, abs=1e-12)
    np.testing.assert_allclose(np.diag(C).real, odmrg.site_densities(bonds, sites, d), atol=1e-12)


def test_spin_lowering_correlation_equals_brute_force():
    # O = S^- on s = S^z + 1: C[i, j] = <S^+_i S^-_j>
    bonds, sites = synth.random_mps(5, 5, 2, 6, 7)
    sp, sm, _, _ = ospin1.local_ops()
    C = oobs.correlation_matrix(bonds, sites, 3, sm)
    ref = brute_correlation(dense_state(bonds, sites, 3), 5, sm)
    np.testing.assert_allclose(C, ref, atol=1e-12, rtol=0)


def test_free_boson_condensate_closed_form():
    L, N, nmax = 6, 3, 3
    bonds, sites, _ = odmrg.run_dmrg(L, N, nmax, 1.0, 0.0, 0.0, 64, seed=5, sweeps=3,
                                      random_mps=synth.random_mps)
    C = oobs.correlation_matrix(bonds, sites, nmax + 1, oobs.annihilator(nmax))
    phi = np.array([math.sqrt(2 / (L + 1)) * math.sin(math.pi * j / (L + 1))
                    for j in range(1, L + 1)])
    np.testing.assert_allclose(C.real, N * np.outer(phi, phi), atol=1e-8)
    assert np.max(np.abs(C.imag)) < 1e-10


def test_reflection_symmetry_of_ground_state():
    # Eq. 2 with V = 0 on an open chain is symmetric under j -> L + 1 - j, so the
    # (non-degenerate) ground state has rho_ij = rho_{L+1-i, L+1-j}
    L, N, nmax = 6, 4, 2
    bonds, sites, _ = odmrg.run_dmrg(L, N, nmax, 1.0, 3.0, 0.0, 64, seed=8, sweeps=3,
                                      random_mps=synth.random_mps)
    C = oobs.correlation_matrix(bonds, sites, nmax + 1, oobs.annihilator(nmax))
    np.testing.assert_allclose(C, C[::-1, ::-1], atol=1e-8)
    assert np.trace(C).real == pytest.approx(N, abs=1e-10)
