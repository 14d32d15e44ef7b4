"""Pins of the spin-1 Heisenberg oracle (the paper's DMRG timing workload).

- two sites: the spectrum of S_1 . S_2 on the S^z = 0 sector is
  {-2, -1, +1} (total spin 0, 1, 2: S1.S2 = (S(S+1) - 4) / 2);
- the occupation-basis Hamiltonian equals the Kronecker-product one
  restricted to S^z = 0 (two independent constructions), L = 3..6;
- the MPO contracted to a dense matrix equals the Kronecker-product
  Hamiltonian, L = 2..5;
- every MPO element respects the bond charges;
- the ground state of an even open chain is a singlet: <S_tot^2> = 0.
"""
import numpy as np
import pytest

from oracle import model, spin1


def test_two_site_spectrum():
    H, basis = spin1.ed_hamiltonian(2, 1.0)
    assert sorted(basis) == [(0, 2), (1, 1), (2, 0)]
    np.testing.assert_allclose(np.linalg.eigvalsh(H), [-2.0, -1.0, 1.0], atol=1e-14)
    assert spin1.ed_ground_energy(2, 0.7) == pytest.approx(-1.4, abs=1e-14)


@pytest.mark.parametrize("L", [3, 4, 5, 6])
def test_occupation_basis_equals_kronecker(L):
    H, _ = spin1.ed_hamiltonian(L, 1.3)
    P = spin1.sector_projector(L)
    Hk = P.T @ spin1.kron_hamiltonian(L, 1.3) @ P
    assert np.abs(Hk.imag).max() < 1e-14
    np.testing.assert_allclose(Hk.real, H, atol=1e-13)


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_mpo_equals_kronecker(L):
    W, qw = spin1.mpo(0.9)
    dense = model.mpo_to_dense([W] * L, spin1.MPO_LEFT, spin1.MPO_RIGHT)
    Hk = spin1.kron_hamiltonian(L, 0.9)
    np.testing.assert_allclose(dense, Hk.real, atol=1e-13)
    assert np.abs(Hk.imag).max() < 1e-14


def test_mpo_charges():
    W, qw = spin1.mpo(1.0)
    for w in range(5):
        for wp in range(5):
            for sp in range(3):
                for s in range(3):
                    if W[w, wp, sp, s] != 0.0:
                        assert sp - s == qw[wp] - qw[w]


@pytest.mark.parametrize("L", [4, 6])
def test_even_chain_ground_state_is_singlet(L):
    Hk = spin1.kron_hamiltonian(L, 1.0)
    P = spin1.sector_projector(L)
    H = (P.T @ Hk @ P).real
    w, v = np.linalg.eigh(H)
    assert w[1] - w[0] > 1e-6  # non-degenerate
    psi = P @ v[:, 0]
    s2 = np.vdot(psi, spin1.total_spin_squared(L) @ psi).real
    assert abs(s2) < 1e-10
