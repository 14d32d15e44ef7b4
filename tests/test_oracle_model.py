"""Pins of the oracle's Hamiltonian, exact diagonalisation and MPO.

Independent checks: closed forms of exactly solvable limits, a second
brute-force construction of Eq. (2) from Kronecker products on the full
d^L space, a two-site analytic spectrum, and the J -> -J gauge symmetry.
"""
import math

import numpy as np
import pytest

from oracle import model


def kron_hamiltonian(L, nmax, J, U, mu=0.0):
    """Eq. (2) on the full d^L space from Kronecker products (site 1 leftmost)."""
    d = nmax + 1
    b = np.diag(np.sqrt(np.arange(1, d)), k=1)
    n = np.diag(np.arange(d, dtype=float))
    I = np.eye(d)

    def op_at(ops):
        out = np.ones((1, 1))
        for j in range(L):
            out = np.kron(out, ops.get(j, I))
        return out

    H = np.zeros((d ** L, d ** L))
    for j in range(L - 1):
        H += -J * op_at({j: b.T, j + 1: b})
        H += -J * op_at({j: b, j + 1: b.T})
    for j in range(L):
        H += op_at({j: 0.5 * U * n @ (n - I) - mu * n})
    return H


@pytest.mark.parametrize("L,N,nmax", [(6, 1, 1), (6, 2, 2), (5, 3, 3), (7, 1, 3)])
def test_free_bosons_closed_form(L, N, nmax):
    # U = 0 with nmax >= N: every boson in the lowest single-particle orbital
    assert model.ed_ground_energy(L, N, nmax, 1.0, 0.0) == pytest.approx(
        model.e0_free_bosons(L, N, 1.0), abs=1e-12)


def test_free_bosons_needs_enough_occupancy():
    # with nmax < N the closed form is not reached (the cut-off costs energy)
    assert model.ed_ground_energy(6, 2, 1, 1.0, 0.0) > model.e0_free_bosons(6, 2, 1.0) + 1e-3


@pytest.mark.parametrize("L,N", [(6, 3), (8, 4), (7, 2)])
def test_hardcore_free_fermions(L, N):
    assert model.ed_ground_energy(L, N, 1, 1.0, 5.0) == pytest.approx(
        model.e0_hardcore(L, N, 1.0), abs=1e-12)


def test_atomic_limit():
    assert model.ed_ground_energy(4, 6, 3, 0.0, 2.0) == pytest.approx(4.0, abs=1e-13)
    assert model.e0_atomic(4, 6, 3, 2.0) == pytest.approx(4.0)


@pytest.mark.parametrize("J,U", [(1.0, 2.0), (0.7, 5.0), (1.0, 0.0)])
def test_two_site_analytic(J, U):
    # basis {|02>, |11>, |20>}: the symmetric sector gives U/2 - sqrt(U^2/4 + 4 J^2)
    e = model.ed_ground_energy(2, 2, 2, J, U)
    assert e == pytest.approx(U / 2 - math.sqrt(U * U / 4 + 4 * J * J), abs=1e-13)


@pytest.mark.parametrize("L,N,nmax,U", [(5, 4, 2, 2.0), (4, 4, 3, 3.3), (6, 3, 2, 1.0)])
def test_ed_matches_kronecker_construction(L, N, nmax, U):
    H, basis = model.ed_hamiltonian(L, N, nmax, 1.0, U, mu=0.3)
    Hk = kron_hamiltonian(L, nmax, 1.0, U, mu=0.3)
    P = model.fixed_n_projector(L, N, nmax)
    np.testing.assert_allclose(P.T @ Hk @ P, H, atol=1e-13)


def test_j_sign_gauge_invariance():
    e1 = np.linalg.eigvalsh(model.ed_hamiltonian(6, 6, 2, 1.0, 2.0)[0])
    e2 = np.linalg.eigvalsh(model.ed_hamiltonian(6, 6, 2, -1.0, 2.0)[0])
    np.testing.assert_allclose(e1, e2, atol=1e-12)


@pytest.mark.parametrize("L,nmax,U", [(4, 2, 2.0), (3, 3, 1.5), (5, 1, 0.0)])
def test_mpo_equals_hamiltonian(L, nmax, U):
    W, qw = model.bh_mpo(nmax, 1.0, U, mu=0.25)
    Hm = model.mpo_to_dense([W] * L)
    Hk = kron_hamiltonian(L, nmax, 1.0, U, mu=0.25)
    np.testing.assert_allclose(Hm, Hk, atol=1e-14)


def test_mpo_charge_rule():
    # every nonzero W[w, w', s', s] obeys s' - s = qw[w'] - qw[w]
    W, qw = model.bh_mpo(4, 1.0, 3.0, 0.5)
    for w, wp, sp, s in zip(*np.nonzero(W)):
        assert sp - s == qw[wp] - qw[w]


def test_mpo_adjoint_pairs():
    # W[w, w'] and W[pair(w), pair(w')]^T are the same operator (real MPO)
    W, qw = model.bh_mpo(3, 1.0, 2.0)
    p = model.MPO_ADJOINT
    for w in range(4):
        for wp in range(4):
            np.testing.assert_array_equal(W[w, wp], W[p[w], p[wp]].T)


def test_cfg1_ed_dimension_and_ground_state():
    H, basis = model.ed_hamiltonian(8, 8, 2, 1.0, 2.0)
    assert len(basis) == 1107
    # variational sanity: the ground energy lies between the atomic and free limits
    e = float(np.linalg.eigvalsh(H)[0])
    assert model.e0_free_bosons(8, 8, 1.0) < e < model.e0_atomic(8, 8, 2, 2.0)
