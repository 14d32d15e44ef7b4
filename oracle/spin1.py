"""Spin-1 isotropic Heisenberg chain: the workload of the paper's DMRG timing
table (Table tab:dmrgtimes, Sec. 3: L = 101, chi = 200, U(1) blocking).

    H = J sum_{j<L} S_j . S_{j+1}
      = J sum_{j<L} [ Sz_j Sz_{j+1} + (S+_j S-_{j+1} + S-_j S+_{j+1}) / 2 ]

Test infrastructure (an oracle): plain NumPy, written from the definition.

Local states are labelled by s = m + 1 in {0, 1, 2} (m = S^z), so the U(1)
charge of a site is s and the total-S^z = 0 sector of L sites is the
total-charge-L sector: the same state space as a boson chain with n_max = 2
and N = L (the occupation basis of `model.fixed_n_basis` enumerates it).
"""
from __future__ import annotations

import math

import numpy as np

from . import model


def local_ops():
    """(S+, S-, Sz, I) as dense 3 x 3 real arrays on s = m + 1 = 0, 1, 2.

    S+|m> = sqrt(2 - m (m + 1)) |m + 1>: both raising elements are sqrt(2)
    for spin 1.
    """
    sp = np.zeros((3, 3))
    for s in range(2):
        m = s - 1
        sp[s + 1, s] = math.sqrt(2 - m * (m + 1))
    sz = np.diag([-1.0, 0.0, 1.0])
    return sp, sp.T.copy(), sz, np.eye(3)


def ed_hamiltonian(L: int, J: float = 1.0):
    """Dense H on the total-S^z = 0 sector, built configuration by
    configuration from the bond terms.  Returns (H, basis)."""
    basis = model.fixed_n_basis(L, L, 2)
    index = {c: i for i, c in enumerate(basis)}
    H = np.zeros((len(basis), len(basis)))
    sq2 = math.sqrt(2.0)
    for i, c in enumerate(basis):
        for j in range(L - 1):
            mj, mk = c[j] - 1, c[j + 1] - 1
            H[i, i] += J * mj * mk
            # S+_j S-_{j+1} / 2: raise site j, lower site j+1 (each factor sqrt(2))
            if c[j] < 2 and c[j + 1] > 0:
                c2 = list(c)
                c2[j] += 1
                c2[j + 1] -= 1
                H[index[tuple(c2)], i] += 0.5 * J * sq2 * sq2
            # S-_j S+_{j+1} / 2
            if c[j] > 0 and c[j + 1] < 2:
                c2 = list(c)
                c2[j] -= 1
                c2[j + 1] += 1
                H[index[tuple(c2)], i] += 0.5 * J * sq2 * sq2
    return H, basis


def kron_hamiltonian(L: int, J: float = 1.0):
    """Dense H on the full 3^L space from Kronecker products of the spin-1
    matrices S^x, S^y, S^z (an independent construction; site 1 most
    significant, state index sum_j s_j 3^(L-j))."""
    sp, sm, sz, I = local_ops()
    sx = 0.5 * (sp + sm)
    sy = -0.5j * (sp - sm)

    def at(op, j):
        out = np.ones((1, 1))
        for k in range(L):
            out = np.kron(out, op if k == j else I)
        return out

    H = np.zeros((3 ** L, 3 ** L), dtype=complex)
    for j in range(L - 1):
        for op in (sx, sy, sz):
            H += J * at(op, j) @ at(op, j + 1)
    return H


def total_spin_squared(L: int):
    """S_tot^2 on the full 3^L space (Kronecker products)."""
    sp, sm, sz, I = local_ops()
    sx = 0.5 * (sp + sm)
    sy = -0.5j * (sp - sm)

    def total(op):
        tot = np.zeros((3 ** L, 3 ** L), dtype=complex)
        for j in range(L):
            out = np.ones((1, 1))
            for k in range(L):
                out = np.kron(out, op if k == j else I)
            tot += out
        return tot

    Sx, Sy, Sz = total(sx), total(sy), total(sz)
    return Sx @ Sx + Sy @ Sy + Sz @ Sz


def sector_projector(L: int):
    """Columns selecting the total-S^z = 0 configurations of the full space
    (the same ordering as `ed_hamiltonian`'s basis)."""
    return model.fixed_n_projector(L, L, 2)


def mpo(J: float = 1.0):
    """Lower-triangular MPO tensor W[w, w', s', s] (D = 5) and bond charges.

        W = [[I,          0,          0,          0,      0],
             [S-,         0,          0,          0,      0],
             [S+,         0,          0,          0,      0],
             [Sz,         0,          0,          0,      0],
             [0,   J/2 S+,     J/2 S-,      J Sz,      I]]

    The chain operator is e_4^T W_1 ... W_L e_0.  Bond charges qw =
    (0, +1, -1, 0, 0): every nonzero element obeys s' - s = qw[w'] - qw[w].
    """
    sp, sm, sz, I = local_ops()
    W = np.zeros((5, 5, 3, 3))
    W[0, 0] = I
    W[1, 0] = sm
    W[2, 0] = sp
    W[3, 0] = sz
    W[4, 1] = 0.5 * J * sp
    W[4, 2] = 0.5 * J * sm
    W[4, 3] = J * sz
    W[4, 4] = I
    return W, [0, 1, -1, 0, 0]


MPO_LEFT = 4   # index selected by the left boundary vector
MPO_RIGHT = 0  # index selected by the right boundary vector


def ed_ground_energy(L: int, J: float = 1.0) -> float:
    H, _ = ed_hamiltonian(L, J)
    return float(np.linalg.eigvalsh(H)[0])
