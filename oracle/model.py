"""Bose-Hubbard model: local operators, exact diagonalisation, closed forms, MPO.

Paper Sec. 5, Eq. (2):
    H = -J sum_{j<L} (b_j^+ b_{j+1} + h.c.) + U/2 sum_j n_j (n_j - 1)
        + V sum_j (j - j_c)^2 n_j
with an occupancy cut-off n_max per site.  A chemical potential term -mu n_j
is allowed as well (a constant -mu N at fixed N).  Every workload here has
V = 0.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


# ---------------------------------------------------------------------------
# local operators on |n>, n = 0..nmax
# ---------------------------------------------------------------------------

def local_ops(nmax: int):
    """(b, bdag, n, I) as dense (d, d) real arrays; b|n> = sqrt(n)|n-1>."""
    d = nmax + 1
    b = np.zeros((d, d))
    for n in range(1, d):
        b[n - 1, n] = math.sqrt(n)
    num = np.diag(np.arange(d, dtype=float))
    return b, b.T.copy(), num, np.eye(d)


def onsite(nmax: int, U: float, mu: float) -> np.ndarray:
    """h = U/2 n(n-1) - mu n (diagonal, (d, d))."""
    n = np.arange(nmax + 1, dtype=float)
    return np.diag(0.5 * U * n * (n - 1.0) - mu * n)


# ---------------------------------------------------------------------------
# exact diagonalisation at fixed particle number, straight from Eq. (2)
# ---------------------------------------------------------------------------

def fixed_n_basis(L: int, N: int, nmax: int):
    """All occupation tuples of L sites (each 0..nmax) with total N, sorted."""
    out = []

    def rec(prefix, left, sites):
        if sites == 0:
            if left == 0:
                out.append(tuple(prefix))
            return
        for n in range(min(nmax, left) + 1):
            if left - n <= (sites - 1) * nmax:
                rec(prefix + [n], left - n, sites - 1)

    rec([], N, L)
    return out


def ed_hamiltonian(L, N, nmax, J, U, mu=0.0, V=0.0, jc=None):
    """Dense Eq. (2) Hamiltonian on the fixed-N occupation basis (real symmetric)."""
    basis = fixed_n_basis(L, N, nmax)
    index = {c: i for i, c in enumerate(basis)}
    dim = len(basis)
    H = np.zeros((dim, dim))
    if jc is None:
        jc = (L + 1) / 2.0
    for i, c in enumerate(basis):
        diag = 0.0
        for j, n in enumerate(c):
            diag += 0.5 * U * n * (n - 1) - mu * n + V * ((j + 1) - jc) ** 2 * n
        H[i, i] = diag
        for j in range(L - 1):
            # b_j^+ b_{j+1}: move one boson from site j+1 to site j
            if c[j + 1] > 0 and c[j] < nmax:
                c2 = list(c)
                amp = math.sqrt(c[j + 1]) * math.sqrt(c[j] + 1)
                c2[j + 1] -= 1
                c2[j] += 1
                H[index[tuple(c2)], i] += -J * amp
            # b_j b_{j+1}^+: move one boson from site j to site j+1
            if c[j] > 0 and c[j + 1] < nmax:
                c2 = list(c)
                amp = math.sqrt(c[j]) * math.sqrt(c[j + 1] + 1)
                c2[j] -= 1
                c2[j + 1] += 1
                H[index[tuple(c2)], i] += -J * amp
    return H, basis


def ed_ground_energy(L, N, nmax, J, U, mu=0.0, V=0.0):
    H, _ = ed_hamiltonian(L, N, nmax, J, U, mu, V)
    return float(np.linalg.eigvalsh(H)[0])


# closed forms -------------------------------------------------------------

def e0_free_bosons(L, N, J):
    """U = 0 and nmax >= N: all bosons in the lowest open-chain orbital."""
    return -2.0 * J * N * math.cos(math.pi / (L + 1))


def e0_hardcore(L, N, J):
    """nmax = 1: Jordan-Wigner free fermions filling the N lowest orbitals."""
    return -2.0 * J * sum(math.cos(k * math.pi / (L + 1)) for k in range(1, N + 1))


def e0_atomic(L, N, nmax, U):
    """J = 0: bosons spread as evenly as possible (U > 0)."""
    base, extra = divmod(N, L)
    occ = [base + 1] * extra + [base] * (L - extra)
    assert max(occ) <= nmax
    return sum(0.5 * U * n * (n - 1) for n in occ)


# ---------------------------------------------------------------------------
# matrix product operator (Sec. 4.3: the Hamiltonian written as a chain)
# ---------------------------------------------------------------------------

def bh_mpo(nmax: int, J: float, U: float, mu: float = 0.0):
    """Lower-triangular Bose-Hubbard MPO tensor W[w, w', s', s] and bond charges.

    Rows w are the left MPO bond, columns w' the right one:
        W = [[I, 0, 0, 0], [b, 0, 0, 0], [b^+, 0, 0, 0], [h, -J b^+, -J b, I]]
    The chain operator is e_3^T W_1 ... W_L e_0.  The MPO bond index carries
    the U(1) charge qw = (0, +1, -1, 0) so that every nonzero element obeys
    s' - s = qw[w'] - qw[w] (the charged singleton-leg idea of appendix
    A.1.1 applied to the MPO bond).
    """
    b, bd, _, I = local_ops(nmax)
    h = onsite(nmax, U, mu)
    d = nmax + 1
    W = np.zeros((4, 4, d, d))
    W[0, 0] = I
    W[1, 0] = b
    W[2, 0] = bd
    W[3, 0] = h
    W[3, 1] = -J * bd
    W[3, 2] = -J * b
    W[3, 3] = I
    qw = [0, 1, -1, 0]
    return W, qw


MPO_LEFT = 3   # index selected by the left boundary vector
MPO_RIGHT = 0  # index selected by the right boundary vector
MPO_ADJOINT = [0, 2, 1, 3]  # W[w] blocks pair with their adjoints: b <-> b^+


def mpo_to_dense(W_list, left=MPO_LEFT, right=MPO_RIGHT):
    """Contract e_left^T W_1 ... W_L e_right into a dense (d^L, d^L) matrix.

    Row index = (s'_1 ... s'_L), column index = (s_1 ... s_L), site 1 most
    significant.
    """
    cur = W_list[0][left]  # (D, d, d): [w', s', s]
    for W in W_list[1:]:
        # cur[w, S, T] with S, T multi-indices; contract the MPO bond
        D, dS, dT = cur.shape
        d = W.shape[2]
        nxt = np.einsum('wST,wvab->vSaTb', cur, W)
        cur = nxt.reshape(W.shape[1], dS * d, dT * d)
    return cur[right]


def fixed_n_projector(L, N, nmax):
    """Column selector (d^L, dim) from the fixed-N basis into the full space."""
    d = nmax + 1
    basis = fixed_n_basis(L, N, nmax)
    P = np.zeros((d ** L, len(basis)))
    for i, c in enumerate(basis):
        idx = 0
        for n in c:
            idx = idx * d + n
        P[idx, i] = 1.0
    return P


def all_configs(L, nmax):
    return list(itertools.product(range(nmax + 1), repeat=L))
