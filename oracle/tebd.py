"""Two-site TEBD time step (time evolution of an MPS by Trotterised two-site
gates, Sec. 1 and the time-evolution example of Sec. 5, Fig.
fig:time_evolve_results; the timing workload of Table tab:tebdtimes).

Test infrastructure (an oracle): plain NumPy / SciPy, written from the
definitions.  H = sum_j h_j over the bonds (j, j+1); one step of dt applies
exp(-i h_j dt/2) for j = 1..L-1 (moving the orthogonality centre right) and
then for j = L-1..1 (moving it back): the symmetric product is a
second-order Trotter step.  Each gate acts on theta = A_j B_{j+1}, which is
then split by the truncated SVD of appendix B.1.2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import model
from . import svd as _svd
from .dmrg import form_theta


def bond_hamiltonians_bh(L, nmax, J, U, mu=0.0):
    """h_j (d^2 x d^2, index s1 d + s2) of Eq. 2 with V = 0:
    -J (b^dagger b + b b^dagger) on the bond plus the on-site terms
    U/2 n(n-1) - mu n, each shared equally by the site's two bonds (an end
    site gives its whole term to its only bond), so that sum_j h_j = H."""
    b, bd, n, I = model.local_ops(nmax)
    hs = model.onsite(nmax, U, mu)
    out = []
    for j in range(1, L):
        wl = 1.0 if j == 1 else 0.5
        wr = 1.0 if j + 1 == L else 0.5
        h = -J * (np.kron(bd, b) + np.kron(b, bd)) + wl * np.kron(hs, I) + wr * np.kron(I, hs)
        out.append(h)
    return out


def bond_hamiltonians_spin1(L, J=1.0):
    """h_j = J S_j . S_{j+1} on s = S^z + 1 (no on-site terms)."""
    from .spin1 import local_ops
    sp, sm, sz, _ = local_ops()
    h = J * (np.kron(sz, sz) + 0.5 * (np.kron(sp, sm) + np.kron(sm, sp)))
    return [h.copy() for _ in range(L - 1)]


def gate(h, tau):
    """exp(-i tau h) as a d^2 x d^2 complex matrix."""
    return scipy.linalg.expm(-1j * tau * np.asarray(h, dtype=float))


def apply_gate(th, G, d):
    """theta'[(qa, s1', s2')] = sum_{s1, s2} G[s1' d + s2', s1 d + s2] theta[(qa, s1, s2)]."""
    out = {}
    for (qa, s1p, s2p), blk in th.items():
        acc = np.zeros_like(blk)
        for s1 in range(d):
            for s2 in range(d):
                src = th.get((qa, s1, s2))
                if src is None or src.shape != blk.shape:
                    continue
                acc = acc + G[s1p * d + s2p, s1 * d + s2] * src
        out[(qa, s1p, s2p)] = acc
    return out


def tebd_step(bonds, sites, hs, dt, d, chi_max, trunc=None):
    """One second-order step on an MPS whose centre is site 1 (sites 2..L
    right-isometries).  Returns (bonds, sites, records) with one record
    (pass, j, eps, chi) per gate; the centre is back on site 1."""
    trunc = dict(trunc or {})
    L = len(sites)
    bonds = [dict(x) for x in bonds]
    sites = [dict(x) for x in sites]
    records = []
    for direction in ("right", "left"):
        js = range(1, L) if direction == "right" else range(L - 1, 0, -1)
        for j in js:
            left, right = bonds[j - 1], bonds[j + 1]
            th = form_theta(sites[j - 1], sites[j], left, right, d)
            th = apply_gate(th, gate(hs[j - 1], dt / 2), d)
            sv = _svd.svd_truncate(th, left, right, d, chi_max, absorb=direction, **trunc)
            sites[j - 1], sites[j] = sv["A"], sv["B"]
            bonds[j] = sv["bond"]
            records.append({"pass": direction, "j": j, "eps": sv["eps"], "chi": sv["chi"]})
    return bonds, sites, records
