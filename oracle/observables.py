"""Observables of a block MPS: the single-particle density matrix
rho_ij = <b^dagger_i b_j> and the densities <n_j> = rho_jj, the outputs of the
paper's ground-state example (Sec. 5, Fig. fig:ground_state_results).

Test infrastructure (an oracle): plain NumPy, written from the definition.
For a real single-site operator O with charge change dq (O_{s's} != 0 only
where s' - s = dq), C[i, j] = <psi| O^dagger_i O_j |psi> / <psi|psi>.  Every
pair is a separate contraction of the whole MPS-MPS network, left to right,
with the operators inserted at their sites; no intermediate is shared between
pairs.  With O = b this is rho_ij; its diagonal is <n_j>.
"""
from __future__ import annotations

import numpy as np


def _transfer(E, A, site_op, d):
    """E'[(qb', qk')] = sum A[(qb, s')]^H E[(qb, qk)] A[(qk, s)] <s'|op|s>."""
    out = {}
    for (qb, qk), e in E.items():
        for sp in range(d):
            Ab = A.get((qb, sp))
            if Ab is None:
                continue
            for s in range(d):
                coef = site_op[sp, s]
                if coef == 0.0:
                    continue
                Ak = A.get((qk, s))
                if Ak is None:
                    continue
                blk = coef * (Ab.conj().T @ e @ Ak)
                key = (qb + sp, qk + s)
                out[key] = out[key] + blk if key in out else blk
    return out


def _network(bonds, sites, d, ops):
    """<psi| prod_j ops[j] |psi> with ops[j] a d x d matrix (None = identity)."""
    q0 = next(iter(bonds[0]))
    E = {(q0, q0): np.ones((1, 1), dtype=complex)}
    I = np.eye(d)
    for j, A in enumerate(sites):
        E = _transfer(E, A, ops[j] if ops[j] is not None else I, d)
    return complex(sum(np.trace(v) for v in E.values()))


def correlation_matrix(bonds, sites, d, op, pairs=None):
    """C[i, j] = <O^dagger_i O_j> / <psi|psi> (0-based i, j) for a real
    operator matrix op[s', s] = <s'|O|s>; with `pairs`, only those (i, j)
    entries are computed (the rest stay zero)."""
    op = np.asarray(op, dtype=float)
    L = len(sites)
    nrm = _network(bonds, sites, d, [None] * L).real
    C = np.zeros((L, L), dtype=complex)
    todo = pairs if pairs is not None else [(i, j) for i in range(L) for j in range(L)]
    for i, j in todo:
        ops = [None] * L
        if i == j:
            ops[i] = op.T @ op
        else:
            ops[i] = op.T.copy()  # <s'|O^dagger|s> = O_{s s'} for a real O
            ops[j] = op
        C[i, j] = _network(bonds, sites, d, ops) / nrm
    return C


def annihilator(nmax: int) -> np.ndarray:
    """b on |n>, n = 0..nmax: b|n> = sqrt(n)|n-1>."""
    b = np.zeros((nmax + 1, nmax + 1))
    for n in range(1, nmax + 1):
        b[n - 1, n] = np.sqrt(n)
    return b
