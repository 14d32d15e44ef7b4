"""U(1) block tensors <-> dense arrays (appendix A.1.1, symmetric nodes).

A block tensor keeps only the elements whose incoming charges sum to the
outgoing charge; the dense form places every block at the index range of
its sectors and is zero elsewhere.  Dense forms are the definition the block
code is checked against.
"""
from __future__ import annotations

import numpy as np


def offsets(bond: dict[int, int]) -> dict[int, int]:
    """Start of each sector in the dense bond index (ascending q)."""
    out, pos = {}, 0
    for q in sorted(bond):
        out[q] = pos
        pos += bond[q]
    return out


def dim(bond) -> int:
    return int(sum(bond.values()))


def site_to_dense(A, left, right, d):
    ol, orr = offsets(left), offsets(right)
    out = np.zeros((dim(left), d, dim(right)), dtype=complex)
    for (q, s), blk in A.items():
        out[ol[q]:ol[q] + left[q], s, orr[q + s]:orr[q + s] + right[q + s]] = blk
    return out


def theta_to_dense(th, left, right, d):
    ol, orr = offsets(left), offsets(right)
    out = np.zeros((dim(left), d, d, dim(right)), dtype=complex)
    for (q, s1, s2), blk in th.items():
        qb = q + s1 + s2
        out[ol[q]:ol[q] + left[q], s1, s2, orr[qb]:orr[qb] + right[qb]] = blk
    return out


def theta_from_dense(X, left, right, d):
    """Read the allowed blocks out of a dense [a, s1, s2, b] array."""
    ol, orr = offsets(left), offsets(right)
    out = {}
    for q in left:
        for s1 in range(d):
            for s2 in range(d):
                qb = q + s1 + s2
                if qb in right:
                    out[(q, s1, s2)] = X[ol[q]:ol[q] + left[q], s1, s2,
                                         orr[qb]:orr[qb] + right[qb]].copy()
    return out


def theta_forbidden_norm(X, left, right, d):
    """2-norm of the entries of a dense theta outside every allowed block."""
    mask = np.ones(X.shape, dtype=bool)
    ol, orr = offsets(left), offsets(right)
    for q in left:
        for s1 in range(d):
            for s2 in range(d):
                qb = q + s1 + s2
                if qb in right:
                    mask[ol[q]:ol[q] + left[q], s1, s2, orr[qb]:orr[qb] + right[qb]] = False
    return float(np.linalg.norm(X[mask]))


def env_to_dense(E, bond, qw):
    """{(w, q): (dim(q+qw[w]), dim(q))} -> dense [a', w, a]."""
    o = offsets(bond)
    D = len(qw)
    out = np.zeros((dim(bond), D, dim(bond)), dtype=complex)
    for (w, q), blk in E.items():
        qp = q + qw[w]
        out[o[qp]:o[qp] + bond[qp], w, o[q]:o[q] + bond[q]] = blk
    return out


def env_from_dense(X, bond, qw):
    o = offsets(bond)
    out = {}
    for q in bond:
        for w in range(len(qw)):
            qp = q + qw[w]
            if qp in bond:
                out[(w, q)] = X[o[qp]:o[qp] + bond[qp], w, o[q]:o[q] + bond[q]].copy()
    return out


def theta_keys(left, right, d):
    return [(q, s1, s2) for q in left for s1 in range(d) for s2 in range(d)
            if (q + s1 + s2) in right]


def flatten(blocks, keys) -> np.ndarray:
    """Concatenate blocks (row-major) in the given key order."""
    if not keys:
        return np.zeros(0, dtype=complex)
    return np.concatenate([blocks[k].reshape(-1) for k in keys])


def unflatten(vec, like, keys):
    out, pos = {}, 0
    for k in keys:
        n = like[k].size
        out[k] = vec[pos:pos + n].reshape(like[k].shape)
        pos += n
    assert pos == vec.size
    return out
