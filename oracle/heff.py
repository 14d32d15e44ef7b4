"""Two-site effective Hamiltonian applied to a vector theta.

Definition (the H_eff contractor of Sec. 4.2, in two-site form: the network
of left environment, two MPO tensors and right environment joined to theta):

    y[a', s1', s2', b'] = sum L[a', w, a] W1[w, v, s1', s1] W2[v, u, s2', s2]
                              R[b', u, b] theta[a, s1, s2, b]

`heff2_dense` is that sum written as one einsum over dense arrays.
`heff2_block` evaluates the same sum block by block with U(1) sectors, as a
sequence of pairwise contractions (appendix B.1.1: reorder so the contracted
index is shared, then a matrix product), contracting theta first with L,
then W1, then W2, then R (the cheap order for a chain, appendix B.1.1 on the
choice of contraction order).
"""
from __future__ import annotations

import numpy as np


def heff2_dense(Ld, W1, W2, Rd, thd):
    """Dense definition.  Ld: [a', w, a], Rd: [b', u, b], thd: [a, s1, s2, b]."""
    spec = 'xwa,wvSs,vuTt,yub,astb->xSTy'
    # a pairwise path with no cap on intermediate size (numpy's default cap
    # would leave a 10-index naive sum)
    path = np.einsum_path(spec, Ld, W1, W2, Rd, thd, optimize=('greedy', 1e15))[0]
    return np.einsum(spec, Ld, W1, W2, Rd, thd, optimize=path)


def heff2_block(L, W1, W2, R, theta, left, right, qw, d, out_sectors=None):
    """Block-sparse H_eff . theta (complex128), same sum as `heff2_dense`.

    L: {(w, q_a): (dim(q_a+qw[w]), dim(q_a))}; R likewise on the right bond;
    theta: {(q_a, s1, s2): (dim(q_a), dim(q_b))}.  Returns y with theta's keys.
    With `out_sectors` (a set of output charges q_a'), only output blocks in
    those sectors are computed (the others are returned as zeros): every
    term of a computed block is still included, so those blocks are exact.
    """
    D = len(qw)
    # stage 1: T1[w; a', s1, s2, b] = sum_a L[a', w, a] theta[a, s1, s2, b]
    T1 = {}
    for (qa, s1, s2), th in theta.items():
        for w in range(D):
            blk = L.get((w, qa))
            if blk is None:
                continue
            if out_sectors is not None and (qa + qw[w]) not in out_sectors:
                continue
            T1[(w, qa + qw[w], s1, s2)] = blk @ th
    # stage 2: T2[v; a', s1', s2, b] = sum_{w, s1} W1[w, v, s1', s1] T1[w; a', s1, s2, b]
    T2 = {}
    for (w, qap, s1, s2), t in T1.items():
        for v in range(D):
            for s1p in range(d):
                c = W1[w, v, s1p, s1]
                if c == 0.0:
                    continue
                key = (v, qap, s1p, s2)
                T2[key] = T2[key] + c * t if key in T2 else c * t
    # stage 3: T3[u; a', s1', s2', b] = sum_{v, s2} W2[v, u, s2', s2] T2[v; a', s1', s2, b]
    T3 = {}
    for (v, qap, s1p, s2), t in T2.items():
        for u in range(D):
            for s2p in range(d):
                c = W2[v, u, s2p, s2]
                if c == 0.0:
                    continue
                key = (u, qap, s1p, s2p)
                T3[key] = T3[key] + c * t if key in T3 else c * t
    # stage 4: y[a', s1', s2', b'] = sum_{u, b} T3[u; a', s1', s2', b] R[b', u, b]
    y = {k: np.zeros_like(v) for k, v in theta.items()}
    for (u, qap, s1p, s2p), t in T3.items():
        key = (qap, s1p, s2p)
        if key not in y:
            continue  # the output block is outside theta's allowed set
        qbp = qap + s1p + s2p
        rblk = R.get((u, qbp - qw[u]))
        if rblk is None:
            continue
        y[key] += t @ rblk.T
    return y


def heff2_matrix_dense(Ld, W1, W2, Rd):
    """Dense H_eff as a matrix on the flattened [a, s1, s2, b] index (small sizes)."""
    Da, D, _ = Ld.shape
    d = W1.shape[2]
    Db = Rd.shape[0]
    M = np.einsum('xwa,wvSs,vuTt,yub->xSTyastb', Ld, W1, W2, Rd, optimize=True)
    n = Da * d * d * Db
    return M.reshape(n, n)


def heff1_block(L, W, R, A, qw, d):
    """One-site form of the contractor (Sec. 4.2, Listing lis:varmincontract):
    y[a', s', b'] = sum L[a', w, a] W[w, u, s', s] R[b', u, b] A[a, s, b].

    L: {(w, q_a): (dim(q_a+qw[w]), dim(q_a))}; R likewise on the right bond;
    A: {(q_a, s): (dim(q_a), dim(q_a+s))}.  Returns y with A's keys.
    """
    D = len(qw)
    # T1[w; a', s, b] = sum_a L[a', w, a] A[a, s, b]  (key: w, q_a', s)
    T1 = {}
    for (qa, s), a in A.items():
        for w in range(D):
            blk = L.get((w, qa))
            if blk is not None:
                T1[(w, qa + qw[w], s)] = blk @ a
    # T2[u; a', s', b] = sum_{w, s} W[w, u, s', s] T1[w; a', s, b]
    T2 = {}
    for (w, qap, s), t in T1.items():
        for u in range(D):
            for sp in range(d):
                c = W[w, u, sp, s]
                if c == 0.0:
                    continue
                key = (u, qap, sp)
                T2[key] = T2[key] + c * t if key in T2 else c * t
    # y[a', s', b'] = sum_{u, b} T2[u; a', s', b] R[b', u, b]; b = a' + s' - qw[u]
    y = {k: np.zeros_like(v) for k, v in A.items()}
    for (u, qap, sp), t in T2.items():
        key = (qap, sp)
        if key not in y:
            continue
        rblk = R.get((u, qap + sp - qw[u]))
        if rblk is None:
            continue
        y[key] += t @ rblk.T
    return y
