"""Algorithmic FLOP count F_alg of one block-sparse two-site H_eff . theta.

Counting rule (a complex multiply-add is 8 real flops; a real scalar times a
complex element added into a sum is 4):
  * MPO product terms: for an output block (q_a', s1', s2') and right MPO
    index u, the slab T3[u; a', s1', s2', b] = sum over (w, s1, s2) of
    c * T1[w; a', s1, s2, b] with c = sum_v W1[w, v, s1', s1] W2[v, u, s2', s2].
    A (w, s1, s2) term exists when c != 0 and the theta block
    (q_a' - qw[w], s1, s2) exists.  A slab is live when it has a term, its
    output block is an allowed theta block and R holds block (u, q_b' - qw[u]).
  * step 1: every T1[w; q_a', s1, s2] slab used by a live slab costs
    8 * dim(q_a') * dim(q_a) * dim(q_b);
  * MPO: every term of a live slab costs 4 * dim(q_a') * dim(q_b);
  * step 4: every live slab costs 8 * dim(q_a') * dim(q_b) * dim(q_b').
This is written out independently of the GPU planner; the two counts must be
equal integers.
"""
from __future__ import annotations


def heff2_flops(left, right, d, qw, W1, W2):
    D = len(qw)
    theta = {(qa, s1, s2) for qa in left for s1 in range(d) for s2 in range(d)
             if qa + s1 + s2 in right}
    # the two-site coefficients c[w][u][s1'][s2'][s1][s2] as plain floats
    W1l, W2l = W1.tolist(), W2.tolist()
    coef = [[[[[[sum(W1l[w][v][s1p][s1] * W2l[v][u][s2p][s2] for v in range(D))
                 for s2 in range(d)] for s1 in range(d)] for s2p in range(d)]
              for s1p in range(d)] for u in range(D)] for w in range(D)]
    live_t1 = set()
    f_mpo = 0
    f_step4 = 0
    for (qap, s1p, s2p) in sorted(theta):
        qbp = qap + s1p + s2p
        for u in range(D):
            qb = qbp - qw[u]
            if qb not in right:
                continue
            terms = []
            for w in range(D):
                qa = qap - qw[w]
                for s1 in range(d):
                    for s2 in range(d):
                        if (qa, s1, s2) not in theta:
                            continue
                        c = coef[w][u][s1p][s2p][s1][s2]
                        if c != 0.0:
                            terms.append((w, qa, s1, s2))
            if not terms:
                continue
            f_mpo += 4 * len(terms) * left[qap] * right[qb]
            f_step4 += 8 * left[qap] * right[qb] * right[qbp]
            for (w, qa, s1, s2) in terms:
                live_t1.add((w, qa, s1, s2))
    f_step1 = 0
    for (w, qa, s1, s2) in live_t1:
        qap = qa + qw[w]
        qb = qa + s1 + s2
        f_step1 += 8 * left[qap] * left[qa] * right[qb]
    return {"step1": f_step1, "mpo": f_mpo, "step4": f_step4,
            "total": f_step1 + f_mpo + f_step4}
