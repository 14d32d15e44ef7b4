"""Truncated SVD of a two-site vector with U(1) sectors (appendix B.1.2).

The paper's SVD splits a node into U S V^+ with the row legs going to U and
the column legs to V^+, singular values in decreasing order.  Truncation
keeps a bond dimension chi decided by four rules; when several are active
the one giving the smallest chi wins:
  (1) chi <= chi_max;
  (2) absolute: discard lambda_i < a;
  (3) relative: discard lambda_i / lambda_0 < r;
  (4) error: discard the largest number of values whose truncation error
      stays below e.
The truncation error is the 2-norm of the discarded values by default (Eq.
trunc_err; the sum of squares or the 1-norm on request).

Readings: the discarded set is everything after the chi largest values
(0-based indices i >= chi, with lambda_0 the largest); the inequalities are
strict exactly as stated; at least one value is always kept; with U(1)
sectors all sectors' values are pooled and sorted together (ties: smaller
middle charge first, then smaller in-sector index); the kept values are
renormalised to unit 2-norm.
"""
from __future__ import annotations

import math

import numpy as np

TYPE_2NORM, TYPE_SUMSQ, TYPE_1NORM = 0, 1, 2


def trunc_error(discarded: np.ndarray, kind: int = TYPE_2NORM) -> float:
    if kind == TYPE_2NORM:
        return math.sqrt(float(np.sum(discarded ** 2)))
    if kind == TYPE_SUMSQ:
        return float(np.sum(discarded ** 2))
    if kind == TYPE_1NORM:
        return float(np.sum(np.abs(discarded)))
    raise ValueError(kind)


def select_chi(lams_desc: np.ndarray, chi_max: int, a: float = -1.0, r: float = -1.0,
               e: float = -1.0, kind: int = TYPE_2NORM) -> int:
    """Number of values kept from a descending spectrum under the four rules."""
    n = len(lams_desc)
    if n == 0:
        return 0
    chi = min(chi_max, n)
    if a > 0:
        chi = min(chi, int(np.sum(lams_desc >= a)))
    if r > 0:
        chi = min(chi, int(np.sum(lams_desc / lams_desc[0] >= r)))
    if e > 0:
        # smallest k whose discarded tail has error < e
        best = n
        for k in range(n, -1, -1):
            if trunc_error(lams_desc[k:], kind) < e:
                best = k
            else:
                break
        chi = min(chi, best)
    return max(chi, 1)


def theta_sectors(left, right, d):
    """Middle charges m with their row list [(s1, q_a)] and column list [(s2, q_b)]."""
    ms = sorted({qa + s1 for qa in left for s1 in range(d)} &
                {qb - s2 for qb in right for s2 in range(d)})
    out = []
    for m in ms:
        rows = [(s1, m - s1) for s1 in range(d) if (m - s1) in left]
        cols = [(s2, m + s2) for s2 in range(d) if (m + s2) in right]
        out.append((m, rows, cols))
    return out


def svd_truncate(theta, left, right, d, chi_max, a=-1.0, r=-1.0, e=-1.0,
                 kind=TYPE_2NORM, absorb="right", renormalise=True):
    """Split theta[a, s1, s2, b] into A[a, s1, c] and B[c, s2, b].

    absorb="right": A = U, B = S V^+ ; absorb="left": A = U S, B = V^+.
    Returns dict(A, B, bond, lambdas (per sector, kept, renormalised),
    eps, lambda0, chi, all_lambdas (descending pooled)).
    """
    secs = theta_sectors(left, right, d)
    dec = {}
    pool = []
    for (m, rows, cols) in secs:
        rdim = [left[qa] for (_, qa) in rows]
        cdim = [right[qb] for (_, qb) in cols]
        M = np.zeros((sum(rdim), sum(cdim)), dtype=complex)
        ro = 0
        for (s1, qa), rd in zip(rows, rdim):
            co = 0
            for (s2, qb), cd in zip(cols, cdim):
                M[ro:ro + rd, co:co + cd] = theta[(qa, s1, s2)]
                co += cd
            ro += rd
        U, S, Vh = np.linalg.svd(M, full_matrices=False)
        dec[m] = (rows, cols, rdim, cdim, U, S, Vh)
        for i, lam in enumerate(S):
            pool.append((float(lam), m, i))
    pool.sort(key=lambda t: (-t[0], t[1], t[2]))
    lams = np.array([p[0] for p in pool])
    chi = select_chi(lams, chi_max, a, r, e, kind)
    kept = {m: 0 for m in dec}
    for (_, m, _) in pool[:chi]:
        kept[m] += 1
    eps = trunc_error(lams[chi:], kind)
    norm_kept = math.sqrt(float(np.sum(lams[:chi] ** 2)))
    scale = 1.0 / norm_kept if renormalise else 1.0
    A, B, bond, lam_out = {}, {}, {}, {}
    for m, (rows, cols, rdim, cdim, U, S, Vh) in dec.items():
        k = kept[m]
        if k == 0:
            continue
        bond[m] = k
        s = S[:k] * scale
        lam_out[m] = s
        Uk = U[:, :k]
        Vk = Vh[:k, :]
        if absorb == "right":
            left_f, right_f = Uk, s[:, None] * Vk
        else:
            left_f, right_f = Uk * s[None, :], Vk
        ro = 0
        for (s1, qa), rd in zip(rows, rdim):
            A[(qa, s1)] = left_f[ro:ro + rd, :].copy()
            ro += rd
        co = 0
        for (s2, qb), cd in zip(cols, cdim):
            B[(m, s2)] = right_f[:, co:co + cd].copy()
            co += cd
    return {"A": A, "B": B, "bond": dict(sorted(bond.items())), "lambdas": lam_out,
            "eps": eps, "lambda0": float(lams[0]) if len(lams) else 0.0, "chi": chi,
            "all_lambdas": lams}
