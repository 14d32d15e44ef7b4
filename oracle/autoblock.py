"""Automatic blocking of a matrix without known symmetries (the library's
auto-blocking mode, described with Fig. fig:autoblocking and Table
tab:tebdtimes): entries of magnitude at most a tolerance are set to zero,
rows and columns are reordered so that the matrix becomes block diagonal
(its blocks are the connected components of the bipartite graph joining row
i to column j when entry (i, j) is nonzero), and every block is decomposed
on its own; the singular values of all blocks together, cut by the
truncation rules of appendix B.1.2, give the truncated SVD of the matrix.

Test infrastructure (an oracle): plain NumPy, written from this description.
"""
from __future__ import annotations

import numpy as np

from . import svd as _svd


def components(mask):
    """Blocks of a boolean m x n pattern: a list of (rows, cols) index arrays,
    ordered by their smallest row; rows or columns with no nonzero entry
    belong to no block."""
    m, n = mask.shape
    seen_r = np.zeros(m, bool)
    seen_c = np.zeros(n, bool)
    out = []
    for start in range(m):
        if seen_r[start] or not mask[start].any():
            continue
        rows, cols = [start], []
        seen_r[start] = True
        stack = [("r", start)]
        while stack:
            kind, i = stack.pop()
            if kind == "r":
                for j in np.nonzero(mask[i])[0]:
                    if not seen_c[j]:
                        seen_c[j] = True
                        cols.append(int(j))
                        stack.append(("c", int(j)))
            else:
                for r in np.nonzero(mask[:, i])[0]:
                    if not seen_r[r]:
                        seen_r[r] = True
                        rows.append(int(r))
                        stack.append(("r", int(r)))
        out.append((np.array(sorted(rows)), np.array(sorted(cols))))
    return out


def auto_block_svd(M, tol, chi_max, a=-1.0, r=-1.0, e=-1.0, kind=_svd.TYPE_2NORM):
    """Truncated SVD through automatic blocking.  Returns dict(lam (kept,
    descending), eps, chi, blocks, approx (the truncated matrix U S V^+))."""
    M = np.asarray(M, dtype=complex)
    Z = np.where(np.abs(M) > tol, M, 0.0)
    blocks = components(np.abs(Z) > 0)
    dec = []
    pool = []
    for b, (rows, cols) in enumerate(blocks):
        U, S, Vh = np.linalg.svd(Z[np.ix_(rows, cols)], full_matrices=False)
        dec.append((rows, cols, U, S, Vh))
        pool += [(s, b, k) for k, s in enumerate(S)]
    pool.sort(key=lambda x: (-x[0], x[1], x[2]))
    lam_all = np.array([p[0] for p in pool])
    chi = _svd.select_chi(lam_all, chi_max, a, r, e, kind) if len(pool) else 0
    eps = _svd.trunc_error(lam_all[chi:], kind) if len(pool) else 0.0
    approx = np.zeros_like(Z)
    for s, b, k in pool[:chi]:
        rows, cols, U, S, Vh = dec[b]
        approx[np.ix_(rows, cols)] += S[k] * np.outer(U[:, k], Vh[k])
    return {"lam": lam_all[:chi], "eps": eps, "chi": chi, "blocks": blocks, "approx": approx,
            "all_lam": lam_all}
