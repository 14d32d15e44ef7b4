"""Two-site variational sweep over a block MPS (Sec. 4.3, in two-site form).

The paper's ground-state routine connects <psi|H|psi>, then for each site
prepares the effective Hamiltonian (everything contracted except the active
tensor), minimises it with the iterative eigensolver and moves on; real runs
sweep back and forth.  The two-site form used here optimises the pair of
sites (j, j+1) and splits the result with the truncated SVD.

One sweep = a right pass over bonds j = 1..L-1 followed by a left pass over
j = L-1..1, starting from a right-canonical state:
  right pass: theta = A_j A_{j+1}; lowest eigenpair; A_j = U, A_{j+1} = S V^+;
              L_j = update of L_{j-1} through site j.
  left pass:  theta = A_j A_{j+1}; lowest eigenpair; A_j = U S, A_{j+1} = V^+;
              R_{j+1} = update of R_{j+2} through site j+1.
Environments: L_0 selects MPO index 3 (the identity-so-far row), R_{L+1}
selects index 0; L_j[a', w, a] (bra index first) and R_j[b', u, b].
"""
from __future__ import annotations

import numpy as np

from . import heff as _heff
from . import lanczos as _lanczos
from . import svd as _svd
from .blocks import flatten, theta_keys, unflatten
from .model import MPO_LEFT, MPO_RIGHT


# ---------------------------------------------------------------------------
# canonical form
# ---------------------------------------------------------------------------

def right_canonicalise(bonds, sites, d):
    """Right-canonicalise sites L..2 by QR; normalise site 1.

    For each left sector of site j the (a) x (s, b) matrix M is factorised as
    M^+ = Q R (reduced QR); R's diagonal is made real positive; site j keeps
    Q^+ (a right isometry) and R^+ is absorbed into site j-1.  Sector
    dimensions shrink to the rank bound min(rows, cols) where needed.
    Returns new (bonds, sites) (inputs untouched).
    """
    bonds = [dict(b) for b in bonds]
    sites = [{k: v.copy() for k, v in s.items()} for s in sites]
    L = len(sites)
    for j in range(L, 1, -1):
        A = sites[j - 1]
        left, right = bonds[j - 1], bonds[j]
        newA, Rfac, newleft = {}, {}, {}
        for q in left:
            cols = [(s, q + s) for s in range(d) if (q, s) in A]
            if not cols:
                continue
            M = np.concatenate([A[(q, s)] for (s, _) in cols], axis=1)
            Q, R = np.linalg.qr(M.conj().T, mode="reduced")
            ph = np.diag(R).copy()
            ph = np.where(np.abs(ph) > 0, ph / np.abs(ph), 1.0)
            Q = Q * ph[None, :]
            R = ph.conj()[:, None] * R
            k = Q.shape[1]
            newleft[q] = k
            Bq = Q.conj().T  # (k, cols)
            co = 0
            for (s, qb) in cols:
                w = right[qb]
                newA[(q, s)] = Bq[:, co:co + w].copy()
                co += w
            Rfac[q] = R.conj().T  # (rows, k): M = R^+ Q^+
        sites[j - 1] = newA
        bonds[j - 1] = dict(sorted(newleft.items()))
        prev = sites[j - 2]
        for key in list(prev):
            qp, s = key
            qr = qp + s
            if qr in Rfac:
                prev[key] = prev[key] @ Rfac[qr]
            else:
                del prev[key]
    # normalise site 1
    nrm = np.sqrt(sum(float(np.sum(np.abs(v) ** 2)) for v in sites[0].values()))
    sites[0] = {k: v / nrm for k, v in sites[0].items()}
    return bonds, sites


# ---------------------------------------------------------------------------
# environments (Sec. 4.3: everything of <psi|H|psi> except the active sites)
# ---------------------------------------------------------------------------

def left_boundary(bond0, qw):
    q = next(iter(bond0))
    return {(MPO_LEFT, q): np.ones((1, 1), dtype=complex)}


def right_boundary(bondL, qw):
    q = next(iter(bondL))
    return {(MPO_RIGHT, q): np.ones((1, 1), dtype=complex)}


def update_left(Lprev, A, W, qw, d, bond_prev, bond_new):
    """L_j[a', w', a] = sum conj(A[c', s', a']) L_{j-1}[c', w, c] W[w, w', s', s] A[c, s, a]."""
    D = len(qw)
    # X[w; c', s, a] = L_{j-1}[c', w, c] A[c, s, a]
    X = {}
    for (w, qc), lblk in Lprev.items():
        for s in range(d):
            ablk = A.get((qc, s))
            if ablk is None:
                continue
            X[(w, qc + qw[w], s)] = lblk @ ablk  # rows c' (q = qc+qw[w]), cols a (q = qc+s)
    # Y[w'; c', s', a] = sum_{w, s} W[w, w', s', s] X[w; c', s, a]
    Y = {}
    for (w, qcp, s), x in X.items():
        for wp in range(D):
            for sp in range(d):
                c = W[w, wp, sp, s]
                if c == 0.0:
                    continue
                key = (wp, qcp, sp)
                Y[key] = Y[key] + c * x if key in Y else c * x
    # L_j[w'; a', a] = sum_{c', s'} conj(A[c', s', a'])^T Y[w'; c', s', a]
    out = {}
    for (wp, qcp, sp), y in Y.items():
        ablk = A.get((qcp, sp))
        if ablk is None:
            continue
        qa = qcp + sp - qw[wp]  # ket sector of the new block (charge rule)
        key = (wp, qa)
        contrib = ablk.conj().T @ y
        out[key] = out[key] + contrib if key in out else contrib
    return {k: out[k] for k in sorted(out, key=lambda t: (t[1], t[0]))
            if k[1] in bond_new and (k[1] + qw[k[0]]) in bond_new}


def update_right(Rnext, B, W, qw, d, bond_new, bond_next):
    """R_j[b', u, b] = sum conj(B[b', s', c']) W[u, u', s', s] R_{j+1}[c', u', c] B[b, s, c]."""
    D = len(qw)
    # X[u'; b, s, c'] = B[b, s, c] R_{j+1}[c', u', c]^T
    X = {}
    for (qb, s), bblk in B.items():
        qc = qb + s
        for up in range(D):
            rblk = Rnext.get((up, qc))
            if rblk is None:
                continue
            X[(up, qb, s)] = bblk @ rblk.T  # rows b (qb), cols c' (qc + qw[up])
    # Y[u; b, s', c'] = sum_{u', s} W[u, u', s', s] X[u'; b, s, c']
    Y = {}
    for (up, qb, s), x in X.items():
        for u in range(D):
            for sp in range(d):
                c = W[u, up, sp, s]
                if c == 0.0:
                    continue
                key = (u, qb, sp)
                Y[key] = Y[key] + c * x if key in Y else c * x
    # R_j[u; b', b] = sum_{s', c'} conj(B[b', s', c']) Y[u; b, s', c']^T
    out = {}
    for (u, qb, sp), y in Y.items():
        qbp = qb + qw[u]
        bblk = B.get((qbp, sp))
        if bblk is None:
            continue
        key = (u, qb)
        contrib = bblk.conj() @ y.T
        out[key] = out[key] + contrib if key in out else contrib
    return {k: out[k] for k in sorted(out, key=lambda t: (t[1], t[0]))
            if k[1] in bond_new and (k[1] + qw[k[0]]) in bond_new}


def form_theta(A, B, left, right, d):
    """theta[a, s1, s2, b] = sum_c A[a, s1, c] B[c, s2, b] (block products)."""
    th = {}
    for (qa, s1, s2) in theta_keys(left, right, d):
        a = A.get((qa, s1))
        b = B.get((qa + s1, s2))
        if a is None or b is None:
            th[(qa, s1, s2)] = np.zeros((left[qa], right[qa + s1 + s2]), dtype=complex)
        else:
            th[(qa, s1, s2)] = a @ b
    return th


def build_right_envs(bonds, sites, W_list, qw, d):
    L = len(sites)
    R = [None] * (L + 2)
    R[L + 1] = right_boundary(bonds[L], qw)
    for j in range(L, 2, -1):
        R[j] = update_right(R[j + 1], sites[j - 1], W_list[j - 1], qw, d, bonds[j - 1], bonds[j])
    return R


# ---------------------------------------------------------------------------
# sweep
# ---------------------------------------------------------------------------

def optimise_bond(Lenv, W1, W2, Renv, theta, left, right, qw, d, lanczos_steps, tol,
                  matvec_noise=None):
    keys = theta_keys(left, right, d)

    def mv(x):
        th = unflatten(x, theta, keys)
        y = _heff.heff2_block(Lenv, W1, W2, Renv, th, left, right, qw, d)
        return flatten(y, keys)

    res = _lanczos.lanczos_ground(mv, flatten(theta, keys), kmax=lanczos_steps, tol=tol)
    res["theta"] = unflatten(res["psi"], theta, keys)
    return res


def sweep(bonds, sites, W_list, qw, d, chi_max, lanczos_steps=20, lanczos_tol=1e-12,
          trunc=None, envs=None, log=None):
    """One full sweep (right pass then left pass) on a right-canonical MPS.

    Returns (bonds, sites, envs, records); records holds one dict per bond
    update (pass, j, E, E_ritz, residual, steps, eps, chi, bond dims).
    `trunc` = dict(a, r, e, kind) of the other truncation rules.
    """
    trunc = dict(trunc or {})
    L = len(sites)
    bonds = [dict(b) for b in bonds]
    sites = [dict(s) for s in sites]
    if envs is None:
        Lenvs = [None] * (L + 1)
        Lenvs[0] = left_boundary(bonds[0], qw)
        Renvs = build_right_envs(bonds, sites, W_list, qw, d)
    else:
        Lenvs, Renvs = envs
    records = []
    for direction in ("right", "left"):
        js = range(1, L) if direction == "right" else range(L - 1, 0, -1)
        for j in js:
            left, right = bonds[j - 1], bonds[j + 1]
            theta = form_theta(sites[j - 1], sites[j], left, right, d)
            res = optimise_bond(Lenvs[j - 1], W_list[j - 1], W_list[j], Renvs[j + 2], theta,
                                left, right, qw, d, lanczos_steps, lanczos_tol)
            sv = _svd.svd_truncate(res["theta"], left, right, d, chi_max,
                                   absorb=direction, **trunc)
            sites[j - 1], sites[j] = sv["A"], sv["B"]
            bonds[j] = sv["bond"]
            if direction == "right":
                Lenvs[j] = update_left(Lenvs[j - 1], sites[j - 1], W_list[j - 1], qw, d,
                                       bonds[j - 1], bonds[j])
            else:
                Renvs[j + 1] = update_right(Renvs[j + 2], sites[j], W_list[j], qw, d,
                                            bonds[j], bonds[j + 1])
            rec = {"pass": direction, "j": j, "E": res["E"], "E_ritz": res["E_ritz"],
                   "residual": res["residual"], "steps": res["steps"], "eps": sv["eps"],
                   "chi": sv["chi"], "bond": dict(sv["bond"]),
                   "lambdas": np.sort(np.concatenate(list(sv["lambdas"].values())))[::-1]}
            records.append(rec)
            if log is not None:
                log(rec)
    return bonds, sites, (Lenvs, Renvs), records


# ---------------------------------------------------------------------------
# whole-network expectation values (the MPS-MPO-MPS network of Sec. 4.3)
# ---------------------------------------------------------------------------

def expectation(bonds, sites, W_list, qw, d):
    """<psi|H|psi> / <psi|psi> by contracting the full network left to right."""
    L = len(sites)
    Le = left_boundary(bonds[0], qw)
    for j in range(1, L + 1):
        Le = update_left(Le, sites[j - 1], W_list[j - 1], qw, d, bonds[j - 1], bonds[j])
    qN = next(iter(bonds[L]))
    num = Le[(MPO_RIGHT, qN)][0, 0]
    return float(np.real(num)) / norm2(bonds, sites, d)


def norm2(bonds, sites, d):
    """<psi|psi> via the transfer matrices."""
    E = {q: np.ones((1, 1), dtype=complex) for q in bonds[0]}
    for j, A in enumerate(sites, start=1):
        new = {}
        for (q, s), blk in A.items():
            if q not in E:
                continue
            c = blk.conj().T @ E[q] @ blk
            qr = q + s
            new[qr] = new[qr] + c if qr in new else c
        E = new
    return float(np.real(sum(np.trace(v) for v in E.values())))


def site_densities(bonds, sites, d):
    """<n_j> for j = 1..L of a normalised MPS (used as an invariant check)."""
    L = len(sites)
    out = []
    for target in range(1, L + 1):
        E = {q: np.ones((1, 1), dtype=complex) for q in bonds[0]}
        for j, A in enumerate(sites, start=1):
            new = {}
            for (q, s), blk in A.items():
                if q not in E:
                    continue
                wgt = float(s) if j == target else 1.0
                c = wgt * (blk.conj().T @ E[q] @ blk)
                qr = q + s
                new[qr] = new[qr] + c if qr in new else c
            E = new
        out.append(float(np.real(sum(np.trace(v) for v in E.values()))))
    nrm = norm2(bonds, sites, d)
    return [x / nrm for x in out]


def run_dmrg(spec_L, spec_N, nmax, J, U, mu, chi, seed, sweeps, lanczos_steps=20,
             trunc=None, random_mps=None, W_list=None, qw=None):
    """Convenience driver: seeded random MPS -> right-canonical -> `sweeps` sweeps."""
    from .model import bh_mpo
    d = nmax + 1
    if W_list is None:
        W, qw = bh_mpo(nmax, J, U, mu)
        W_list = [W] * spec_L
    bonds, sites = random_mps(spec_L, spec_N, nmax, chi, seed)
    bonds, sites = right_canonicalise(bonds, sites, d)
    all_records = []
    envs = None
    for _ in range(sweeps):
        bonds, sites, envs, rec = sweep(bonds, sites, W_list, qw, d, chi, lanczos_steps,
                                        trunc=trunc, envs=envs)
        all_records.append(rec)
    return bonds, sites, all_records
