"""Pin of the one-site H_eff oracle against the (separately pinned) two-site
one: for any site tensor B of site j+1, contracting H_eff2 . (A_j B_{j+1})
with conj(B_{j+1}) over (s2, b) gives H_eff1 . A_j with the right
environment R_{j+1} built from B (the definition of the environment update),
so a dropped term, a wrong charge or a transposed environment fails.  Also:
H_eff1 is Hermitian (<x, H y> = <H x, y>) on a right-canonical chain.
"""
import numpy as np
import pytest

import synth
from oracle import dmrg as odmrg
from oracle import heff as oheff
from oracle import model


@pytest.mark.parametrize("L,N,nmax,chi,j,seed", [(6, 4, 2, 9, 2, 1), (8, 5, 3, 12, 4, 2),
                                                 (5, 5, 2, 9, 1, 3)])
def test_heff1_from_heff2(L, N, nmax, chi, j, seed):
    d = nmax + 1
    W, qw = model.bh_mpo(nmax, 1.0, 2.5, 0.3)
    bonds, sites = synth.random_mps(L, N, nmax, chi, seed)
    bonds, sites = odmrg.right_canonicalise(bonds, sites, d)
    Ws = [W] * L
    R = odmrg.build_right_envs(bonds, sites, Ws, qw, d)
    Lenv = odmrg.left_boundary(bonds[0], qw)
    for k in range(1, j):
        Lenv = odmrg.update_left(Lenv, sites[k - 1], W, qw, d, bonds[k - 1], bonds[k])
    Rj2 = R[j + 2] if j + 2 <= L else odmrg.right_boundary(bonds[L], qw)
    Rj1 = odmrg.update_right(Rj2, sites[j], W, qw, d, bonds[j], bonds[j + 1])
    A, B = sites[j - 1], sites[j]
    y1 = oheff.heff1_block(Lenv, W, Rj1, A, qw, d)
    th = odmrg.form_theta(A, B, bonds[j - 1], bonds[j + 1], d)
    y2 = oheff.heff2_block(Lenv, W, W, Rj2, th, bonds[j - 1], bonds[j + 1], qw, d)
    z = {k: np.zeros_like(v) for k, v in A.items()}
    for (qa, s1, s2), blk in y2.items():
        Bb = B.get((qa + s1, s2))
        if Bb is not None and (qa, s1) in z:
            z[(qa, s1)] += blk @ Bb.conj().T
    for k in A:
        np.testing.assert_allclose(y1[k], z[k], atol=1e-12 * max(1.0, np.abs(z[k]).max()))
    # Hermitian
    rng = np.random.default_rng(seed)
    x = {k: rng.normal(size=v.shape) + 1j * rng.normal(size=v.shape) for k, v in A.items()}
    yv = {k: rng.normal(size=v.shape) + 1j * rng.normal(size=v.shape) for k, v in A.items()}
    Hx = oheff.heff1_block(Lenv, W, Rj1, x, qw, d)
    Hy = oheff.heff1_block(Lenv, W, Rj1, yv, qw, d)
    lhs = sum(np.vdot(x[k], Hy[k]) for k in A)
    rhs = sum(np.vdot(Hx[k], yv[k]) for k in A)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
