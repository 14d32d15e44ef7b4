"""GPU one-site H_eff (tnt_heff1_apply) against the one-site oracle.

Environments and site tensors of a seeded right-canonicalised chain (the
oracle's environment updates), FP64: normwise relative error <= 1e-12, at a
small chain, a ragged multi-sector bond and the chi = 256 middle bond.
Mismatched descriptors are refused.
"""
import numpy as np
import pytest

import synth
from oracle import dmrg as odmrg
from oracle import heff as oheff
from oracle import model

pytestmark = pytest.mark.gpu


def site_inputs(L, N, nmax, chi, j, seed, U=2.5):
    d = nmax + 1
    W, qw = model.bh_mpo(nmax, 1.0, U, 0.3)
    bonds, sites = synth.random_mps(L, N, nmax, chi, seed)
    Lenv = odmrg.left_boundary(bonds[0], qw)
    for k in range(1, j):
        Lenv = odmrg.update_left(Lenv, sites[k - 1], W, qw, d, bonds[k - 1], bonds[k])
    Renv = odmrg.right_boundary(bonds[L], qw)
    for k in range(L, j, -1):
        Renv = odmrg.update_right(Renv, sites[k - 1], W, qw, d, bonds[k - 1], bonds[k])
    return W, qw, d, Lenv, Renv, sites[j - 1]


@pytest.mark.parametrize("L,N,nmax,chi,j,seed", [(6, 4, 2, 9, 3, 1), (10, 7, 3, 40, 5, 2),
                                                 (16, 16, 4, 256, 8, 3)])
def test_heff1_matches_oracle(tnt, L, N, nmax, chi, j, seed):
    from paper_1610_02244_amd import binding as B
    print(f"[heff1] L={L} chi={chi} site={j}", flush=True)
    W, qw, d, Lenv, Renv, A = site_inputs(L, N, nmax, chi, j, seed)
    Wg, qg = tnt.bose_hubbard_mpo(nmax, 1.0, 2.5, 0.3)
    mpo = B.Mpo(Wg, qg)
    Ld, Rd, Ad = tnt.env(Lenv, qg), tnt.env(Renv, qg), tnt.site(A)
    out = tnt.site_like(Ad)
    tnt.heff1_apply(Ld, mpo, Rd, Ad, out)
    got = tnt.download(out)
    ref = oheff.heff1_block(Lenv, W, Renv, A, qw, d)
    num = np.sqrt(sum(np.linalg.norm(got[k] - ref[k]) ** 2 for k in ref))
    den = np.sqrt(sum(np.linalg.norm(ref[k]) ** 2 for k in ref))
    print(f"  rel err {num / den:.2e}")
    assert num <= 1e-12 * den


def test_heff1_rejects_mismatched_output(tnt):
    from paper_1610_02244_amd import binding as B
    W, qw, d, Lenv, Renv, A = site_inputs(6, 4, 2, 9, 3, 1)
    Wg, qg = tnt.bose_hubbard_mpo(2, 1.0, 2.5, 0.3)
    mpo = B.Mpo(Wg, qg)
    Ad = tnt.site(A)
    # an output whose block set lacks one of A's blocks
    A2 = dict(A)
    A2.pop(sorted(A2)[0])
    with pytest.raises(B.TntError) as ei:
        tnt.heff1_apply(tnt.env(Lenv, qg), mpo, tnt.env(Renv, qg), Ad, tnt.site(A2))
    assert ei.value.code == -2  # TNT_E_SHAPE


def test_heff1_rejects_non_fp64_or_null_planes(tnt):
    """Environments described as FP32 (or with a missing plane) are refused
    before anything runs: the contraction reads FP64 planes only."""
    from paper_1610_02244_amd import binding as B
    W, qw, d, Lenv, Renv, A = site_inputs(6, 4, 2, 9, 3, 1)
    Wg, qg = tnt.bose_hubbard_mpo(2, 1.0, 2.5, 0.3)
    mpo = B.Mpo(Wg, qg)
    Ad, od = tnt.site(A), tnt.site(A)
    for which in ("L", "R"):
        Ld, Rd = tnt.env(Lenv, qg), tnt.env(Renv, qg)
        (Ld if which == "L" else Rd).c.dtype = B.TNT_DT_F32
        with pytest.raises(B.TntError) as ei:
            tnt.heff1_apply(Ld, mpo, Rd, Ad, od)
        assert ei.value.code == -1  # TNT_E_ARG
    Ld, Rd = tnt.env(Lenv, qg), tnt.env(Renv, qg)
    Rd.c.im = None
    with pytest.raises(B.TntError) as ei:
        tnt.heff1_apply(Ld, mpo, Rd, Ad, od)
    assert ei.value.code == -1
    # the context stays usable
    tnt.heff1_apply(tnt.env(Lenv, qg), mpo, tnt.env(Renv, qg), Ad, od)
