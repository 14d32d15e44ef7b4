"""Pins of the oracle's two-site H_eff . theta.

* The dense einsum equals P^+ H P theta, where P is the mixed-canonical
  embedding of the two-site space into the full Hilbert space and H is the
  Kronecker-product Hamiltonian (no MPO, no environments involved).
* The block evaluation equals the dense einsum on embedded inputs.
* H_eff is Hermitian for Hermitian-paired environments; the output stays in
  the allowed U(1) blocks (particle number conservation).
* The F_alg counter on a case counted by hand.
"""
import numpy as np
import pytest

import synth
from oracle import blocks, dmrg, flops, heff, model, svd
from tests.test_oracle_model import kron_hamiltonian


def mixed_canonical(L, N, nmax, chi, seed, j):
    """Seeded MPS, right-canonical, then centre moved to bond j (sites j, j+1)."""
    d = nmax + 1
    bonds, sites = synth.random_mps(L, N, nmax, chi, seed)
    bonds, sites = dmrg.right_canonicalise(bonds, sites, d)
    for k in range(1, j):
        th = dmrg.form_theta(sites[k - 1], sites[k], bonds[k - 1], bonds[k + 1], d)
        sv = svd.svd_truncate(th, bonds[k - 1], bonds[k + 1], d, chi_max=10 ** 6,
                              absorb="right", renormalise=False)
        sites[k - 1], sites[k] = sv["A"], sv["B"]
        bonds[k] = sv["bond"]
    return bonds, sites


def full_embedding(bonds, sites, j, d):
    """Dense P: theta[a, s1, s2, b] -> full-space vector (site 1 most significant)."""
    L = len(sites)
    left = np.ones((1, 1))  # [configs, a]
    for k in range(1, j):
        A = blocks.site_to_dense(sites[k - 1], bonds[k - 1], bonds[k], d)
        left = np.einsum('ca,asb->csb', left, A).reshape(-1, A.shape[2])
    right = np.ones((1, 1))  # [b, configs]
    for k in range(L, j + 1, -1):
        B = blocks.site_to_dense(sites[k - 1], bonds[k - 1], bonds[k], d)
        right = np.einsum('asb,bc->asc', B, right).reshape(B.shape[0], -1)
    Da, Db = left.shape[1], right.shape[0]
    # P[config_left, s1, s2, config_right ; a, s1, s2, b]
    P = np.einsum('ca,st,uv,be->csueatvb', left, np.eye(d), np.eye(d), right)
    return P.reshape(left.shape[0] * d * d * right.shape[1], Da * d * d * Db)


@pytest.mark.parametrize("L,N,nmax,chi,j,U", [(5, 5, 2, 6, 2, 2.0), (6, 4, 2, 9, 3, 3.0),
                                             (6, 3, 1, 4, 1, 1.0), (5, 5, 2, 6, 4, 0.5)])
def test_dense_heff_equals_projected_hamiltonian(L, N, nmax, chi, j, U):
    d = nmax + 1
    bonds, sites = mixed_canonical(L, N, nmax, chi, seed=11 + j, j=j)
    W, qw = model.bh_mpo(nmax, 1.0, U, mu=0.1)
    Wl = [W] * L
    Lenv = dmrg.left_boundary(bonds[0], qw)
    for k in range(1, j):
        Lenv = dmrg.update_left(Lenv, sites[k - 1], W, qw, d, bonds[k - 1], bonds[k])
    Renvs = dmrg.build_right_envs(bonds, sites, Wl, qw, d)
    Renv = Renvs[j + 2] if j + 2 <= L else dmrg.right_boundary(bonds[L], qw)
    left, right = bonds[j - 1], bonds[j + 1]
    th = dmrg.form_theta(sites[j - 1], sites[j], left, right, d)
    thd = blocks.theta_to_dense(th, left, right, d)
    y = heff.heff2_dense(blocks.env_to_dense(Lenv, left, qw), W, W,
                         blocks.env_to_dense(Renv, right, qw), thd)
    P = full_embedding(bonds, sites, j, d)
    np.testing.assert_allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-12)
    H = kron_hamiltonian(L, nmax, 1.0, U, mu=0.1)
    yref = (P.conj().T @ (H @ (P @ thd.reshape(-1)))).reshape(thd.shape)
    np.testing.assert_allclose(y, yref, atol=1e-12 * max(1.0, np.abs(yref).max()))


def _random_case(left, right, nmax, seed, U=2.5, herm=False):
    d = nmax + 1
    W, qw = model.bh_mpo(nmax, 1.0, U, mu=0.2)
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = model.MPO_ADJOINT if herm else None
    Le = synth.random_env(left, qw, rng, pairs)
    Re = synth.random_env(right, qw, rng, pairs)
    th = synth.random_theta(left, right, d, rng)
    return W, qw, Le, Re, th


CASES = [
    ({2: 3, 3: 4, 4: 2}, {4: 2, 5: 3, 6: 4, 7: 1}, 2),
    ({0: 1}, {0: 1, 1: 2, 2: 1}, 1),
    ({12: 2, 13: 5, 14: 7, 15: 4}, {14: 3, 15: 6, 16: 8, 17: 5, 18: 2}, 4),
]


@pytest.mark.parametrize("left,right,nmax", CASES)
def test_block_heff_equals_dense(left, right, nmax):
    d = nmax + 1
    W, qw, Le, Re, th = _random_case(left, right, nmax, seed=5)
    y = heff.heff2_block(Le, W, W, Re, th, left, right, qw, d)
    yd = heff.heff2_dense(blocks.env_to_dense(Le, left, qw), W, W,
                          blocks.env_to_dense(Re, right, qw),
                          blocks.theta_to_dense(th, left, right, d))
    assert blocks.theta_forbidden_norm(yd, left, right, d) == 0.0
    ref = blocks.theta_from_dense(yd, left, right, d)
    assert set(ref) == set(y)
    for k in ref:
        np.testing.assert_allclose(y[k], ref[k], atol=1e-12)


@pytest.mark.parametrize("left,right,nmax", CASES)
def test_heff_hermitian_and_conserving(left, right, nmax):
    d = nmax + 1
    W, qw, Le, Re, _ = _random_case(left, right, nmax, seed=9, herm=True)
    rng = np.random.Generator(np.random.PCG64(3))
    keys = blocks.theta_keys(left, right, d)
    for _ in range(3):
        x = synth.random_theta(left, right, d, rng)
        y = synth.random_theta(left, right, d, rng)
        hx = heff.heff2_block(Le, W, W, Re, x, left, right, qw, d)
        hy = heff.heff2_block(Le, W, W, Re, y, left, right, qw, d)
        a = np.vdot(blocks.flatten(y, keys), blocks.flatten(hx, keys))
        b = np.vdot(blocks.flatten(x, keys), blocks.flatten(hy, keys))
        assert abs(a - np.conj(b)) <= 1e-12 * max(1.0, abs(a))
    if blocks.dim(left) * blocks.dim(right) * d * d <= 2000:
        M = heff.heff2_matrix_dense(blocks.env_to_dense(Le, left, qw), W, W,
                                    blocks.env_to_dense(Re, right, qw))
        np.testing.assert_allclose(M, M.conj().T, atol=1e-12)
        # N conservation: no element maps an allowed block outside the allowed set
        mask = np.zeros((blocks.dim(left), d, d, blocks.dim(right)), dtype=bool)
        ol, orr = blocks.offsets(left), blocks.offsets(right)
        for (q, s1, s2) in keys:
            qb = q + s1 + s2
            mask[ol[q]:ol[q] + left[q], s1, s2, orr[qb]:orr[qb] + right[qb]] = True
        m = mask.reshape(-1)
        assert np.abs(M[np.ix_(~m, m)]).max(initial=0.0) == 0.0


def test_flops_hand_count():
    # one left sector {0: 2}, hard-core bosons (d = 2), right bond {0: 3, 1: 1, 2: 4}
    left, right, nmax = {0: 2}, {0: 3, 1: 1, 2: 4}, 1
    W, qw = model.bh_mpo(nmax, 1.0, 2.0, mu=0.5)
    f = flops.heff2_flops(left, right, 2, qw, W, W)
    # theta blocks (0,s1,s2): (0,0,0)->qb 0, (0,0,1),(0,1,0)->qb 1, (0,1,1)->qb 2.
    # Only w = 0, 3 have L blocks (qa' = qa = 0).  Output blocks and live u:
    #   u = 0: every output block; terms from w = 0 (identity) and w = 3 (h x I +
    #   I x h, hopping b^+ x b and b x b^+ within the allowed s range).
    #   u = 1 needs R block (1, qb' - 1); u = 2 needs (2, qb' + 1); u = 3 needs (3, qb').
    # Counted by hand: step1 = 8*2*2*(3+1+1+4)*2 = 576 (w = 0 and w = 3, all blocks)
    assert f["step1"] == 576
    # step 4: per output block with R-block qb = qb' - qw[u] present and a live term:
    #  (0,0,0) qb'=0: u0 (K=3), u3 (K=3)  [u1 needs qb=-1: absent; u2: qb=1 but W2[3,2]=-Jb
    #                 acting into s2'=0 from s2=1: needs theta (0,0,1)(w=3): yes -> K=1]
    #  (0,0,1) qb'=1: u0 K=1, u1 K=3 (-J b^+ from s2=0), u3 K=1, u2 qb=2 K=4 (from s2=2: no) -> 0
    #  (0,1,0) qb'=1: u0 K=1, u3 K=1, u2 qb=2: from s2=1 -> theta (0,1,1): yes K=4; u1 none
    #  (0,1,1) qb'=2: u0 K=4, u1 qb=1 K=1 (from s2=0), u3 K=4
    step4 = 8 * 2 * (3 * 3 + 3 * 3 + 1 * 3) \
        + 8 * 2 * (1 * 1 + 3 * 1 + 1 * 1) \
        + 8 * 2 * (1 * 1 + 1 * 1 + 4 * 1) \
        + 8 * 2 * (4 * 4 + 1 * 4 + 4 * 4)
    assert f["step4"] == step4
    assert f["total"] == f["step1"] + f["mpo"] + f["step4"]
