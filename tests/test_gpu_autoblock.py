"""GPU automatic blocking (tnt_auto_block_svd) against the auto-blocking oracle.

Matrices with hidden block structure (random row and column permutations of
a block-diagonal matrix, plus entries below the tolerance, zero rows and
columns): the number of blocks, the kept singular values (as a multiset) and
the truncation error equal the oracle's, U has orthonormal columns, and U B
equals the oracle's truncated matrix.  FP64; bar 1e-10 of the largest
singular value.
"""
import numpy as np
import pytest

from oracle import autoblock as oab

pytestmark = pytest.mark.gpu


def hidden_blocks(rng, sizes, m_extra=0, n_extra=0, noise=0.0):
    m = sum(s[0] for s in sizes) + m_extra
    n = sum(s[1] for s in sizes) + n_extra
    M = np.zeros((m, n), complex)
    r = c = 0
    for (a, b) in sizes:
        M[r:r + a, c:c + b] = rng.normal(size=(a, b)) + 1j * rng.normal(size=(a, b))
        r += a
        c += b
    if noise:
        M += noise * rng.uniform(-1, 1, size=(m, n))
    return M[rng.permutation(m)][:, rng.permutation(n)]


@pytest.mark.parametrize("seed,sizes,chi", [
    (0, [(3, 4), (5, 2), (1, 1), (6, 6)], 100),
    (1, [(40, 30), (17, 50), (64, 64), (5, 90), (33, 2)], 120),
    (2, [(40, 30), (17, 50), (64, 64), (5, 90), (33, 2)], 25),
])
def test_auto_block_svd_matches_oracle(tnt, seed, sizes, chi):
    print(f"[autoblock] seed={seed} blocks={len(sizes)} chi={chi}", flush=True)
    rng = np.random.default_rng(100 + seed)
    M = hidden_blocks(rng, sizes, m_extra=2, n_extra=3, noise=1e-9)
    tol = 1e-6
    got = tnt.auto_block_svd(M, tol, chi)
    ref = oab.auto_block_svd(M, tol, chi)
    assert got["nblocks"] == len(ref["blocks"]) == len(sizes)
    assert got["chi"] == ref["chi"]
    scale = ref["all_lam"][0]
    np.testing.assert_allclose(np.sort(got["S"])[::-1], ref["lam"], atol=1e-10 * scale)
    assert got["eps"] == pytest.approx(ref["eps"], abs=1e-9 * scale)
    U = got["U"]
    np.testing.assert_allclose(U.conj().T @ U, np.eye(got["chi"]), atol=1e-12)
    err = np.max(np.abs(U @ got["B"] - ref["approx"]))
    print(f"  max|UB - oracle| = {err:.2e}")
    assert err <= 1e-10 * scale


def test_auto_block_svd_all_below_tolerance(tnt):
    M = 1e-9 * np.ones((4, 5))
    got = tnt.auto_block_svd(M, 1e-6, 3)
    assert got["chi"] == 0 and got["nblocks"] == 0


@pytest.mark.parametrize("shape", [(1, 7), (9, 1), (40, 25)])
def test_auto_block_svd_dense_and_thin(tnt, shape):
    # no structure: one block, the plain truncated SVD
    rng = np.random.default_rng(sum(shape))
    M = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    got = tnt.auto_block_svd(M, 0.0, 50)
    S = np.linalg.svd(M, compute_uv=False)
    assert got["nblocks"] == 1 and got["chi"] == min(shape)
    np.testing.assert_allclose(np.sort(got["S"])[::-1], S, atol=1e-10 * S[0])
    np.testing.assert_allclose(got["U"] @ got["B"], M, atol=1e-10 * S[0])
