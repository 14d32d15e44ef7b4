"""Pins of the automatic-blocking oracle.

* The blocks are the connected components that scipy's graph routine finds
  for the bipartite row-column graph, and the reordered matrix is block
  diagonal.
* The pooled singular values of the blocks equal numpy's SVD of the whole
  (tolerance-zeroed) matrix; the truncated product obeys Eckart-Young.
"""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph

from oracle import autoblock as oab


def hidden_blocks(rng, sizes, m_extra=0, n_extra=0, noise=0.0):
    """Block-diagonal complex matrix with random row / column orders; rows and
    columns `extra` are zero; `noise` adds entries below the tolerance."""
    m = sum(s[0] for s in sizes) + m_extra
    n = sum(s[1] for s in sizes) + n_extra
    M = np.zeros((m, n), complex)
    r = c = 0
    for (a, b) in sizes:
        M[r:r + a, c:c + b] = rng.normal(size=(a, b)) + 1j * rng.normal(size=(a, b))
        r += a
        c += b
    if noise:
        M += noise * (rng.uniform(-1, 1, size=(m, n)))
    return M[rng.permutation(m)][:, rng.permutation(n)]


@pytest.mark.parametrize("seed", range(3))
def test_components_equal_scipy(seed):
    rng = np.random.default_rng(seed)
    M = hidden_blocks(rng, [(3, 4), (5, 2), (1, 1), (6, 6)], m_extra=2, n_extra=1, noise=1e-9)
    mask = np.abs(M) > 1e-6
    blocks = oab.components(mask)
    m, n = mask.shape
    g = scipy.sparse.bmat([[None, scipy.sparse.csr_matrix(mask)],
                           [scipy.sparse.csr_matrix(mask.T), None]])
    ncomp, lab = scipy.sparse.csgraph.connected_components(g, directed=False)
    got = sorted((tuple(r), tuple(c)) for r, c in blocks)
    want = []
    for k in range(ncomp):
        rows = tuple(int(i) for i in np.nonzero(lab[:m] == k)[0])
        cols = tuple(int(j) for j in np.nonzero(lab[m:] == k)[0])
        if rows and cols:
            want.append((rows, cols))
    assert got == sorted(want)
    assert len(blocks) == 4
    # reordered: block diagonal
    order_r = np.concatenate([r for r, _ in blocks])
    order_c = np.concatenate([c for _, c in blocks])
    P = np.where(mask, 1, 0)[np.ix_(order_r, order_c)]
    r0 = c0 = 0
    for r, c in blocks:
        P[r0:r0 + len(r), c0:c0 + len(c)] = 0
        r0 += len(r)
        c0 += len(c)
    assert not P.any()


@pytest.mark.parametrize("seed,chi", [(0, 100), (1, 7), (2, 3)])
def test_spectrum_and_eckart_young(seed, chi):
    rng = np.random.default_rng(10 + seed)
    M = hidden_blocks(rng, [(4, 6), (7, 3), (2, 2)], m_extra=1, noise=1e-10)
    out = oab.auto_block_svd(M, 1e-8, chi)
    Z = np.where(np.abs(M) > 1e-8, M, 0)
    S = np.linalg.svd(Z, compute_uv=False)
    np.testing.assert_allclose(out["all_lam"], S[:len(out["all_lam"])], atol=1e-12)
    assert out["chi"] == min(chi, len(out["all_lam"]))
    err = np.linalg.norm(Z - out["approx"])
    assert err == pytest.approx(np.sqrt(np.sum(S[out["chi"]:] ** 2)), abs=1e-10)
    assert out["eps"] == pytest.approx(err, abs=1e-10)
