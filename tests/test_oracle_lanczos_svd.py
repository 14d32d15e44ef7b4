"""Pins of the oracle's eigensolver and truncated SVD.

Lanczos: with as many steps as the dimension it returns the lowest
eigenvalue of `numpy.linalg.eigh`; with fewer, the Ritz value bounds the true
one from above (interlacing); an exact eigenvector as start stops at once.
SVD: Eckart-Young (the Frobenius error of the truncated product equals the
2-norm truncation error), isometric factors, unit norm after renormalising,
sector spectra equal the dense SVD of the whole theta matrix, and the
truncation rules on hand-made spectra.
"""
import math

import numpy as np
import pytest

import synth
from oracle import blocks, lanczos, svd


def herm(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (A + A.conj().T) / 2


@pytest.mark.parametrize("n", [1, 5, 12])
def test_lanczos_full_dimension_is_exact(n):
    H = herm(n, n)
    x0 = np.ones(n, dtype=complex)
    res = lanczos.lanczos_ground(lambda v: H @ v, x0, kmax=20)
    assert res["E"] == pytest.approx(np.linalg.eigvalsh(H)[0], abs=1e-11)
    assert res["steps"] <= n
    assert res["residual"] < 1e-9


def test_lanczos_interlacing_and_monotone():
    H = herm(60, 1)
    e0 = np.linalg.eigvalsh(H)[0]
    x0 = np.random.Generator(np.random.PCG64(2)).standard_normal(60) + 0j
    prev = np.inf
    for k in (2, 5, 10, 20):
        r = lanczos.lanczos_ground(lambda v: H @ v, x0, kmax=k)
        assert r["E_ritz"] >= e0 - 1e-12
        assert r["E_ritz"] <= prev + 1e-12
        prev = r["E_ritz"]
        # the Rayleigh quotient of the Ritz vector equals the Ritz value
        assert r["E"] == pytest.approx(r["E_ritz"], abs=1e-10)


def test_lanczos_exact_eigenvector_start():
    H = herm(10, 4)
    w, V = np.linalg.eigh(H)
    res = lanczos.lanczos_ground(lambda v: H @ v, V[:, 0] * (0.3 + 0.4j), kmax=20)
    assert res["steps"] == 1
    assert res["E"] == pytest.approx(w[0], abs=1e-12)


# --------------------------------------------------------------------------

LEFT = {3: 4, 4: 6, 5: 3}
RIGHT = {5: 3, 6: 5, 7: 6, 8: 2}


def _theta(seed, nmax=2):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.random_theta(LEFT, RIGHT, nmax + 1, rng)


def _product(A, B, left, right, d):
    out = {}
    for (qa, s1, s2) in blocks.theta_keys(left, right, d):
        a, b = A.get((qa, s1)), B.get((qa + s1, s2))
        out[(qa, s1, s2)] = (a @ b) if (a is not None and b is not None) else \
            np.zeros((left[qa], right[qa + s1 + s2]), dtype=complex)
    return out


@pytest.mark.parametrize("chi,absorb", [(5, "right"), (9, "left"), (1000, "right")])
def test_svd_eckart_young_and_isometries(chi, absorb):
    d = 3
    th = _theta(1)
    res = svd.svd_truncate(th, LEFT, RIGHT, d, chi, absorb=absorb, renormalise=False)
    approx = _product(res["A"], res["B"], LEFT, RIGHT, d)
    keys = blocks.theta_keys(LEFT, RIGHT, d)
    err = np.linalg.norm(blocks.flatten(th, keys) - blocks.flatten(approx, keys))
    assert err == pytest.approx(res["eps"], abs=1e-12)
    # isometric factor: U^+ U = 1 (right absorb) or V V^+ = 1 (left absorb)
    for m, k in res["bond"].items():
        if absorb == "right":
            U = np.concatenate([res["A"][(m - s1, s1)] for s1 in range(d)
                                if (m - s1, s1) in res["A"]], axis=0)
            np.testing.assert_allclose(U.conj().T @ U, np.eye(k), atol=1e-13)
        else:
            V = np.concatenate([res["B"][(m, s2)] for s2 in range(d) if (m, s2) in res["B"]],
                               axis=1)
            np.testing.assert_allclose(V @ V.conj().T, np.eye(k), atol=1e-13)


def test_svd_sector_spectrum_equals_dense_spectrum():
    d = 3
    th = _theta(2)
    res = svd.svd_truncate(th, LEFT, RIGHT, d, 10 ** 6, renormalise=False)
    dense = blocks.theta_to_dense(th, LEFT, RIGHT, d)
    M = dense.reshape(dense.shape[0] * d, d * dense.shape[3])
    s = np.linalg.svd(M, compute_uv=False)
    s = s[s > 1e-12]
    np.testing.assert_allclose(np.sort(res["all_lambdas"])[::-1], s, rtol=1e-12)


def test_svd_renormalised_unit_norm():
    res = svd.svd_truncate(_theta(3), LEFT, RIGHT, 3, 7)
    tot = sum(float(np.sum(v ** 2)) for v in res["lambdas"].values())
    assert tot == pytest.approx(1.0, abs=1e-14)
    assert sum(res["bond"].values()) == 7


def test_select_chi_rules():
    lam = np.array([1.0, 0.5, 0.5, 0.1, 0.01, 0.001])
    assert svd.select_chi(lam, 10) == 6
    assert svd.select_chi(lam, 3) == 3
    # absolute: discard lambda < a (strict): a = 0.1 keeps the 0.1
    assert svd.select_chi(lam, 10, a=0.1) == 4
    assert svd.select_chi(lam, 10, a=0.1000001) == 3
    # relative: lambda / lambda0 < r discarded
    assert svd.select_chi(lam, 10, r=0.01) == 5
    # error rule: largest discard with sqrt(sum discarded^2) < e
    tail = math.sqrt(0.01 ** 2 + 0.001 ** 2)
    assert svd.select_chi(lam, 10, e=tail + 1e-12) == 4
    assert svd.select_chi(lam, 10, e=tail) == 5   # strict: equal error is not below
    # the smallest chi among the active rules wins
    assert svd.select_chi(lam, 5, a=0.4, r=0.05, e=1.0) == 1
    assert svd.select_chi(lam, 2, a=0.4) == 2
    # never fewer than one value
    assert svd.select_chi(lam, 10, a=5.0) == 1
    # other error kinds
    assert svd.select_chi(lam, 10, e=0.0111, kind=svd.TYPE_1NORM) == 4
    assert svd.select_chi(lam, 10, e=0.0109, kind=svd.TYPE_1NORM) == 5
    assert svd.select_chi(lam, 10, e=0.0001011, kind=svd.TYPE_SUMSQ) == 4


def test_svd_truncation_picks_global_largest():
    # the kept set is the chi largest values pooled over all sectors
    th = _theta(4)
    full = svd.svd_truncate(th, LEFT, RIGHT, 3, 10 ** 6, renormalise=False)
    cut = svd.svd_truncate(th, LEFT, RIGHT, 3, 6, renormalise=False)
    kept = np.sort(np.concatenate(list(cut["lambdas"].values())))[::-1]
    np.testing.assert_allclose(kept, full["all_lambdas"][:6], rtol=1e-13)
    assert cut["eps"] == pytest.approx(
        math.sqrt(float(np.sum(full["all_lambdas"][6:] ** 2))), rel=1e-12)
