"""GPU parity of tnt_lanczos_ground and tnt_theta_svd_truncate with the oracle.

Lanczos: same start vector and Hermitian operator on both sides; the FP64
path must reproduce the oracle's refined energy to 1e-11 (relative) and its
ground vector up to a phase; the FP32 path's energy is checked against the
same reference (the matvec error enters the final Rayleigh quotient only
through the Krylov vectors).
SVD: kept singular values, kept dims per sector, chi, epsilon, and the
gauge-invariant product A.B, for both absorb directions and several
truncation rules.  Singular values are compared with an absolute tolerance of
16 n eps lambda_0 (n the sector order): the backward error of any stable FP64
SVD, the oracle's included, is of that size, so no sharper bar separates two
correct results; values far above it agree to 1e-12 relative.
"""
import contextlib

import numpy as np
import pytest

import synth
from oracle import blocks, heff as oheff, lanczos as olanczos, model, svd as osvd

pytestmark = pytest.mark.gpu


def herm_case(left, right, nmax, seed, U=3.0):
    d = nmax + 1
    W, qw = model.bh_mpo(nmax, 1.0, U, 0.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    Le = synth.random_env(left, qw, rng, model.MPO_ADJOINT)
    Re = synth.random_env(right, qw, rng, model.MPO_ADJOINT)
    th = synth.random_theta(left, right, d, rng)
    return W, qw, Le, Re, th, (nmax, 1.0, U, 0.0)


def gpu_mpo(tnt, params):
    """The library's own Bose-Hubbard MPO (the oracle's is not handed over)."""
    from paper_1610_02244_amd import binding as B
    Wg, qg = tnt.bose_hubbard_mpo(*params)
    return B.Mpo(Wg, qg)


def oracle_lanczos(W, qw, Le, Re, th, left, right, d, kmax):
    keys = sorted(th)

    def mv(x):
        y = oheff.heff2_block(Le, W, W, Re, blocks.unflatten(x, th, keys), left, right, qw, d)
        return blocks.flatten(y, keys)

    return olanczos.lanczos_ground(mv, blocks.flatten(th, keys), kmax=kmax), keys


LCASES = {
    "small": ({2: 2, 3: 3}, {4: 2, 5: 3, 6: 1}, 2),
    "cfg2_like": ({13: 7, 14: 26, 15: 57, 16: 40}, {15: 20, 16: 57, 17: 75, 18: 26}, 4),
}


@pytest.mark.parametrize("name", list(LCASES))
def test_lanczos_fp64_parity(tnt, name):
    from paper_1610_02244_amd import binding as B
    left, right, nmax = LCASES[name]
    print(f"[lanczos fp64] {name}", flush=True)
    W, qw, Le, Re, th, params = herm_case(left, right, nmax, seed=3)
    ref, keys = oracle_lanczos(W, qw, Le, Re, th, left, right, nmax + 1, 20)
    mpo = gpu_mpo(tnt, params)
    td = tnt.theta(th, keys)
    res = tnt.lanczos_ground(tnt.env(Le, qw), mpo, mpo, tnt.env(Re, qw), td, kmax=20)
    print(f"  E gpu {res['E']:.15f} oracle {ref['E']:.15f} steps {res['steps']}/{ref['steps']}")
    assert res["steps"] == ref["steps"]
    assert abs(res["E"] - ref["E"]) <= 1e-11 * abs(ref["E"])
    assert abs(res["E_ritz"] - ref["E_ritz"]) <= 1e-11 * abs(ref["E"])
    assert res["residual"] == pytest.approx(ref["residual"], rel=1e-6, abs=1e-12)
    psi = blocks.flatten(tnt.download(td), keys)
    ov = abs(np.vdot(psi, ref["psi"]))
    assert ov == pytest.approx(1.0, abs=1e-11)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", list(LCASES))
def test_lanczos_fp32_energy(tnt, name, precision):
    from paper_1610_02244_amd import binding as B
    left, right, nmax = LCASES[name]
    W, qw, Le, Re, th, params = herm_case(left, right, nmax, seed=4)
    ref, keys = oracle_lanczos(W, qw, Le, Re, th, left, right, nmax + 1, 20)
    mpo = gpu_mpo(tnt, params)
    td = tnt.theta(th, keys)
    res = tnt.lanczos_ground(tnt.env(Le, qw), mpo, mpo, tnt.env(Re, qw), td, kmax=20,
                             precision=precision)
    rel = abs(res["E"] - ref["E"]) / abs(ref["E"])
    print(f"  [lanczos {precision}] {name}: |dE/E| = {rel:.3e}")
    assert rel <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_lanczos_graph_replays_match_eager(tnt, precision):
    """The recurrence replayed from a HIP graph gives bitwise the eager
    result, on every replay (eager work and synchronisations in between)."""
    left, right, nmax = LCASES["cfg2_like"]
    W, qw, Le, Re, th, params = herm_case(left, right, nmax, seed=9)
    keys = sorted(th)
    mpo = gpu_mpo(tnt, params)
    Ld, Rd = tnt.env(Le, qw), tnt.env(Re, qw)

    def run():
        td = tnt.theta(th, keys)
        r = tnt.lanczos_ground(Ld, mpo, mpo, Rd, td, kmax=20, precision=precision)
        return r, tnt.download(td)

    ref, psi_ref = run()
    try:
        tnt.set_graphs(True)
        for rep in range(3):
            got, psi = run()
            print(f"  [graph {precision}] replay {rep}: E = {got['E']:.15f}", flush=True)
            assert got["E"] == ref["E"] and got["E_ritz"] == ref["E_ritz"]
            assert got["steps"] == ref["steps"]
            for k in psi_ref:
                assert np.array_equal(psi[k], psi_ref[k])
            tnt.heff2_apply(Ld, mpo, mpo, Rd, tnt.theta(th, keys),
                            tnt.theta_like(tnt.theta(th, keys)), "fp64")
            tnt.sync()
    finally:
        tnt.set_graphs(False)


SCASE_L = {10: 6, 11: 17, 12: 9, 13: 2}
SCASE_R = {12: 4, 13: 11, 14: 15, 15: 8, 16: 1}


@pytest.mark.parametrize("absorb", ["right", "left"])
@pytest.mark.parametrize("rules", [dict(chi_max=12), dict(chi_max=1000),
                                   dict(chi_max=40, rel_tol=0.05),
                                   dict(chi_max=1000, err_tol=0.3),
                                   dict(chi_max=1000, abs_tol=0.4)])
def test_svd_truncate_parity(tnt, absorb, rules):
    d = 3
    rng = np.random.Generator(np.random.PCG64(9))
    th = synth.random_theta(SCASE_L, SCASE_R, d, rng)
    ref = osvd.svd_truncate(th, SCASE_L, SCASE_R, d, rules["chi_max"],
                            a=rules.get("abs_tol", -1.0), r=rules.get("rel_tol", -1.0),
                            e=rules.get("err_tol", -1.0), absorb=absorb)
    got = tnt.svd_truncate(tnt.theta(th), absorb=absorb, **rules)
    assert got["chi"] == ref["chi"]
    assert got["bond"] == ref["bond"]
    n = max(sum(SCASE_L.values()), sum(SCASE_R.values()))
    lam0 = ref["lambda0"] / ref["norm_kept"] if "norm_kept" in ref else None
    all_ref = np.concatenate([ref["lambdas"][m] for m in ref["bond"]])
    lam0 = all_ref.max()
    for m in ref["bond"]:
        r_ = ref["lambdas"][m]
        tol = 1e-12 * r_ + 16 * n * 2.2e-16 * lam0
        assert np.all(np.abs(got["lambdas"][m] - r_) <= tol), m
    assert got["eps"] == pytest.approx(ref["eps"], rel=1e-9, abs=1e-12)
    # the product A.B is gauge invariant
    for (qa, s1, s2) in blocks.theta_keys(SCASE_L, SCASE_R, d):
        mid = qa + s1
        if mid not in ref["bond"]:
            continue
        g = got["A"][(qa, s1)] @ got["B"][(mid, s2)]
        r = ref["A"][(qa, s1)] @ ref["B"][(mid, s2)]
        np.testing.assert_allclose(g, r, atol=1e-10)
    # the isometric factor is orthonormal to working precision
    for m, k in got["bond"].items():
        if absorb == "right":
            U = np.concatenate([got["A"][(m - s1, s1)] for s1 in range(d)
                                if (m - s1, s1) in got["A"]], axis=0)
            np.testing.assert_allclose(U.conj().T @ U, np.eye(k), atol=1e-13)
        else:
            V = np.concatenate([got["B"][(m, s2)] for s2 in range(d) if (m, s2) in got["B"]],
                               axis=1)
            np.testing.assert_allclose(V @ V.conj().T, np.eye(k), atol=1e-13)


SMALL_L0 = {0: 1, 1: 2, 2: 5, 3: 7, 4: 4}
SMALL_R0 = {1: 3, 2: 6, 3: 5, 4: 8, 5: 2, 6: 1}


# 21 charges of dimension 24 on each side, d = 2: 20 sectors whose Gram
# matrices have order 48, one batched library call of 20 problems
MID_L = {q: 24 for q in range(21)}
MID_R = {q: 24 for q in range(1, 23)}


# The SVD's sector eigenproblems either through rocSOLVER's batched Hermitian
# eigensolver ("library") or, from padded order 48 up, through the library's
# own panel tridiagonal reduction followed by rocSOLVER's divide and conquer
# and back-transformation ("own"); the context's default is restored after.
EIG_PATHS = {"library": 0, "own": 48}


@contextlib.contextmanager
def eig_path(tnt, path):
    tnt.set_eig_reduction(EIG_PATHS[path])
    try:
        yield
    finally:
        tnt.set_eig_reduction(-1)


@pytest.mark.parametrize("eig", list(EIG_PATHS))
@pytest.mark.parametrize("absorb", ["right", "left"])
@pytest.mark.parametrize("shape", ["small", "mid"])
def test_svd_truncate_small_sectors_graded(tnt, absorb, shape, eig):
    """Only small sectors: Gram orders 1..~20, odd and even (the Jacobi
    eigensolver's range), or 20 sectors of order 48 (one batched library
    eigensolve), with theta's blocks scaled by a geometric factor per block so
    the Gram eigenvalues span ~10 orders of magnitude; every value is kept.
    Checked against the oracle like the general case."""
    d, SMALL_L, SMALL_R = (3, SMALL_L0, SMALL_R0) if shape == "small" else (2, MID_L, MID_R)
    rng = np.random.Generator(np.random.PCG64(21))
    th = synth.random_theta(SMALL_L, SMALL_R, d, rng)
    step = 0.12 if shape == "small" else 10.0 / len(th)
    for i, k in enumerate(sorted(th)):
        th[k] = th[k] * 10.0 ** (-step * i)
    ref = osvd.svd_truncate(th, SMALL_L, SMALL_R, d, 10 ** 4, absorb=absorb)
    with eig_path(tnt, eig):
        got = tnt.svd_truncate(tnt.theta(th), absorb=absorb, chi_max=10 ** 4)
    assert got["chi"] == ref["chi"]
    assert got["bond"] == ref["bond"]
    all_ref = np.concatenate([ref["lambdas"][m] for m in ref["bond"]])
    lam0 = all_ref.max()
    n = max(sum(SMALL_L.values()), sum(SMALL_R.values()))
    for m in ref["bond"]:
        r_ = ref["lambdas"][m]
        tol = 1e-12 * r_ + 16 * n * 2.2e-16 * lam0
        assert np.all(np.abs(got["lambdas"][m] - r_) <= tol), m
    for (qa, s1, s2) in blocks.theta_keys(SMALL_L, SMALL_R, d):
        mid = qa + s1
        if mid not in ref["bond"]:
            continue
        g = got["A"][(qa, s1)] @ got["B"][(mid, s2)]
        r = ref["A"][(qa, s1)] @ ref["B"][(mid, s2)]
        np.testing.assert_allclose(g, r, atol=1e-10 * lam0)
    for m, k in got["bond"].items():
        if absorb == "right":
            U = np.concatenate([got["A"][(m - s1, s1)] for s1 in range(d)
                                if (m - s1, s1) in got["A"]], axis=0)
            np.testing.assert_allclose(U.conj().T @ U, np.eye(k), atol=1e-13)
        else:
            V = np.concatenate([got["B"][(m, s2)] for s2 in range(d) if (m, s2) in got["B"]],
                               axis=1)
            np.testing.assert_allclose(V @ V.conj().T, np.eye(k), atol=1e-13)


@pytest.mark.parametrize("eig", list(EIG_PATHS))
@pytest.mark.parametrize("absorb", ["right", "left"])
def test_svd_truncate_large_sectors_with_zero_rows(tnt, absorb, eig):
    """Sectors of 100-200 rows (the eigensolver's divide-and-conquer range),
    with every fifth row and column of theta exactly zero: the Gram matrices
    then have exact zero rows, which must not break the padded batched
    eigensolve."""
    d = 3
    L = {10: 40, 11: 65, 12: 50, 13: 20}
    R = {12: 30, 13: 55, 14: 70, 15: 45, 16: 10}
    rng = np.random.Generator(np.random.PCG64(21))
    th = synth.random_theta(L, R, d, rng)
    for k in th:
        th[k][::5, :] = 0
        th[k][:, ::5] = 0
    chi_max = 150
    print(f"[svd zero rows {absorb}]", flush=True)
    ref = osvd.svd_truncate(th, L, R, d, chi_max, absorb=absorb)
    with eig_path(tnt, eig):
        got = tnt.svd_truncate(tnt.theta(th), absorb=absorb, chi_max=chi_max)
    assert got["chi"] == ref["chi"]
    assert got["bond"] == ref["bond"]
    n = max(sum(L.values()), sum(R.values()))
    lam0 = np.concatenate([ref["lambdas"][m] for m in ref["bond"]]).max()
    for m in ref["bond"]:
        r_ = ref["lambdas"][m]
        assert np.all(np.isfinite(got["lambdas"][m]))
        tol = 1e-12 * r_ + 16 * n * 2.2e-16 * lam0
        assert np.all(np.abs(got["lambdas"][m] - r_) <= tol), m
    for (qa, s1, s2) in blocks.theta_keys(L, R, d):
        mid = qa + s1
        if mid not in ref["bond"]:
            continue
        g = got["A"][(qa, s1)] @ got["B"][(mid, s2)]
        r = ref["A"][(qa, s1)] @ ref["B"][(mid, s2)]
        np.testing.assert_allclose(g, r, atol=1e-10)


def sector_spectrum_theta(left, right, d, rng, spectrum):
    """theta whose sector m = q_a + s1 has the singular values spectrum(m, k)
    (k = min(rows, cols) values) with random unitary vectors; returned as
    blocks, with the exact spectra per sector."""
    th, exact = {}, {}
    for (m, rows, cols) in osvd.theta_sectors(left, right, d):
        R = sum(left[qa] for (_, qa) in rows)
        Cn = sum(right[qb] for (_, qb) in cols)
        k = min(R, Cn)
        sig = np.asarray(spectrum(m, k), dtype=float)
        qa_, _ = np.linalg.qr(synth._cnormal(rng, (R, k)))
        qb_, _ = np.linalg.qr(synth._cnormal(rng, (Cn, k)))
        M = (qa_ * sig[None, :]) @ qb_.conj().T
        exact[m] = np.sort(sig)[::-1]
        ro = 0
        for (s1, qa) in rows:
            co = 0
            for (s2, qb) in cols:
                th[(qa, s1, s2)] = M[ro:ro + left[qa], co:co + right[qb]].copy()
                co += right[qb]
            ro += left[qa]
    keys = blocks.theta_keys(left, right, d)
    return {k: th[k] for k in keys}, exact


def check_svd_vs_oracle(tnt, th, left, right, d, absorb, n, eig="library", **rules):
    ref = osvd.svd_truncate(th, left, right, d, rules.get("chi_max", 10 ** 6),
                            a=rules.get("abs_tol", -1.0), r=rules.get("rel_tol", -1.0),
                            e=rules.get("err_tol", -1.0), absorb=absorb)
    with eig_path(tnt, eig):
        got = tnt.svd_truncate(tnt.theta(th), absorb=absorb, **rules)
    assert got["chi"] == ref["chi"]
    assert got["bond"] == ref["bond"]
    lam0 = np.concatenate([ref["lambdas"][m] for m in ref["bond"]]).max()
    tol_abs = 16 * n * 2.2e-16 * lam0
    worst = 0.0
    for m in ref["bond"]:
        r_ = ref["lambdas"][m]
        err = np.abs(got["lambdas"][m] - r_)
        worst = max(worst, float(np.max(err / (1e-12 * r_ + tol_abs))))
        assert np.all(err <= 1e-12 * r_ + tol_abs), m
    # epsilon: sqrt of the discarded squares, each value to tol_abs
    assert got["eps"] == pytest.approx(ref["eps"], rel=1e-9, abs=tol_abs * 4)
    for (qa, s1, s2) in blocks.theta_keys(left, right, d):
        mid = qa + s1
        if mid not in ref["bond"]:
            continue
        g = got["A"][(qa, s1)] @ got["B"][(mid, s2)]
        r = ref["A"][(qa, s1)] @ ref["B"][(mid, s2)]
        np.testing.assert_allclose(g, r, atol=1e-9 * lam0)
    for m, k in got["bond"].items():
        if absorb == "right":
            U = np.concatenate([got["A"][(m - s1, s1)] for s1 in range(d)
                                if (m - s1, s1) in got["A"]], axis=0)
            np.testing.assert_allclose(U.conj().T @ U, np.eye(k), atol=1e-12)
        else:
            V = np.concatenate([got["B"][(m, s2)] for s2 in range(d) if (m, s2) in got["B"]],
                               axis=1)
            np.testing.assert_allclose(V @ V.conj().T, np.eye(k), atol=1e-12)
    return ref, got, worst


GRADED_L = {10: 9, 11: 30, 12: 47, 13: 20, 14: 3}
GRADED_R = {12: 5, 13: 26, 14: 52, 15: 33, 16: 11, 17: 2}


@pytest.mark.parametrize("absorb", ["right", "left"])
@pytest.mark.parametrize("rules", [dict(chi_max=10 ** 6, rel_tol=1e-12),
                                   dict(chi_max=10 ** 6),
                                   dict(chi_max=130),
                                   dict(chi_max=10 ** 6, err_tol=1e-9)])
@pytest.mark.parametrize("eig", list(EIG_PATHS))
def test_svd_truncate_deep_spectrum(tnt, absorb, rules, eig):
    """Sector spectra that fall geometrically from 1 to 1e-15 (orders 2..~140,
    both eigensolver paths): the relative cut at 1e-12, keeping everything,
    a chi cut deep in the spectrum and the error rule at 1e-9 must all give
    the oracle's kept set, values and error.  This needs singular values far
    below the square root of the FP64 rounding level of a Gram matrix."""
    d = 3
    rng = np.random.Generator(np.random.PCG64(31))

    m0 = min(GRADED_L) + 0  # the smallest middle charge holds lambda_0 = 1

    def spec(m, k):
        # exponents 0..15.6 with the window (11.7, 12.3) left empty, so no value
        # lies within a factor 1.6 of the relative cut; a factor per sector in
        # [0.8, 1] (distinct) keeps values of different sectors apart
        e = np.linspace(0.0, 15.0, k) if k > 1 else np.array([0.0])
        e = np.where(e < 11.7, e, e + 0.6)
        return 10.0 ** (-e) * (1.0 - 0.02 * (m - m0)) * (1 + 0.003 * np.arange(k) / max(k, 1))

    th, exact = sector_spectrum_theta(GRADED_L, GRADED_R, d, rng, spec)
    n = max(sum(GRADED_L.values()), sum(GRADED_R.values()))
    print(f"[svd deep spectrum {absorb} {rules} {eig}]", flush=True)
    ref, got, worst = check_svd_vs_oracle(tnt, th, GRADED_L, GRADED_R, d, absorb, n, eig,
                                          **rules)
    print(f"  chi {got['chi']} eps {got['eps']:.3e} (oracle {ref['eps']:.3e}) worst/tol {worst:.2e}")


def graded_theta(left, right, d, rng, decades):
    """Seeded theta with every block's rows and columns scaled geometrically
    (10^-decades over each block's extent), so each sector's spectrum spreads
    over ~2 decades' worth of orders."""
    th = synth.random_theta(left, right, d, rng)
    for k, v in th.items():
        r = 10.0 ** (-decades * np.arange(v.shape[0]) / max(v.shape[0], 1))
        c = 10.0 ** (-decades * np.arange(v.shape[1]) / max(v.shape[1], 1))
        th[k] = (r[:, None] * v) * c[None, :]
    return th


@pytest.mark.parametrize("eig", list(EIG_PATHS))
@pytest.mark.parametrize("cfg,chi_max", [("cfg3", 1024), ("cfg5", 2048)])
def test_svd_truncate_full_size(tnt, cfg, chi_max, eig):
    """The middle-bond theta of the chi = 1024 and chi = 2048 chains (sectors
    up to 963 and 1925 rows), with a graded spectrum spanning ~12 decades:
    kept set, values and error equal the oracle's for a chi cut and for the
    relative cut 1e-6, and with every value kept (chi = 1024 case, both absorb
    directions)."""
    s = synth.CONFIGS[cfg]
    bonds = synth.chain_bonds(s.L, s.N, s.nmax, s.chi)
    j = s.L // 2
    left, right = bonds[j - 1], bonds[j + 1]
    rng = np.random.Generator(np.random.PCG64(s.seed * 101))
    th = graded_theta(left, right, s.d, rng, decades=6.0)
    secs = osvd.theta_sectors(left, right, s.d)
    n = max(max(sum(left[qa] for (_, qa) in r), sum(right[qb] for (_, qb) in c_))
            for (_, r, c_) in secs)
    # (a relative cut at 1e-12 is not compared here: a random spectrum this
    # dense puts values within the FP64 backward error of such a cut, where
    # two correct SVDs may keep different counts)
    cases = [("right", dict(chi_max=chi_max)), ("left", dict(chi_max=10 ** 6, rel_tol=1e-6))]
    if cfg == "cfg3":
        cases += [("left", dict(chi_max=chi_max)), ("right", dict(chi_max=10 ** 6))]
    for absorb, rules in cases:
        print(f"[svd full size {cfg} {absorb} {rules} {eig}] max sector order {n}", flush=True)
        ref, got, worst = check_svd_vs_oracle(tnt, th, left, right, s.d, absorb, n, eig,
                                              **rules)
        print(f"  chi {got['chi']} eps {got['eps']:.6e} (oracle {ref['eps']:.6e}) "
              f"worst/tol {worst:.2e}", flush=True)
