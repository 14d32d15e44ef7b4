"""GPU parity of tnt_heff2_apply against the oracle's block H_eff . theta.

Inputs are seeded synthetic blocks (synth); the oracle and the HIP library
each compute H_eff . theta on the same arrays.  Bars (normwise relative
error over all blocks): FP64 <= 1e-12; FP32-MFMA <= 2e-6 (FP32 rounding of
operands and sums over K <= ~4 * 300 terms); BF16x3 <= 1e-4: each operand
is split as hi + lo with a residual <= 2^-16 |x| and the lo*lo term is
dropped, so one real product is off by <= 3 * 2^-16 relative; the two GEMM
stages (L . theta, then . R on re-split slabs) give <= 6 * 2^-16 = 9.2e-5
elementwise in the |A||B| sense, and the normwise error is below that.
"""
import numpy as np
import pytest

import synth
from oracle import heff as oheff
from oracle import model

pytestmark = pytest.mark.gpu


def rel_err(a: dict, b: dict) -> float:
    num = sum(float(np.sum(np.abs(a[k] - b[k]) ** 2)) for k in b)
    den = sum(float(np.sum(np.abs(b[k]) ** 2)) for k in b)
    return (num / den) ** 0.5


class Model(tuple):
    """The oracle's MPO (W, qw) plus the model parameters the GPU side uses to
    build its own MPO with the library."""


def make_case(left, right, nmax, seed, U=3.0, J=1.0, mu=0.0, herm=True):
    d = nmax + 1
    W, qw = model.bh_mpo(nmax, J, U, mu)
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = model.MPO_ADJOINT if herm else None
    Le = synth.random_env(left, qw, rng, pairs)
    Re = synth.random_env(right, qw, rng, pairs)
    th = synth.random_theta(left, right, d, rng)
    Wm = Model((W, (nmax, J, U, mu)))
    return Wm, qw, Le, Re, th


def gpu_mpo(tnt, Wm):
    """The library's own Bose-Hubbard MPO for the model parameters of Wm."""
    from paper_1610_02244_amd import binding as B
    nmax, J, U, mu = Wm[1]
    Wg, qg = tnt.bose_hubbard_mpo(nmax, J, U, mu)
    return B.Mpo(Wg, qg)


def bonds_of(cfg):
    s = synth.CONFIGS[cfg]
    b = synth.chain_bonds(s.L, s.N, s.nmax, s.chi)
    j = s.L // 2
    return b[j - 1], b[j + 1], s.nmax


CASES = {
    "tiny": ({0: 1}, {0: 1, 1: 2, 2: 1}, 1),
    "cfg1_mid": bonds_of("cfg1"),
    "ragged": ({10: 37, 11: 130, 12: 65, 13: 3}, {12: 9, 13: 70, 14: 129, 15: 64, 16: 1}, 2),
    "cfg2_mid": bonds_of("cfg2"),
}


def run_gpu(tnt, Wm, qw, Le, Re, th, precision):
    mpo = gpu_mpo(tnt, Wm)
    Ld, Rd, td = tnt.env(Le, qw), tnt.env(Re, qw), tnt.theta(th)
    out = tnt.theta_like(td)
    tnt.heff2_apply(Ld, mpo, mpo, Rd, td, out, precision)
    return tnt.download(out)


@pytest.mark.parametrize("name", list(CASES))
def test_heff_fp64_parity(tnt, name):
    left, right, nmax = CASES[name]
    print(f"[heff fp64] case={name} left={left} right={right}", flush=True)
    W, qw, Le, Re, th = make_case(left, right, nmax, seed=17)
    ref = oheff.heff2_block(Le, W[0], W[0], Re, th, left, right, qw, nmax + 1)
    got = run_gpu(tnt, W, qw, Le, Re, th, "fp64")
    assert set(got) == set(ref)
    err = rel_err(got, ref)
    print(f"  rel err fp64 = {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_heff_bf16x3_parity(tnt, name):
    left, right, nmax = CASES[name]
    print(f"[heff bf16x3] case={name}", flush=True)
    W, qw, Le, Re, th = make_case(left, right, nmax, seed=29)
    ref = oheff.heff2_block(Le, W[0], W[0], Re, th, left, right, qw, nmax + 1)
    got = run_gpu(tnt, W, qw, Le, Re, th, "bf16x3")
    assert set(got) == set(ref)
    err = rel_err(got, ref)
    print(f"  rel err bf16x3 = {err:.3e}")
    assert err <= 1e-4
    # the split-product arithmetic really ran: FP32 would be ~100x closer
    assert err >= 1e-7


@pytest.mark.parametrize("name", list(CASES))
def test_heff_fp32_parity(tnt, name):
    left, right, nmax = CASES[name]
    print(f"[heff fp32] case={name}", flush=True)
    W, qw, Le, Re, th = make_case(left, right, nmax, seed=23)
    ref = oheff.heff2_block(Le, W[0], W[0], Re, th, left, right, qw, nmax + 1)
    got = run_gpu(tnt, W, qw, Le, Re, th, "fp32")
    err = rel_err(got, ref)
    print(f"  rel err fp32 = {err:.3e}")
    assert err <= 2e-6


def test_heff_fp64_deterministic(tnt):
    left, right, nmax = CASES["cfg2_mid"]
    W, qw, Le, Re, th = make_case(left, right, nmax, seed=5)
    a = run_gpu(tnt, W, qw, Le, Re, th, "fp64")
    b = run_gpu(tnt, W, qw, Le, Re, th, "fp64")
    for k in a:
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_heff_autotuned_equals_default_tiles(tnt, prec):
    """Every tile shape sums K in the same order: tuned and default results
    are bitwise identical."""
    left, right, nmax = bonds_of("cfg3")
    W, qw, Le, Re, th = make_case(left, right, nmax, seed=41)
    try:
        tnt.set_autotune(False)
        a = run_gpu(tnt, W, qw, Le, Re, th, prec)
        tnt.set_autotune(True)
        b = run_gpu(tnt, W, qw, Le, Re, th, prec)   # tunes on first use
        c = run_gpu(tnt, W, qw, Le, Re, th, prec)   # tuned choice from the cache
    finally:
        tnt.set_autotune(True)
    for k in a:
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k


@pytest.mark.parametrize("cfg,seed", [("cfg3", 31), ("cfg5", 51)])
def test_heff_full_size_all_sectors(tnt, cfg, seed):
    """The chi = 1024 (L = 64) and chi = 2048 (L = 128; blocks up to 601 x 601)
    middle bonds, in the tile shapes the autotuner picks there: every output
    block of the full launch against the oracle's block matvec, on all three
    paths."""
    left, right, nmax = bonds_of(cfg)
    print(f"[heff full size {cfg}] left={left}", flush=True)
    W, qw, Le, Re, th = make_case(left, right, nmax, seed=seed)
    ref = oheff.heff2_block(Le, W[0], W[0], Re, th, left, right, qw, nmax + 1)
    for prec, bar in (("fp64", 1e-12), ("fp32", 2e-6), ("bf16x3", 1e-4)):
        got = run_gpu(tnt, W, qw, Le, Re, th, prec)
        assert set(got) == set(ref)
        err = rel_err(got, ref)
        # and the worst output sector on its own
        worst = max(rel_err({k: got[k] for k in ref if k[0] == q},
                            {k: ref[k] for k in ref if k[0] == q})
                    for q in {k[0] for k in ref}
                    if sum(float(np.sum(np.abs(ref[k]) ** 2)) for k in ref if k[0] == q) > 0)
        print(f"  {prec}: rel err {err:.3e} over {len(ref)} blocks, worst sector {worst:.3e}",
              flush=True)
        assert err <= bar
        assert worst <= 4 * bar


def test_heff_rejects_charge_violation(tnt):
    """A descriptor edited in place after a successful call is parsed again
    (the library caches operators by descriptor content, not by address)."""
    from paper_1610_02244_amd import binding as B
    left, right, nmax = CASES["tiny"]
    W, qw, Le, Re, th = make_case(left, right, nmax, seed=1)
    mpo = gpu_mpo(tnt, W)
    Ld, Rd, td = tnt.env(Le, qw), tnt.env(Re, qw), tnt.theta(th)
    ok = tnt.theta_like(td)
    tnt.heff2_apply(Ld, mpo, mpo, Rd, td, ok, "fp32")
    td.qn[3] += 1
    with pytest.raises(B.TntError) as ei:
        tnt.heff2_apply(Ld, mpo, mpo, Rd, td, ok, "fp32")
    assert ei.value.code == -3
