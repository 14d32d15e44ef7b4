"""The allocation-free entry point tnt_heff2_apply_noalloc against the
existing tnt_heff2_apply (through the C-ABI).

Both run the same plan and kernels, so the results must agree to the H_eff
parity bars (FP64 1e-12, FP32 2e-6, BF16x3 1e-4 normwise; in practice they
are bitwise equal).  Two calls in a row, the second on a smaller operator,
show that the shared scratch array carries nothing from one call to the next;
an operator larger than the array is refused before anything runs.
"""
import numpy as np
import pytest

import synth
from oracle import model

pytestmark = pytest.mark.gpu

BARS = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 1e-4}


def case(cfg, seed, nmax_override=None):
    s = synth.CONFIGS[cfg]
    bonds = synth.chain_bonds(s.L, s.N, s.nmax, s.chi)
    j = s.L // 2
    left, right = bonds[j - 1], bonds[j + 1]
    W, qw = model.bh_mpo(s.nmax, s.J, s.U, s.mu)
    rng = np.random.Generator(np.random.PCG64(seed))
    Le = synth.random_env(left, qw, rng, model.MPO_ADJOINT)
    Re = synth.random_env(right, qw, rng, model.MPO_ADJOINT)
    th = synth.random_theta(left, right, s.d, rng)
    return s, qw, Le, Re, th


def both(tnt, s, qw, Le, Re, th, precision):
    from paper_1610_02244_amd import binding as B
    Wg, qg = tnt.bose_hubbard_mpo(s.nmax, s.J, s.U, s.mu)
    mpo = B.Mpo(Wg, qg)
    Ld, Rd, td = tnt.env(Le, qw), tnt.env(Re, qw), tnt.theta(th)
    o1, o2 = tnt.theta_like(td), tnt.theta_like(td)
    tnt.heff2_apply(Ld, mpo, mpo, Rd, td, o1, precision)
    tnt.sync()
    tnt.heff2_apply_noalloc(Ld, mpo, mpo, Rd, td, o2, precision)
    return tnt.download(o1), tnt.download(o2)


def rel(a, b):
    num = sum(float(np.sum(np.abs(a[k] - b[k]) ** 2)) for k in b)
    den = sum(float(np.sum(np.abs(b[k]) ** 2)) for k in b)
    return (num / den) ** 0.5


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_heff2_apply(tnt, precision):
    for cfg, seed in (("cfg2", 41), ("cfg1", 43)):  # the second call is smaller
        s, qw, Le, Re, th = case(cfg, seed)
        print(f"[noalloc {precision}] {cfg} middle bond, {len(th)} theta blocks", flush=True)
        ref, got = both(tnt, s, qw, Le, Re, th, precision)
        assert set(got) == set(ref)
        err = rel(got, ref)
        same = all(np.array_equal(got[k], ref[k]) for k in ref)
        print(f"  rel err vs tnt_heff2_apply {err:.2e} bitwise equal {same}", flush=True)
        assert err <= BARS[precision]


def test_noalloc_refuses_operators_beyond_scratch(tnt):
    from paper_1610_02244_amd import binding as B
    s, qw, Le, Re, th = case("cfg3", 47)
    print("[noalloc] chi = 1024 middle bond (beyond the 64 MiB scratch)", flush=True)
    Wg, qg = tnt.bose_hubbard_mpo(s.nmax, s.J, s.U, s.mu)
    mpo = B.Mpo(Wg, qg)
    Ld, Rd, td = tnt.env(Le, qw), tnt.env(Re, qw), tnt.theta(th)
    out = tnt.theta_like(td)
    with pytest.raises(B.TntError) as ei:
        tnt.heff2_apply_noalloc(Ld, mpo, mpo, Rd, td, out, "fp64")
    assert ei.value.code == -4  # TNT_E_CAPACITY
    # the context stays usable
    s1, qw1, Le1, Re1, th1 = case("cfg1", 49)
    ref, got = both(tnt, s1, qw1, Le1, Re1, th1, "fp64")
    assert rel(got, ref) <= 1e-12
