"""Host-side checks of the C-ABI library (no GPU needed).

* libtnt_mi355x.so loads and exports every function include/tnt.h declares.
* The library's integer FLOP counter equals the oracle's independent count.
* Truncation-rule selection on the host equals the oracle's rules.
* The model MPO builders equal the oracle's MPOs.
* Descriptor validation returns the documented error codes.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import flops as oflops
from oracle import model, spin1 as ospin1, svd as osvd
from paper_1610_02244_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return B.open_library()


def header_functions():
    text = open(os.path.join(ROOT, "include", "tnt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tnt_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.SIGNATURES), set(names) ^ set(B.SIGNATURES)


class HostDesc:
    """Descriptor with host metadata only (no device planes)."""

    def __init__(self, rank, qn, ext, off, total):
        self.qn = np.ascontiguousarray(np.asarray(qn, dtype=np.int32).reshape(-1))
        self.ext = np.ascontiguousarray(np.asarray(ext, dtype=np.int32).reshape(-1))
        self.off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
        self.c = B.BTensor(rank, len(off), self.qn.ctypes.data_as(B.I32P),
                           self.ext.ctypes.data_as(B.I32P), self.off.ctypes.data_as(B.I64P),
                           None, None, B.TNT_DT_F64, int(total))
        self.ref = C.byref(self.c)


def theta_desc(left, right, d):
    qn, ext, off, pos = [], [], [], 0
    for q in sorted(left):
        for s1 in range(d):
            for s2 in range(d):
                qb = q + s1 + s2
                if qb in right:
                    qn.append((q, s1, s2, qb))
                    ext.append((left[q], 1, 1, right[qb]))
                    off.append(pos)
                    pos += left[q] * right[qb]
    return HostDesc(4, qn, ext, off, pos)


def env_desc(bond, qw):
    qn, ext, off, pos = [], [], [], 0
    for q in sorted(bond):
        for w in range(len(qw)):
            qp = q + qw[w]
            if qp in bond:
                qn.append((qp, w, q))
                ext.append((bond[qp], 1, bond[q]))
                off.append(pos)
                pos += bond[qp] * bond[q]
    return HostDesc(3, qn, ext, off, pos)


@pytest.mark.parametrize("cfg", ["cfg1", "cfg2", "cfg3", "cfg5"])
def test_flop_counter_matches_oracle(lib, cfg):
    s = synth.CONFIGS[cfg]
    W, qw = model.bh_mpo(s.nmax, s.J, s.U)
    bonds = synth.chain_bonds(s.L, s.N, s.nmax, s.chi)
    j = s.L // 2
    left, right = bonds[j - 1], bonds[j + 1]
    Ld, Rd, th = env_desc(left, qw), env_desc(right, qw), theta_desc(left, right, s.d)
    mpo = B.Mpo(W, qw)
    parts = np.zeros(3, dtype=np.int64)
    f = lib.tnt_heff2_flops(Ld.ref, mpo.ref, mpo.ref, Rd.ref, th.ref,
                            parts.ctypes.data_as(B.I64P))
    ref = oflops.heff2_flops(left, right, s.d, qw, W, W)
    assert f == ref["total"]
    assert list(parts) == [ref["step1"], ref["mpo"], ref["step4"]]


def test_flop_counter_rejects_charge_violation(lib):
    left, right, d = {2: 3, 3: 2}, {4: 2, 5: 3}, 2
    W, qw = model.bh_mpo(1, 1.0, 1.0)
    th = theta_desc(left, right, d)
    th.qn[3] += 1  # q_b != q_a + s1 + s2 for the first block
    Ld, Rd = env_desc(left, qw), env_desc(right, qw)
    mpo = B.Mpo(W, qw)
    assert lib.tnt_heff2_flops(Ld.ref, mpo.ref, mpo.ref, Rd.ref, th.ref, None) == -1


@pytest.mark.parametrize("nmax,J,U,mu", [(1, 1.0, 0.0, 0.0), (2, 1.0, 2.0, 0.0),
                                         (4, 0.7, 3.3, 0.4)])
def test_library_mpo_equals_oracle_mpo(lib, nmax, J, U, mu):
    # two independent constructions of Eq. (2)'s MPO; the oracle's is pinned to ED
    Wl, ql = B.bose_hubbard_mpo(lib, nmax, J, U, mu)
    Wo, qo = model.bh_mpo(nmax, J, U, mu)
    np.testing.assert_array_equal(Wl, Wo)
    assert list(ql) == list(qo)
    assert (B.MPO_LEFT, B.MPO_RIGHT) == (model.MPO_LEFT, model.MPO_RIGHT)


@pytest.mark.parametrize("J", [1.0, -0.3, 2.5])
def test_library_spin1_mpo_equals_oracle_mpo(lib, J):
    # the oracle's spin-1 MPO is pinned to Kronecker-product Hamiltonians
    Wl, ql = B.spin1_heisenberg_mpo(lib, J)
    Wo, qo = ospin1.mpo(J)
    np.testing.assert_allclose(Wl, Wo, rtol=0, atol=1e-15)
    assert list(ql) == list(qo)
    assert (B.SPIN1_LEFT, B.SPIN1_RIGHT) == (ospin1.MPO_LEFT, ospin1.MPO_RIGHT)


@pytest.mark.parametrize("L,nmax,J,U,mu", [(2, 1, 1.0, 0.0, 0.0), (5, 2, 0.8, 2.5, 0.3),
                                           (4, 4, 1.0, 4.0, -0.2)])
def test_library_bond_hamiltonians_equal_oracle(lib, L, nmax, J, U, mu):
    from oracle import tebd as otebd
    got = B.bond_hamiltonians_bose_hubbard(lib, L, nmax, J, U, mu)
    want = otebd.bond_hamiltonians_bh(L, nmax, J, U, mu)
    np.testing.assert_allclose(got, np.array(want), rtol=0, atol=1e-14)
    got1 = B.bond_hamiltonians_spin1(lib, L, J)
    np.testing.assert_allclose(got1, np.array(otebd.bond_hamiltonians_spin1(L, J)), rtol=0,
                               atol=1e-14)


def test_spin1_mpo_rejects_nonfinite(lib):
    W = np.zeros((5, 5, 3, 3))
    qw = np.zeros(5, np.int32)
    code = lib.tnt_mpo_spin1_heisenberg(float("nan"), W.ctypes.data_as(B.F64P),
                                        qw.ctypes.data_as(B.I32P))
    assert code != 0
    assert lib.tnt_mpo_spin1_heisenberg(1.0, None, None) != 0


@pytest.mark.parametrize("seed", range(6))
def test_trunc_select_matches_oracle(lib, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.ascontiguousarray(np.sort(rng.exponential(size=40) ** 3)[::-1])
    lam[5] = lam[6]  # a tie
    for chi_max, a, r, e, kind in [(10, -1, -1, -1, 0), (100, lam[12], -1, -1, 0),
                                   (100, -1, 1e-2, -1, 0), (100, -1, -1, 0.05, 0),
                                   (7, 0.01, 1e-3, 0.5, 0), (100, -1, -1, 0.05, 1),
                                   (100, -1, -1, 0.5, 2), (100, 1e9, -1, -1, 0)]:
        p = B.TruncParams(chi_max, kind, a, r, e, 1)
        eps = C.c_double()
        got = lib.tnt_trunc_select(lam.ctypes.data_as(B.F64P), len(lam), C.byref(p),
                                   C.byref(eps))
        want = osvd.select_chi(lam, chi_max, a, r, e, kind)
        assert got == want, (chi_max, a, r, e, kind)
        assert eps.value == pytest.approx(osvd.trunc_error(lam[want:], kind), rel=1e-12, abs=1e-300)
