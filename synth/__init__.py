"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no part of the DMRG arithmetic: it only decides block
shapes (how a bond dimension chi is split over U(1) particle-number sectors)
and draws seeded complex-normal numbers into those shapes.  Both the CPU
oracle and the GPU path consume exactly these arrays, so neither side ever
produces the other's inputs.

Shapes follow the paper's U(1) block rule (appendix A.1.1, symmetric nodes):
an element of a site tensor A[a, s, b] is kept only when the incoming charges
match the outgoing one, q(b) = q(a) + s, and the kept elements are stored as
one dense block per charge label.

Conventions (used everywhere in this repository)
- A bond is a dict {q: dim} with ascending q (q = bosons to the left of it).
- A site tensor is a dict {(q_left, s): complex array (dim_left, dim_right)}
  with q_right = q_left + s; the array is row-major [a, b].
- A two-site vector theta is a dict {(q_a, s1, s2): array (dim_a, dim_b)} with
  q_b = q_a + s1 + s2.
- A left environment is a dict {(w, q_a): array (dim(q_a + qw[w]), dim(q_a))}
  (bra index first); a right environment {(u, q_b): array (dim(q_b + qw[u]),
  dim(q_b))}.
- Complex normals: a block of shape (r, c) is standard_normal((r, c, 2))
  mapped to (x + i y)/sqrt(2), so E|z|^2 = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SIGMA = 1.36  # width of the Gaussian sector weights (in bosons)


# ---------------------------------------------------------------------------
# sector shapes
# ---------------------------------------------------------------------------

def count_configs(nsites: int, q: int, nmax: int, cap: int | None = None) -> int:
    """Number of occupation strings of `nsites` sites, each 0..nmax, summing to q.

    Exact integer count (restricted compositions); if `cap` is given the
    result is min(count, cap) (the count can be astronomically large).
    """
    if q < 0 or q > nsites * nmax:
        return 0
    ways = [1] + [0] * q
    for _ in range(nsites):
        new = [0] * (q + 1)
        for tot in range(q + 1):
            acc = 0
            for n in range(0, min(nmax, tot) + 1):
                acc += ways[tot - n]
            new[tot] = acc if cap is None else min(acc, cap)
        ways = new
    return ways[q] if cap is None else min(ways[q], cap)


def config_table(nsites_max: int, qmax: int, nmax: int, cap: int):
    """table[n][q] = min(count_configs(n, q, nmax), cap) for n <= nsites_max, q <= qmax."""
    table = [[1] + [0] * qmax]
    for _ in range(nsites_max):
        prev = table[-1]
        row = [0] * (qmax + 1)
        for tot in range(qmax + 1):
            acc = 0
            for n in range(0, min(nmax, tot) + 1):
                acc += prev[tot - n]
            row[tot] = min(acc, cap)
        table.append(row)
    return table


def bond_sectors(L: int, N: int, nmax: int, ell: int, chi: int,
                 sigma: float = SIGMA, table=None) -> dict[int, int]:
    """Sector dimensions {q: dim} of bond `ell` (0..L) of an L-site chain.

    Recipe: allowed charges are those reachable from both ends; each gets a
    cap c(q) = min(#configs of the left ell sites holding q, #configs of the
    right L-ell sites holding N-q); if sum(c) <= chi the caps are used (exact
    bond), otherwise chi is apportioned by largest remainder over Gaussian
    weights exp(-(q - N ell/L)^2 / (2 sigma^2)), ties to the smaller
    |q - N ell / L| then the smaller q, never above c(q), with the surplus of
    capped sectors redistributed.  Sectors that end with dim 0 are omitted.
    """
    if ell == 0:
        return {0: 1}
    if ell == L:
        return {N: 1}
    qlo = max(0, N - (L - ell) * nmax)
    qhi = min(N, ell * nmax)
    caps = {}
    if table is None:
        table = config_table(L, N, nmax, chi + 1)
    for q in range(qlo, qhi + 1):
        c = min(table[ell][q], table[L - ell][N - q])
        if c > 0:
            caps[q] = c
    if sum(caps.values()) <= chi:
        return dict(sorted(caps.items()))
    centre = N * ell / L
    weight = {q: math.exp(-(q - centre) ** 2 / (2.0 * sigma * sigma)) for q in caps}
    alloc: dict[int, int] = {}
    active = sorted(caps)
    remaining = chi
    while True:
        wsum = sum(weight[q] for q in active)
        quota = {q: remaining * weight[q] / wsum for q in active}
        base = {q: int(math.floor(quota[q])) for q in active}
        leftover = remaining - sum(base.values())
        order = sorted(active, key=lambda q: (-(quota[q] - base[q]), abs(q - centre), q))
        tent = dict(base)
        for q in order[:leftover]:
            tent[q] += 1
        over = [q for q in active if tent[q] > caps[q]]
        if not over:
            alloc.update(tent)
            break
        for q in over:
            alloc[q] = caps[q]
            remaining -= caps[q]
            active.remove(q)
        if not active or remaining <= 0:
            break
    return {q: d for q, d in sorted(alloc.items()) if d > 0}


def chain_bonds(L: int, N: int, nmax: int, chi: int) -> list[dict[int, int]]:
    """Sector dims of bonds 0..L, made mutually consistent.

    A sector on bond ell that cannot be reached from any sector of bond ell-1
    by adding 0..nmax bosons (or cannot reach bond ell+1) would give empty
    blocks; such sectors are dropped, sweeping left to right then right to
    left, so every block of every site tensor is connected.
    """
    table = config_table(L, N, nmax, chi + 1)
    bonds = [bond_sectors(L, N, nmax, ell, chi, table=table) for ell in range(L + 1)]
    changed = True
    while changed:
        changed = False
        for ell in range(1, L + 1):
            keep = {q: d for q, d in bonds[ell].items()
                    if any((q - s) in bonds[ell - 1] for s in range(nmax + 1))}
            if keep != bonds[ell]:
                bonds[ell] = keep
                changed = True
        for ell in range(L - 1, -1, -1):
            keep = {q: d for q, d in bonds[ell].items()
                    if any((q + s) in bonds[ell + 1] for s in range(nmax + 1))}
            if keep != bonds[ell]:
                bonds[ell] = keep
                changed = True
    return bonds


# ---------------------------------------------------------------------------
# seeded complex blocks
# ---------------------------------------------------------------------------

def _cnormal(rng: np.random.Generator, shape) -> np.ndarray:
    x = rng.standard_normal(tuple(shape) + (2,))
    return (x[..., 0] + 1j * x[..., 1]) / math.sqrt(2.0)


def site_keys(left: dict[int, int], right: dict[int, int], d: int):
    """Block keys (q_left, s) of a site tensor, in storage order."""
    return [(q, s) for q in left for s in range(d) if (q + s) in right]


def theta_keys(left: dict[int, int], right: dict[int, int], d: int):
    """Block keys (q_a, s1, s2) of a two-site vector, in storage order."""
    return [(q, s1, s2) for q in left for s1 in range(d) for s2 in range(d)
            if (q + s1 + s2) in right]


def env_keys(bond: dict[int, int], qw):
    """Block keys (w, q) of an environment on `bond`, in storage order."""
    return [(w, q) for q in bond for w in range(len(qw)) if (q + qw[w]) in bond]


def random_mps(L: int, N: int, nmax: int, chi: int, seed: int):
    """Seeded random (not canonical) block MPS.

    Returns (bonds, sites): bonds[0..L] sector dicts and sites[0..L-1] block
    dicts (sites[j-1] is site j).  Fill order: sites 1..L, blocks ascending
    (q_left, s), one complex-normal draw per block.
    """
    d = nmax + 1
    bonds = chain_bonds(L, N, nmax, chi)
    rng = np.random.Generator(np.random.PCG64(seed))
    sites = []
    for j in range(1, L + 1):
        left, right = bonds[j - 1], bonds[j]
        blocks = {}
        for (q, s) in site_keys(left, right, d):
            blocks[(q, s)] = _cnormal(rng, (left[q], right[q + s]))
        sites.append(blocks)
    return bonds, sites


def product_mps(config):
    """Product state |n_1 ... n_L> as a block MPS: every bond one sector of
    dimension 1 (the charge to its left), every site one 1 x 1 block = 1."""
    bonds, q = [{0: 1}], 0
    sites = []
    for s in config:
        sites.append({(q, int(s)): np.ones((1, 1), dtype=complex)})
        q += int(s)
        bonds.append({q: 1})
    return bonds, sites


def random_theta(left, right, d, rng):
    return {k: _cnormal(rng, (left[k[0]], right[k[0] + k[1] + k[2]]))
            for k in theta_keys(left, right, d)}


def random_env(bond, qw, rng, hermitian_pairs=None):
    """Random environment blocks {(w, q): (dim(q+qw[w]), dim(q))}.

    With `hermitian_pairs` (a list pairing each MPO bond index with its
    adjoint partner, e.g. [0, 2, 1, 3]), the draw is symmetrised so that
    block (w, q) equals the conjugate transpose of block (pair[w], q+qw[w]);
    an effective Hamiltonian built from such environments is Hermitian when
    the MPO pairs its bond indices the same way.
    """
    env = {k: _cnormal(rng, (bond[k[1] + qw[k[0]]], bond[k[1]])) for k in env_keys(bond, qw)}
    if hermitian_pairs is not None:
        out = {}
        for (w, q), blk in env.items():
            pw = hermitian_pairs[w]
            partner = env[(pw, q + qw[w])]
            out[(w, q)] = 0.5 * (blk + partner.conj().T)
        env = out
    return env


# ---------------------------------------------------------------------------
# workload table
# ---------------------------------------------------------------------------

@dataclass
class ChainSpec:
    L: int
    N: int
    nmax: int
    J: float
    U: float
    mu: float
    chi: int
    seed: int
    sweeps: int = 1
    lanczos_steps: int = 20
    rel_cutoff: float = 1e-12
    extra: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return self.nmax + 1


CONFIGS = {
    # small FP64 case checked against exact diagonalisation
    "cfg1": ChainSpec(L=8, N=8, nmax=2, J=1.0, U=2.0, mu=0.0, chi=16, seed=1, sweeps=2),
    # mid-size chain: single matvec + one sweep, FP64 vs FP32
    "cfg2": ChainSpec(L=32, N=32, nmax=4, J=1.0, U=4.0, mu=0.0, chi=256, seed=2, sweeps=1),
    # chi = 1024 chain (superfluid .. Mott); same MPS for every U
    "cfg3": ChainSpec(L=64, N=64, nmax=4, J=1.0, U=3.3, mu=0.0, chi=1024, seed=3, sweeps=4,
                      extra={"U_list": [2.0, 3.3, 6.0]}),
    # large bond
    "cfg5": ChainSpec(L=128, N=128, nmax=4, J=1.0, U=3.3, mu=0.0, chi=2048, seed=5, sweeps=2),
}


def batched_specs(seed: int = 4, n: int = 64):
    """The many-chain workload: n independent chains drawn from `seed`.

    In order from one PCG64 stream: L ~ integers(16, 65), U/J ~ uniform(1, 8),
    chi ~ choice([64, 128, 256, 384]); N = L, nmax = 4, chain i's MPS seed is
    1000*seed + i.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = rng.integers(16, 65, n)
    Us = rng.uniform(1.0, 8.0, n)
    chis = rng.choice([64, 128, 256, 384], n)
    return [ChainSpec(L=int(Ls[i]), N=int(Ls[i]), nmax=4, J=1.0, U=float(Us[i]), mu=0.0,
                      chi=int(chis[i]), seed=1000 * seed + i) for i in range(n)]


def middle_bond_inputs(spec: ChainSpec, qw, seed_offset: int = 0, hermitian_pairs=None):
    """Seeded (left bond, right bond, L env, R env, theta) at the middle bond j = L/2.

    theta lives on sites j, j+1 (left bond j-1, right bond j+1); the shapes
    are those of the sector recipe at the spec's chi.  Used for single-matvec
    parity and timing.
    """
    bonds = chain_bonds(spec.L, spec.N, spec.nmax, spec.chi)
    j = spec.L // 2
    left, right = bonds[j - 1], bonds[j + 1]
    rng = np.random.Generator(np.random.PCG64(spec.seed * 7919 + 17 + seed_offset))
    Lenv = random_env(left, qw, rng, hermitian_pairs)
    Renv = random_env(right, qw, rng, hermitian_pairs)
    theta = random_theta(left, right, spec.d, rng)
    return left, right, Lenv, Renv, theta
