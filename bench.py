#!/usr/bin/env python3
"""Benchmark of the two-site DMRG hot path on one MI355X.

One step = one full two-site sweep (right pass + left pass over every bond:
theta formation, Lanczos with H_eff matvecs, truncated SVD, environment
update) of a Bose-Hubbard chain, on device-resident state.  The headline
`value` is the H_eff matvec throughput of the whole timed sweeps:
algorithmic flops of every matvec the sweeps performed / timed wall time.

Default workload: the chi = 1024 chain, L = 64, N = 64, nmax = 4 (d = 5),
J = 1, U = 3.3 (seeded random MPS, seed 3), matvecs on FP32 MFMA; Krylov
vectors, SVD, energies and environments in FP64.  The energy after sweep k
(k = the number of sweeps the oracle's stored run has) is compared with the
oracle's.  Also reported: two sweeps each on the FP64 and the BF16x3 GPU
paths from the same initial state, single-matvec rates at the middle bond,
the 64-chain batch, the grouped-GEMM roofline figure and the CPU oracle
(block matvec single-threaded and on all cores, plus its sweep time from the
stored run).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2-site H_eff matvec TFLOP/s + sweep time: FP32-MFMA vs FP64, |ΔE/E|<=1e-9"
PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0}
# MPO bond index pairs (w, w') exchanged by Hermitian conjugation of the
# Bose-Hubbard MPO (b and b^dagger channels): random environments drawn with
# this symmetry give a Hermitian H_eff
HERM_PAIRS = [0, 2, 1, 3]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_chain(tnt, B, spec):
    import synth
    W, qw = tnt.bose_hubbard_mpo(spec.nmax, spec.J, spec.U, spec.mu)
    bonds, sites = synth.random_mps(spec.L, spec.N, spec.nmax, spec.chi, spec.seed)
    mps = tnt.mps(bonds, sites, spec.d)
    mps.right_canonicalize()
    env = B.Env(tnt, mps, [W] * spec.L, qw, B.MPO_LEFT, B.MPO_RIGHT)
    return mps, env


class Roctx:
    """roctx range around the timed region (the profiler SDK's roctx library,
    which rocprofv3 --marker-trace records; a no-op without it)."""

    def __init__(self):
        import ctypes
        self.lib = None
        for p in ("/opt/rocm/lib/librocprofiler-sdk-roctx.so", "librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(p)
                self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                break
            except OSError:
                continue

    def push(self, name):
        if self.lib:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib:
            self.lib.roctxRangePop()


TIMED_RANGE = "tnt_bench_timed"


def run_sweeps(tnt, torch, mps, env, spec, precision, warmup, steps, roctx=None, energies=None,
               stats=None):
    """W untimed then K timed sweeps; `energies` (a list) gets every sweep's
    final energy and `stats` every sweep's result, warm-up sweeps included,
    in order."""
    kw = dict(kmax=spec.lanczos_steps, precision=precision, rel_tol=spec.rel_cutoff)
    for i in range(warmup):
        r = tnt.sweep(mps, env, spec.chi, **kw)
        if energies is not None:
            energies.append(r["energy"])
        if stats is not None:
            stats.append(r)
        log(f"  warmup sweep {i + 1} [{precision}]: E = {r['energy']:.12f} ({r['seconds_total']:.2f}s)")
    torch.cuda.synchronize()
    if roctx:
        roctx.push(TIMED_RANGE)
    t0 = time.perf_counter()
    res = []
    for i in range(steps):
        # tnt_dmrg_sweep returns when its sweep is done; one progress line per
        # sweep (a long timed region must not look silent)
        r = tnt.sweep(mps, env, spec.chi, **kw)
        res.append(r)
        log(f"  timed sweep {i + 1} [{precision}]: E = {r['energy']:.12f} ({r['seconds_total']:.2f}s)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if roctx:
        roctx.pop()
    for r in res:
        if energies is not None:
            energies.append(r["energy"])
        if stats is not None:
            stats.append(r)
    return res, dt


def reference_schedule_flops(left, right, d, W, qw):
    """F_alg of the unpruned contraction order (Sec. 4.2, Fig. mpspmpomps):
    step 1 for every (w, theta block) whose L block exists, W1 and W2 as two
    separate real-times-complex passes over every slab they produce, step 4
    for every produced slab whose output block is allowed and whose R block
    exists.  8 flops per complex multiply-add, 4 per real-times-complex term
    and element.  The library's own count (tnt_heff2_flops) prunes slabs that
    reach no output and combines W1 W2 into one pass, so it is a few percent
    lower; both are reported."""
    import numpy as np
    W = np.asarray(W)
    D = len(qw)
    theta = [(qa, s1, s2) for qa in sorted(left) for s1 in range(d) for s2 in range(d)
             if qa + s1 + s2 in right]
    nz = [(w, v, sp, s) for w in range(D) for v in range(D) for sp in range(d) for s in range(d)
          if W[w, v, sp, s] != 0]
    f1 = fm = f4 = 0
    t1 = set()
    for qa, s1, s2 in theta:
        qb = qa + s1 + s2
        for w in range(D):
            qap = qa + qw[w]
            if qap in left:
                f1 += 8 * left[qap] * left[qa] * right[qb]
                t1.add((w, qap, s1, s2, qb))
    t2 = set()
    for w, qap, s1, s2, qb in t1:   # T2[v] = sum_{w, s1} W1[w, v, s1', s1] T1[w]
        for ww, v, s1p, ss in nz:
            if ww == w and ss == s1:
                fm += 4 * left[qap] * right[qb]
                t2.add((v, qap, s1p, s2, qb))
    t3 = set()
    for v, qap, s1p, s2, qb in t2:  # T3[u] = sum_{v, s2} W2[v, u, s2', s2] T2[v]
        for vv, u, s2p, ss in nz:
            if vv == v and ss == s2:
                fm += 4 * left[qap] * right[qb]
                t3.add((u, qap, s1p, s2p, qb))
    for u, qap, s1p, s2p, qb in t3:
        qbp = qap + s1p + s2p
        if qbp in right and qb == qbp - qw[u]:
            f4 += 8 * left[qap] * right[qb] * right[qbp]
    return {"step1": f1, "mpo": fm, "step4": f4, "total": f1 + fm + f4}


def matvec_rates(tnt, B, torch, spec, precs=("fp64", "fp32", "bf16x3"), reps=20):
    """Single H_eff applications at the middle bond (seeded synthetic L, R,
    theta): `reps` back-to-back tnt_heff2_apply calls between two events on
    the library's stream (torch's current stream), per precision."""
    import synth
    W, qw = tnt.bose_hubbard_mpo(spec.nmax, spec.J, spec.U, spec.mu)
    left, right, Le, Re, th = synth.middle_bond_inputs(spec, qw)
    mpo = B.Mpo(W, qw)
    Ld, Rd, td = tnt.env(Le, qw), tnt.env(Re, qw), tnt.theta(th)
    out = tnt.theta_like(td)
    flops, parts = tnt.heff2_flops(Ld, mpo, mpo, Rd, td)
    f_ref = reference_schedule_flops(left, right, spec.d, W, qw)["total"]
    rates = {}
    for prec in precs:
        for _ in range(3):   # plan, tile-shape tuning, warm caches
            tnt.heff2_apply(Ld, mpo, mpo, Rd, td, out, prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            tnt.heff2_apply(Ld, mpo, mpo, Rd, td, out, prec)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        rates[prec] = {"s": t, "tflops": flops / t / 1e12,
                       "frac_fp32_peak": flops / t / 1e12 / PEAK["fp32"],
                       "tflops_reference_schedule": f_ref / t / 1e12}
    del Ld, Rd, td, out
    return {"chi": spec.chi, "bond": f"middle bond of L={spec.L}",
            "flops": int(flops), "parts": [int(x) for x in parts],
            "flops_reference_schedule": int(f_ref), **rates}


def batched_sweep(tnt, B, torch, precision="fp32"):
    """The 64-chain workload, whole sweeps: one lockstep sweep of every chain
    through the batched path (tnt_dmrg_sweep_batched: one merged H_eff
    operator and one Lanczos recurrence per step, the sector eigensolves of
    all chains of a step in shared batched calls) against the same sweep run
    chain by chain; both start from the same seeded states and follow one
    warm-up sweep."""
    import synth
    specs = synth.batched_specs(4)
    kw = dict(kmax=specs[0].lanczos_steps, precision=precision, rel_tol=specs[0].rel_cutoff)
    chis = [s.chi for s in specs]

    def build():
        return [make_chain(tnt, B, s) for s in specs]

    chains = build()
    ms, es = [c[0] for c in chains], [c[1] for c in chains]
    tnt.sweep_batched(ms, es, chis, **kw)
    torch.cuda.synchronize()
    log("  warm-up lockstep sweep done")
    t0 = time.perf_counter()
    rb = tnt.sweep_batched(ms, es, chis, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"  timed lockstep sweep: {t_batch:.2f}s")
    del chains, ms, es
    chains = build()
    for (m, e), s in zip(chains, specs):
        tnt.sweep(m, e, s.chi, **kw)
    torch.cuda.synchronize()
    log("  warm-up chain-by-chain sweeps done")
    t0 = time.perf_counter()
    rs = [tnt.sweep(m, e, s.chi, **kw) for (m, e), s in zip(chains, specs)]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    log(f"  timed chain-by-chain sweeps: {t_single:.2f}s")
    del chains
    flops = sum(r["matvec_flops"] for r in rb)
    per = {k: sum(r[k] for r in rb) / len(rb) for k in
           ("seconds_svd", "seconds_lanczos", "seconds_matvec", "seconds_setup")}
    return {"workload": f"{len(specs)} chains (batched_specs seed 4), one sweep each, "
                        "second sweep from seeded random states",
            "precision": precision, "bond_updates": int(sum(r["updates"] for r in rb)),
            "batched_sweep_s": t_batch, "chain_by_chain_sweeps_s": t_single,
            "batching_speedup": t_single / t_batch,
            "batched_matvec_tflops": flops / t_batch / 1e12,
            "batched_breakdown_s": per,
            "max_rel_dE_batched_vs_single": max(abs(a["energy"] - b["energy"]) / abs(b["energy"])
                                                for a, b in zip(rb, rs))}


def batched_lockstep_vs_oracle(tnt, B, torch, precision="fp32", sweeps=4):
    """The 64-chain workload swept `sweeps` times in lockstep
    (tnt_dmrg_sweep_batched) from its seeded states; the chains with a stored
    oracle run (one per chi class) are compared with the oracle's energy
    after the same number of sweeps."""
    import synth
    specs = synth.batched_specs(4)
    kw = dict(kmax=specs[0].lanczos_steps, precision=precision, rel_tol=specs[0].rel_cutoff)
    chains = [make_chain(tnt, B, s) for s in specs]
    ms, es = [c[0] for c in chains], [c[1] for c in chains]
    times = []
    res = None
    for _ in range(sweeps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = tnt.sweep_batched(ms, es, [s.chi for s in specs], **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"  lockstep sweep {len(times)} of {len(specs)} chains: {times[-1]:.2f}s")
    del chains, ms, es
    per_chain = {}
    for f in sorted(os.listdir(os.path.join(ROOT, "tests", "golden"))):
        if not (f.startswith("sweep_cfg4_chain") and f.endswith(".json")):
            continue
        i = int(f[len("sweep_cfg4_chain"):-len(".json")])
        with open(os.path.join(ROOT, "tests", "golden", f)) as fh:
            g = json.load(fh)
        if len(g["sweeps"]) < sweeps:
            continue
        e_ref = g["sweeps"][sweeps - 1]["E"][-1]
        e = res[i]["energy"]
        per_chain[str(i)] = {"L": specs[i].L, "chi": specs[i].chi, "gpu": e, "oracle": e_ref,
                             "rel_err": abs(e - e_ref) / abs(e_ref)}
    return {"sweeps": sweeps, "precision": precision, "sweep_s": times,
            "bond_updates_per_sweep": int(sum(r["updates"] for r in res)),
            "matvec_tflops_last_sweep": sum(r["matvec_flops"] for r in res) / times[-1] / 1e12,
            "vs_oracle": per_chain,
            "max_rel_err_vs_oracle": max((v["rel_err"] for v in per_chain.values()),
                                         default=None)}


def spin1_sweeps(tnt, B, torch, precisions=("fp32", "fp64"), steps=2):
    """The DMRG timing workload of the paper's Sec. 3 table: spin-1
    Heisenberg chain, L = 101, chi = 200, U(1) blocks (S^z = 0 is total
    charge L with s = S^z + 1), from a seeded random MPS; one warm-up sweep,
    then `steps` timed sweeps per matvec precision."""
    import synth
    L, chi, kmax = 101, 200, 20
    W, qw = tnt.spin1_heisenberg_mpo(1.0)
    out = {"workload": f"spin-1 Heisenberg open chain L={L}, S^z=0, chi={chi}, "
                       f"Lanczos kmax={kmax}, seeded random MPS (seed 5)",
           "paper_s_per_sweep": {"cpu_mkl_nag": 135.0, "gpu_magma_k40": 161.0,
                                 "cpu_arpack": 377.0}}
    kw = dict(kmax=kmax, rel_tol=1e-12)
    for prec in precisions:
        bonds, sites = synth.random_mps(L, L, 2, chi, 5)
        mps = tnt.mps(bonds, sites, 3)
        mps.right_canonicalize()
        env = B.Env(tnt, mps, [W] * L, qw, B.SPIN1_LEFT, B.SPIN1_RIGHT)
        r0 = tnt.sweep(mps, env, chi, precision=prec, **kw)
        log(f"  spin-1 warm-up sweep [{prec}]: E = {r0['energy']:.12f}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = [tnt.sweep(mps, env, chi, precision=prec, **kw) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        r = rs[-1]
        out[prec] = {"s_per_sweep": dt, "energy": r["energy"],
                     "energy_per_bond": r["energy"] / (L - 1),
                     "max_chi": int(max(r["bond_chi"])), "max_eps": float(max(r["bond_eps"])),
                     "breakdown_s": {k: r[k] for k in ("seconds_svd", "seconds_lanczos",
                                                       "seconds_matvec", "seconds_setup",
                                                       "seconds_theta", "seconds_env")},
                     "speedup_vs_paper_cpu": 135.0 / dt}
        log(f"  spin-1 [{prec}]: {dt:.3f} s/sweep, E = {r['energy']:.12f}")
        del mps, env
    return out


def observables_pass(tnt, B, torch, spec, reps=3):
    """rho_ij = <b^dagger_i b_j> for every pair (and <n_j>) of the chain's
    state after one sweep from the seeded random MPS: one
    tnt_mps_correlation pass, timed `reps` times after a warm-up call."""
    import numpy as np
    mps, env = make_chain(tnt, B, spec)
    tnt.sweep(mps, env, spec.chi, kmax=spec.lanczos_steps, precision="fp32",
              rel_tol=spec.rel_cutoff)
    b = np.zeros((spec.d, spec.d))
    for n in range(1, spec.d):
        b[n - 1, n] = n ** 0.5
    rho, flops = mps.correlation(b, -1, with_flops=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rho, flops = mps.correlation(b, -1, with_flops=True)
    dt = (time.perf_counter() - t0) / reps
    return {"workload": f"rho_ij and <n_j> of the L={spec.L}, chi={spec.chi} Bose-Hubbard state "
                        "after one sweep", "seconds": dt, "gflop": flops / 1e9,
            "tflops": flops / dt / 1e12, "trace_rho": float(np.trace(rho).real),
            "max_chi": max(sum(b.values()) for b in mps.bonds())}


def tebd_steps(tnt, B, torch):
    """TEBD time steps (second-order: every bond gated twice per step).
    (1) The timing-table shape: spin-1 Heisenberg, L = 101, chi = 1000, from
    a seeded random MPS of that bond dimension (right-canonicalised), one
    warm-up step and one timed step.  (2) The time-evolution example: hard-
    core bosons, L = 51, CDW of 25 bosons, dt = 0.01, chi = 200, 100 steps."""
    import synth
    out = {"paper_s_per_step_u1": {"mkl_nag_magma": 59.0, "mkl_nag": 57.0, "mkl_arpack": 73.0}}
    L, chi = 101, 1000
    h = tnt.bond_hamiltonians_spin1(L)
    bonds, sites = synth.random_mps(L, L, 2, chi, 6)
    mps = tnt.mps(bonds, sites, 3)
    mps.right_canonicalize()
    r0 = tnt.tebd_step(mps, h, 0.01, chi, rel_tol=-1.0)
    log(f"  spin-1 TEBD warm-up step: {r0['seconds_total']:.2f} s, max chi {r0['max_chi']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = tnt.tebd_step(mps, h, 0.01, chi, rel_tol=-1.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["spin1_L101_chi1000"] = {"s_per_step": dt, "seconds_svd": r["seconds_svd"],
                                 "seconds_theta_gate": r["seconds_gate"],
                                 "max_chi": r["max_chi"], "sum_eps": r["sum_eps"],
                                 "gates_per_step": 2 * (L - 1),
                                 "speedup_vs_paper_u1_best": 57.0 / dt}
    log(f"  spin-1 TEBD step: {dt:.2f} s")
    del mps
    L = 51
    h = tnt.bond_hamiltonians_bose_hubbard(L, 1, 1.0, 0.0)
    for name, rel in (("chi_only", -1.0), ("rel_cut_1e-12", 1e-12)):
        bonds, sites = synth.product_mps(tuple(j % 2 for j in range(L)))
        mps = tnt.mps(bonds, sites, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eps = 0.0
        for step in range(100):
            r = tnt.tebd_step(mps, h, 0.01, 200, rel_tol=rel, renormalise=False)
            eps += r["sum_eps"]
            if (step + 1) % 20 == 0:
                log(f"  hard-core CDW ({name}): step {step + 1}, chi {r['max_chi']}")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"hardcore_cdw_L51_chi200_{name}"] = {"s_per_step": dt / 100, "steps": 100,
                                                  "max_chi_at_t1": r["max_chi"],
                                                  "accumulated_eps": eps}
        log(f"  hard-core CDW ({name}): {dt / 100 * 1e3:.1f} ms per step, chi {r['max_chi']}")
        del mps
    return out


def heff1_rates(tnt, B, torch, spec, reps=20):
    """One-site H_eff . A (tnt_heff1_apply, FP64) at the middle site of the
    chain's sector recipe: seeded random environments and site tensor.
    Each call builds its task lists on the host and synchronises, so the
    per-call time includes that host work; algorithmic flops counted from
    the block structure (8 real flops per complex MAC)."""
    import numpy as np
    import synth
    W, qw = tnt.bose_hubbard_mpo(spec.nmax, spec.J, spec.U, spec.mu)
    bonds = synth.chain_bonds(spec.L, spec.N, spec.nmax, spec.chi)
    j = spec.L // 2
    left, right = bonds[j - 1], bonds[j]
    rng = np.random.Generator(np.random.PCG64(spec.seed * 7919 + 29))
    Lenv = synth.random_env(left, qw, rng, HERM_PAIRS)
    Renv = synth.random_env(right, qw, rng, HERM_PAIRS)
    A = {k: rng.normal(size=(left[k[0]], right[k[0] + k[1]])) + 0j
         for k in synth.site_keys(left, right, spec.d)}
    D, d = len(qw), spec.d
    flops, ykeys = 0.0, {}
    for (qa, s), a in A.items():
        for w in range(D):
            if (w, qa) in Lenv:
                flops += 8.0 * Lenv[(w, qa)].shape[0] * a.shape[1] * a.shape[0]
                for u in range(D):
                    for sp in range(d):
                        if W[w, u, sp, s] != 0.0:
                            ykeys[(u, qa + qw[w], sp)] = a.shape[1]
    for (u, qap, sp), K in ykeys.items():
        if (qap, sp) in A and (u, qap + sp - qw[u]) in Renv:
            flops += 8.0 * A[(qap, sp)].shape[0] * A[(qap, sp)].shape[1] * K
    mpo = B.Mpo(W, qw)
    Ld, Rd, Ad = tnt.env(Lenv, qw), tnt.env(Renv, qw), tnt.site(A)
    out = tnt.site_like(Ad)
    tnt.heff1_apply(Ld, mpo, Rd, Ad, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tnt.heff1_apply(Ld, mpo, Rd, Ad, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"workload": f"one-site H_eff at site {j} of the L={spec.L}, chi={spec.chi} recipe",
            "seconds_per_call": dt, "gflop": flops / 1e9, "tflops_fp64": flops / dt / 1e12,
            "site_elems": int(sum(a.size for a in A.values()))}


def autoblock_svd_rates(tnt, B, torch, reps=3):
    """Truncated SVD of a 3000 x 3000 complex matrix whose block structure
    (20 blocks of 60..240 rows and columns) is hidden by random row and column
    permutations: tnt_auto_block_svd against torch.linalg.svd of the whole
    matrix (the unblocked library SVD)."""
    import numpy as np
    rng = np.random.default_rng(7)
    sizes = [(int(a), int(b)) for a, b in zip(rng.integers(60, 240, 20), rng.integers(60, 240, 20))]
    m, n = sum(a for a, _ in sizes), sum(b for _, b in sizes)
    M = np.zeros((m, n), complex)
    r = c = 0
    for a, b in sizes:
        M[r:r + a, c:c + b] = rng.normal(size=(a, b)) + 1j * rng.normal(size=(a, b))
        r += a
        c += b
    M = M[rng.permutation(m)][:, rng.permutation(n)]
    chi = min(m, n)
    tnt.auto_block_svd(M, 1e-12, chi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        got = tnt.auto_block_svd(M, 1e-12, chi)
    torch.cuda.synchronize()
    t_auto = (time.perf_counter() - t0) / reps
    Md = torch.from_numpy(M).to("cuda")
    torch.linalg.svdvals(Md)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.linalg.svd(Md, full_matrices=False)
    torch.cuda.synchronize()
    t_dense = (time.perf_counter() - t0) / reps
    return {"workload": f"{m} x {n} complex, 20 hidden blocks, all singular values kept "
                        "(host round trip of the input and factors included for auto-blocking)",
            "auto_block_s": t_auto, "dense_library_svd_s": t_dense,
            "speedup": t_dense / t_auto, "nblocks": got["nblocks"], "chi": got["chi"]}


def batched_rates(tnt, B, torch, precision="fp32", reps=10):
    """The 64-chain workload (L 16..64, chi 64..384, seeded) at every chain's
    middle bond: one batched H_eff application over all chains, the same 64
    applications one by one, and one batched Lanczos ground-state solve
    (20 steps + FP64 refinement), eager and replayed from a HIP graph."""
    import synth
    specs = synth.batched_specs(4)
    mpos, Ls, Rs, ths, thetas, outs = [], [], [], [], [], []
    flops = 0
    for s in specs:
        W, qw = tnt.bose_hubbard_mpo(s.nmax, s.J, s.U, s.mu)
        left, right, Le, Re, th = synth.middle_bond_inputs(s, qw, hermitian_pairs=HERM_PAIRS)
        mpo = B.Mpo(W, qw)
        Ld, Rd, td = tnt.env(Le, qw), tnt.env(Re, qw), tnt.theta(th)
        mpos.append(mpo)
        Ls.append(Ld)
        Rs.append(Rd)
        ths.append(th)
        thetas.append(td)
        outs.append(tnt.theta_like(td))
        flops += tnt.heff2_flops(Ld, mpo, mpo, Rd, td)[0]

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / n

    t_batch = timed(lambda: tnt.heff2_apply_batched(Ls, mpos, mpos, Rs, thetas, outs, precision),
                    reps)

    def one_by_one():
        for i in range(len(specs)):
            tnt.heff2_apply(Ls[i], mpos[i], mpos[i], Rs[i], thetas[i], outs[i], precision)

    t_single = timed(one_by_one, max(1, reps // 2))

    def lanczos():
        tds = [tnt.theta(th) for th in ths]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = tnt.lanczos_ground_batched(Ls, mpos, mpos, Rs, tds, kmax=20, precision=precision)
        return time.perf_counter() - t0, r

    lanczos()  # plans, tile tuning
    t_eager, r_eager = lanczos()
    tnt.set_graphs(True)
    try:
        lanczos()  # records the graph
        t_graph, r_graph = lanczos()
    finally:
        tnt.set_graphs(False)
    same = all(a["E"] == b["E"] for a, b in zip(r_eager, r_graph))
    chis = {}
    for s in specs:
        chis[s.chi] = chis.get(s.chi, 0) + 1
    return {"workload": f"{len(specs)} chains, L {min(s.L for s in specs)}..{max(s.L for s in specs)}, "
                        f"chi counts {dict(sorted(chis.items()))}, middle bonds, seeded",
            "precision": precision, "flops_per_batched_matvec": int(flops),
            "batched_matvec_s": t_batch, "batched_matvec_tflops": flops / t_batch / 1e12,
            "one_by_one_matvecs_s": t_single, "batching_speedup": t_single / t_batch,
            "batched_lanczos_eager_s": t_eager, "batched_lanczos_graph_s": t_graph,
            "graph_energies_equal_eager": bool(same),
            "lanczos_matvec_tflops_graph": 21 * flops / t_graph / 1e12}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(spec, config, budget_s=10.0):
    """The oracle's block H_eff at the middle bond, repeated for ~budget_s
    seconds on all of the host's BLAS threads and again single-threaded, plus
    the oracle's sweep time at this configuration from its stored run."""
    import synth
    from oracle import flops as oflops
    from oracle import heff as oheff
    from oracle import model
    W, qw = model.bh_mpo(spec.nmax, spec.J, spec.U, spec.mu)
    left, right, Le, Re, th = synth.middle_bond_inputs(spec, qw)
    f = oflops.heff2_flops(left, right, spec.d, qw, W, W)["total"]

    def timed(budget):
        n, t0 = 0, time.perf_counter()
        while True:
            oheff.heff2_block(Le, W, W, Re, th, left, right, qw, spec.d)
            n += 1
            if time.perf_counter() - t0 >= budget:
                break
        return n, time.perf_counter() - t0

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count() or 1
    n, dt = timed(budget_s)
    out = {"value": f * n / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} block H_eff matvecs (oracle, complex128 NumPy) at the middle bond of "
                     f"the same chain, {dt:.1f}s, {cores} BLAS threads",
           "cpu_model": cpu_model(), "flops_per_matvec": f}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, dt1 = timed(budget_s)
        out["single_thread"] = {"value": f * n1 / dt1 / 1e12, "matvecs": n1, "seconds": dt1}
    g = golden(config)
    if g is not None and g["sweeps"]:
        walls = [s_["wall_s"] for s_ in g["sweeps"] if "wall_s" in s_]
        if walls:
            out["oracle_sweep_s"] = {"per_sweep": walls, "host": g.get("host"),
                                     "note": "the oracle's own two-site sweeps (block mode) at "
                                             "this configuration, from its stored run"}
    return out


def traffic_for(config, precision):
    """HBM bytes per grouped-GEMM launch of this workload from the committed
    PMC summary, if the kernel source is unchanged since the counters were
    taken (else None)."""
    path = os.path.join(ROOT, "profiles", "gemm_traffic.json")
    src = os.path.join(ROOT, "paper_1610_02244_amd", "csrc", "gemm_packed.hip")
    try:
        with open(path) as f:
            t = json.load(f)
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
        if t.get("gemm_packed_hip_sha256") != h:
            return None
        return t.get("workloads", {}).get(config, {}).get(precision, {}).get("bytes_per_launch")
    except Exception:
        return None


def summarize_trace(root):
    """Per-kernel statistics of the dispatches inside the timed roctx range,
    from the CSV files of `rocprofv3 --kernel-trace --marker-trace
    --output-format csv -d ROOT`."""
    import csv
    kfiles, mfiles = [], []
    for dp, _, fs in os.walk(root):
        for f in fs:
            if f.endswith("kernel_trace.csv"):
                kfiles.append(os.path.join(dp, f))
            elif f.endswith("marker_api_trace.csv"):
                mfiles.append(os.path.join(dp, f))
    t0 = t1 = None
    for mf in mfiles:
        with open(mf) as f:
            for row in csv.DictReader(f):
                if any(TIMED_RANGE in str(v) for v in row.values()):
                    t0, t1 = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
    if t0 is None:
        raise SystemExit("timed roctx range not found in the marker trace")
    stats = {}
    for kf in kfiles:
        with open(kf) as f:
            for row in csv.DictReader(f):
                s, e = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
                if s < t0 or e > t1:
                    continue
                st = stats.setdefault(row["Kernel_Name"], [0, 0])
                st[0] += 1
                st[1] += e - s
    top = sorted(stats.items(), key=lambda kv: -kv[1][1])
    gemm = [(k, v) for k, v in stats.items() if "packed_gemm_kernel<0" in k]
    gc = sum(v[0] for _, v in gemm)
    gt = sum(v[1] for _, v in gemm)
    return {"range_ns": t1 - t0, "kernel_ns_total": sum(v[1] for v in stats.values()),
            "fp32_packed_gemm": {"launches": gc, "total_ns": gt,
                                  "avg_ns": gt / gc if gc else None},
            "top": [{"kernel": k[:160], "calls": v[0], "total_ms": v[1] / 1e6,
                     "avg_us": v[1] / v[0] / 1e3} for k, v in top[:25]]}


def pmc_traffic(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir,
                kernel_prefix="tnt::packed_gemm_kernel<0,"):
    """HBM bytes per launch of the dominant kernel from `rocprofv3 --pmc
    FETCH_SIZE` and `--pmc WRITE_SIZE` runs (CSV output directories): the
    per-dispatch averages over every dispatch whose name starts with
    kernel_prefix, each counter scaled so that the same counter reads the
    known size of a plain device copy (bench.py --calibrate-copy runs)."""
    import csv

    def rows(root, counter):
        out = []
        for dp, _, fs in os.walk(root):
            for f in fs:
                if f.endswith("counter_collection.csv"):
                    with open(os.path.join(dp, f)) as fh:
                        for r in csv.DictReader(fh):
                            if r["Counter_Name"] == counter:
                                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return out

    def factor(root, counter):
        vals = [v for k, v in rows(root, counter) if "copyBuffer" in k]
        if not vals:
            raise SystemExit(f"no copy kernel in the calibration run {root}")
        return (64 * 1024 * 1024 * 4 / 1024) / (sum(vals) / len(vals))

    res = {}
    for name, root, cal, counter in (("fetch", fetch_dir, cal_fetch_dir, "FETCH_SIZE"),
                                     ("write", write_dir, cal_write_dir, "WRITE_SIZE")):
        vals = [v for k, v in rows(root, counter)
                if k.replace("void ", "").startswith(kernel_prefix)]
        f = factor(cal, counter)
        res[name] = {"dispatches": len(vals), "kib_per_dispatch_raw": sum(vals) / len(vals),
                     "scale": f, "bytes_per_launch": sum(vals) / len(vals) * 1024 * f}
    res["bytes_per_launch"] = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    with open(os.path.join(ROOT, "paper_1610_02244_amd", "csrc", "gemm_packed.hip"), "rb") as fh:
        res["gemm_packed_hip_sha256"] = hashlib.sha256(fh.read()).hexdigest()
    return res


def mfma_util(root, simds=1024, xcds=8):
    """MFMA utilisation per kernel from a `rocprofv3 --pmc GRBM_GUI_ACTIVE
    SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_MFMA ...` run (CSV output directory):
    busy MFMA cycles summed over the SIMDs / (SIMDs x the dispatch's GPU
    cycles); GRBM_GUI_ACTIVE counts every XCD, so one dispatch lasts
    GRBM_GUI_ACTIVE / xcds cycles."""
    import csv
    disp = {}
    for dp, _, fs in os.walk(root):
        for f in fs:
            if f.endswith("counter_collection.csv"):
                with open(os.path.join(dp, f)) as fh:
                    for r in csv.DictReader(fh):
                        key = (r.get("Dispatch_Id"), r["Kernel_Name"])
                        disp.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    agg = {}
    for (_, name), c in disp.items():
        if "GRBM_GUI_ACTIVE" not in c or "SQ_VALU_MFMA_BUSY_CYCLES" not in c:
            continue
        if c["SQ_VALU_MFMA_BUSY_CYCLES"] <= 0:
            continue
        short = name.replace("void ", "").split("(")[0]
        a = agg.setdefault(short, {"dispatches": 0, "gpu_cycles": 0.0, "mfma_busy": 0.0,
                                   "mfma_insts": 0.0})
        a["dispatches"] += 1
        a["gpu_cycles"] += c["GRBM_GUI_ACTIVE"] / xcds
        a["mfma_busy"] += c["SQ_VALU_MFMA_BUSY_CYCLES"]
        a["mfma_insts"] += c.get("SQ_INSTS_MFMA", 0.0)
    out = {}
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["mfma_busy"]):
        out[k] = {"dispatches": a["dispatches"],
                  "avg_gpu_cycles": a["gpu_cycles"] / a["dispatches"],
                  "mfma_busy_frac": a["mfma_busy"] / (simds * a["gpu_cycles"]),
                  "avg_mfma_insts": a["mfma_insts"] / a["dispatches"]}
    return out


GOLDEN_CASE = {"cfg1": "cfg1", "cfg2": "cfg2_4sweeps", "cfg3": "cfg3", "cfg3_U2": "cfg3_U2",
               "cfg3_U6": "cfg3_U6"}


def golden(config):
    """The oracle's stored sweeps for a configuration's default chain (None if
    there are none): per-sweep bond energies, kept dims and errors."""
    case = GOLDEN_CASE.get(config)
    if case is None:
        return None
    p = os.path.join(ROOT, "tests", "golden", f"sweep_{case}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)


def oracle_compare(config, energies):
    """GPU energy after sweep k against the oracle's, k = the last sweep both
    have; None without a stored oracle run."""
    g = golden(config)
    if g is None or not g["sweeps"] or not energies:
        return None
    k = min(len(g["sweeps"]), len(energies))
    e_ref = g["sweeps"][k - 1]["E"][-1]
    e = energies[k - 1]
    return {"sweep": k, "gpu": e, "oracle": e_ref, "rel_err": abs(e - e_ref) / abs(e_ref),
            "oracle_sweeps_stored": len(g["sweeps"])}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg3", choices=["cfg1", "cfg2", "cfg3", "cfg5"])
    ap.add_argument("--U", type=float, default=None,
                    help="on-site interaction of the chain (default: the configuration's); "
                         "the chi = 1024 chain has stored oracle runs at U = 2 and 6 as well")
    ap.add_argument("--leg-sweeps", type=int, default=2,
                    help="sweeps of the FP64 and BF16x3 comparison legs (from the same state)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--eig-reduction", type=int, default=None, metavar="ORDER",
                    help="padded sector order from which the SVD's eigenproblems use the "
                         "library's own tridiagonal reduction (0: rocSOLVER's eigensolver "
                         "for all; default: the library's)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path sweeps")
    ap.add_argument("--no-bf16x3", action="store_true", help="skip the BF16x3-path sweeps")
    ap.add_argument("--no-chi1024", action="store_true",
                    help="skip the single-matvec timing at the chi = 1024 middle bond")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-chain batched matvec / Lanczos timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-only", action="store_true",
                    help="only time single H_eff matvecs at the config's middle bond "
                         "(prints their JSON and exits; for profiling)")
    ap.add_argument("--batched-sweep", action="store_true",
                    help="only run one lockstep sweep of the 64 chains, batched and chain by "
                         "chain (prints its JSON and exits; takes about two minutes)")
    ap.add_argument("--heff1", action="store_true",
                    help="time the one-site H_eff at the --config chain's middle site")
    ap.add_argument("--autoblock", action="store_true",
                    help="time the auto-blocking SVD of a matrix with hidden blocks")
    ap.add_argument("--tebd", action="store_true",
                    help="time TEBD steps (spin-1 L = 101, chi = 1000; hard-core CDW L = 51)")
    ap.add_argument("--observables", action="store_true",
                    help="time the rho_ij / <n_j> pass on the --config state")
    ap.add_argument("--spin1", action="store_true",
                    help="time sweeps of the spin-1 Heisenberg chain (L = 101, chi = 200)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 64-chain batched timing (prints its JSON and exits)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 256 MiB each way (three times), the "
                         "reference that scales the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--pmc-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR",
                                                       "CAL_WRITE_DIR"),
                    help="print the scaled HBM bytes per FP32 packed-GEMM launch from rocprofv3 "
                         "--pmc CSV runs and exit")
    ap.add_argument("--mfma-util", metavar="DIR",
                    help="MFMA utilisation per kernel from a rocprofv3 --pmc run "
                         "(GRBM_GUI_ACTIVE, SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_MFMA)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print timed-region kernel statistics of a rocprofv3 CSV trace and exit")
    args = ap.parse_args()
    if args.pmc_traffic:
        print(json.dumps(pmc_traffic(*args.pmc_traffic), indent=1))
        return
    if args.mfma_util:
        print(json.dumps(mfma_util(args.mfma_util), indent=1))
        return
    if args.summarize_trace:
        print(json.dumps(summarize_trace(args.summarize_trace), indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X and has no "
              "multi-GPU mode (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": x.numel() * 4, "copies": 3}), flush=True)
        return
    import synth
    from paper_1610_02244_amd import binding as B

    spec = synth.CONFIGS[args.config]
    case = args.config
    if args.U is not None and args.U != spec.U:
        import dataclasses
        spec = dataclasses.replace(spec, U=args.U)
        case = f"{args.config}_U{args.U:g}"
    tnt = B.load()
    if args.eig_reduction is not None:
        tnt.set_eig_reduction(args.eig_reduction)
    if args.batched_sweep:
        print(json.dumps(batched_sweep(tnt, B, torch, args.precision)), flush=True)
        return
    if args.heff1:
        print(json.dumps(heff1_rates(tnt, B, torch, spec)), flush=True)
        return
    if args.autoblock:
        print(json.dumps(autoblock_svd_rates(tnt, B, torch)), flush=True)
        return
    if args.tebd:
        print(json.dumps(tebd_steps(tnt, B, torch)), flush=True)
        return
    if args.observables:
        print(json.dumps(observables_pass(tnt, B, torch, spec)), flush=True)
        return
    if args.spin1:
        print(json.dumps(spin1_sweeps(tnt, B, torch)), flush=True)
        return
    if args.batched_only:
        print(json.dumps(batched_rates(tnt, B, torch, args.precision)), flush=True)
        return
    if args.matvec_only:
        print(json.dumps(matvec_rates(tnt, B, torch, spec, precs=(args.precision,))), flush=True)
        return
    log(f"[bench] {args.config}: L={spec.L} N={spec.N} d={spec.d} chi={spec.chi} U={spec.U} "
        f"precision={args.precision} warmup={args.warmup} steps={args.steps}")

    mps, env = make_chain(tnt, B, spec)
    e_main, s_main = [], []
    res, dt = run_sweeps(tnt, torch, mps, env, spec, args.precision, args.warmup, args.steps,
                         roctx=Roctx(), energies=e_main, stats=s_main)
    flops = sum(r["matvec_flops"] for r in res)
    value = flops / dt / 1e12
    gemm_flops = sum(r["gemm_flops"] for r in res)
    gemm_s = sum(r["seconds_gemm"] for r in res)
    launches = sum(r["gemm_launches"] for r in res)
    achieved = gemm_flops / gemm_s / 1e12 if gemm_s > 0 else 0.0
    e_final = res[-1]["energy"]
    cmp_main = oracle_compare(case, e_main)
    free_b, total_b = torch.cuda.mem_get_info()
    lib_mem = tnt.memory()
    mem = {"device_used_gb_after_main_run": (total_b - free_b) / 1e9,
           "torch_reserved_gb": torch.cuda.memory_reserved() / 1e9,
           **{k + "_gb": v / 1e9 for k, v in lib_mem.items()},
           "note": "device_used is the whole device (library pool, library handles' "
                   "workspace, torch's cache); the pool figures are the library's own"}
    del env, mps

    def leg(precision):
        """A short run of another matvec path from the same initial state: its
        energies at the same sweep indices as the main run's, sweep times."""
        m, e = make_chain(tnt, B, spec)
        en = []
        k = max(1, args.leg_sweeps)
        r, t = run_sweeps(tnt, torch, m, e, spec, precision, k - 1, 1, energies=en)
        out = {"sweeps": k, "last_sweep_s": r[-1]["seconds_total"], "energy_by_sweep": en,
               "matvec_tflops_last_sweep": r[-1]["matvec_flops"] / t / 1e12,
               "matvec_device_s_last_sweep": r[-1]["seconds_matvec"],
               "seconds_svd_last_sweep": r[-1]["seconds_svd"],
               "rel_dE_vs_main_path_same_sweep": abs(en[-1] - e_main[k - 1]) / abs(e_main[k - 1])
               if len(e_main) >= k else None,
               "vs_oracle": oracle_compare(case, en)}
        del m, e
        return out

    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        fp64 = leg("fp64")
        # against the main path's sweep of the same index (like for like)
        k = fp64["sweeps"]
        if k <= len(s_main):
            m = s_main[k - 1]
            fp64["main_path_same_sweep_s"] = m["seconds_total"]
            fp64["speedup_main_over_fp64_sweep"] = fp64["last_sweep_s"] / m["seconds_total"]
            fp64["speedup_main_over_fp64_matvec_device"] = (fp64["matvec_device_s_last_sweep"] /
                                                            m["seconds_matvec"])
    bf = None
    if not args.no_bf16x3 and args.precision != "bf16x3":
        bf = leg("bf16x3")

    bt = None if args.no_batched else batched_rates(tnt, B, torch, args.precision
                                                     if args.precision != "fp64" else "fp32")
    if bt is not None:
        log("[bench] 64-chain lockstep sweeps against the oracle")
        bt["lockstep_sweeps"] = batched_lockstep_vs_oracle(
            tnt, B, torch, args.precision if args.precision != "fp64" else "fp32")
    mv = matvec_rates(tnt, B, torch, spec)
    mv_big = None
    if not args.no_chi1024 and spec.chi < 1024:
        mv_big = matvec_rates(tnt, B, torch, synth.CONFIGS["cfg3"])
    peak = PEAK[args.precision]
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic_for(args.config, args.precision),
            "kernel": ("grouped_gemm_kernel (FP64)" if args.precision == "fp64" else
                       f"packed_gemm_kernel ({args.precision})") + ", H_eff steps 1 and 4",
            "launches": int(launches),
            "avg_launch_s": gemm_s / launches if launches else None,
            "avg_flops_per_launch": gemm_flops / launches if launches else None}
    cpu = None if args.no_cpu_baseline else cpu_baseline(spec, case)
    per = {k: sum(r[k] for r in res) / len(res) for k in
           ("seconds_total", "seconds_matvec", "seconds_lanczos", "seconds_svd", "seconds_env",
            "seconds_theta", "seconds_setup")}
    line = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"{case}: Bose-Hubbard open chain L={spec.L}, N={spec.N}, "
                               f"nmax={spec.nmax} (d={spec.d}), J={spec.J}, U={spec.U}, "
                               f"chi={spec.chi}, seeded random MPS (seed {spec.seed}), "
                               f"one two-site sweep per step, Lanczos {spec.lanczos_steps} steps",
                   "L": spec.L, "chi": spec.chi, "d": spec.d, "precision": args.precision,
                   "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu,
        "sweep_breakdown_s": per,
        "matvec_flops_per_sweep": flops / len(res),
        "matvec_device_tflops": flops / sum(r["seconds_matvec"] for r in res) / 1e12,
        "energy": {"final": e_final, "by_sweep": e_main,
                   "oracle": cmp_main["oracle"] if cmp_main else None,
                   "rel_err_vs_oracle": cmp_main["rel_err"] if cmp_main else None,
                   "compared_at_sweep": cmp_main["sweep"] if cmp_main else None,
                   "max_residual": max(r["max_residual"] for r in res),
                   "max_trunc_eps": max(r["max_eps"] for r in res)},
        "memory": mem,
        "fp64_path": fp64, "bf16x3_path": bf, "single_matvec_middle_bond": mv,
        "single_matvec_chi1024": mv_big, "batched_64_chains": bt,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
