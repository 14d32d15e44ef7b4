"""Write the oracle's reference sweep results for the GPU sweep tests.

Calls only `oracle/` (and the seeded inputs of `synth`); nothing here comes
from the HIP path.  Usage:  python tests/golden/make_golden.py cfg1 cfg2 ...
Each case writes tests/golden/sweep_<case>.json with, per sweep, the
per-bond FP64 energies, truncation errors, kept chi and Lanczos steps, plus
the middle-bond Schmidt spectrum after the last sweep and the wall time.
The file is rewritten after every sweep ("complete": false until the last),
so a long case (the chi = 1024 chain) can be used sweep by sweep.  Cases
"cfg4_chain<i>" are chain i of the many-chain draw (`synth.batched_specs`).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import dmrg, model  # noqa: E402

# case -> (config name, chi override, sweeps override, U override)
CASES = {
    "cfg1": ("cfg1", None, None, None),
    "cfg1_exact": ("cfg1", 81, 2, None),
    "cfg2": ("cfg2", None, 1, None),
    "cfg2_2sweeps": ("cfg2", None, 2, None),
    "cfg2_4sweeps": ("cfg2", None, 4, None),
    "cfg3_chi128": ("cfg3", 128, 2, None),
    "cfg3": ("cfg3", None, 4, None),
    "cfg3_U2": ("cfg3", None, 4, 2.0),
    "cfg3_U6": ("cfg3", None, 4, 6.0),
}


def _spec(case: str):
    if case.startswith("cfg4_chain"):
        i = int(case[len("cfg4_chain"):])
        return "cfg4", synth.batched_specs(4)[i], 4
    name, chi, sweeps, U = CASES[case]
    s = synth.CONFIGS[name]
    return name, synth.ChainSpec(L=s.L, N=s.N, nmax=s.nmax, J=s.J,
                                 U=s.U if U is None else U, mu=s.mu,
                                 chi=s.chi if chi is None else chi, seed=s.seed,
                                 lanczos_steps=s.lanczos_steps,
                                 rel_cutoff=s.rel_cutoff), (s.sweeps if sweeps is None
                                                            else sweeps)


def _host():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0)}


def run(case: str):
    name, s, sweeps = _spec(case)
    chi, U = s.chi, s.U
    d = s.nmax + 1
    W, qw = model.bh_mpo(s.nmax, s.J, U, s.mu)
    bonds, sites = synth.random_mps(s.L, s.N, s.nmax, chi, s.seed)
    bonds, sites = dmrg.right_canonicalise(bonds, sites, d)
    t0 = time.time()
    out = {"case": case, "config": name, "L": s.L, "N": s.N, "nmax": s.nmax, "J": s.J, "U": U,
           "mu": s.mu, "chi": chi, "seed": s.seed, "lanczos_steps": s.lanczos_steps,
           "rel_cutoff": s.rel_cutoff, "host": _host(), "sweeps": [], "complete": False}
    path = os.path.join(HERE, f"sweep_{case}.json")

    def write():
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)

    envs = None
    for k in range(sweeps):
        ts = time.time()
        bonds, sites, envs, recs = dmrg.sweep(bonds, sites, [W] * s.L, qw, d, chi,
                                              s.lanczos_steps, trunc=dict(r=s.rel_cutoff),
                                              envs=envs)
        out["sweeps"].append({
            "E": [r["E"] for r in recs], "eps": [r["eps"] for r in recs],
            "chi": [r["chi"] for r in recs], "steps": [r["steps"] for r in recs],
            "wall_s": time.time() - ts})
        out["wall_s"] = time.time() - t0
        if k + 1 < sweeps:
            write()
        print(f"{case}: sweep {k + 1} E = {recs[-1]['E']:.15f} ({time.time() - t0:.1f}s)",
              flush=True)
    j = s.L // 2
    th = dmrg.form_theta(sites[j - 1], sites[j], bonds[j - 1], bonds[j + 1], d)
    from oracle import svd as osvd
    sv = osvd.svd_truncate(th, bonds[j - 1], bonds[j + 1], d, 10 ** 6, renormalise=False)
    out["mid_spectrum"] = [float(x) for x in sv["all_lambdas"][:64]]
    out["expectation"] = dmrg.expectation(bonds, sites, [W] * s.L, qw, d)
    out["wall_s"] = time.time() - t0
    out["complete"] = True
    write()


if __name__ == "__main__":
    for c in sys.argv[1:] or ["cfg1", "cfg1_exact"]:
        run(c)
