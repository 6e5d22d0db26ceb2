"""Energy drift and temperatures of the CPU oracle at N = 65,536 (density 3),
stored for the benchmark's GPU-vs-oracle comparison of long runs.

Calls only the oracle (and the seeded input generators): the stored values
never come from the GPU library.  Protocol, the same as the GPU legs:
  * state from workloads.equilibrium_state(65536, cube, eps0, seed=2000+s),
    noise seed s, for s = 1..4;
  * 1000 relaxation steps, then 10^4 steps recording every step;
  * drift per 10^4 steps = 10^4 times the least-squares slope of
    (E_n - E_0)/|E_0| against n over the recorded steps (Sec. 4.2.1, eq.
    E_drift), E_0 the energy after relaxation;
  * T_kin and T_int averaged over the recorded steps (eqs. Tkin, Tint).
Workloads: the linear EOS (C_v = 100, eps0 = 100) at dt = 0.005 and 0.01, and
the Einstein EOS (n = 50, omega = 2, c0 = 10, eps0 = eps(theta = 1), Newton
inversion) at dt = 0.005.

The single-threaded oracle takes ~40 min per run at this size, so the runs go
to a pool of worker processes (one oracle per core); each finished run is
cached in --cache so an interrupted job resumes.  Usage:
    python tests/golden/make_oracle_drift.py --procs 8
writes tests/golden/oracle_drift_n65536.json.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 65536
SEEDS = (1, 2, 3, 4)
RELAX = 1000
STEPS = 10000
JOBS = [("linear", 0.005), ("linear", 0.01), ("einstein", 0.005)]
OUT = os.path.join(HERE, "oracle_drift_n65536.json")


def slope_per_1e4(E):
    E = np.asarray(E, dtype=float)
    n = np.arange(len(E), dtype=float)
    return float(1e4 * np.polyfit(n, (E - E[0]) / abs(E[0]), 1)[0])


def run_one(job):
    eos, dt, seed, cache = job
    path = os.path.join(cache, f"{eos}_dt{dt}_seed{seed}.json")
    if os.path.exists(path):
        return json.load(open(path))
    import oracle as O
    import workloads as W
    L = W.cubic_side(N)
    kw = dict(dt=dt, seed=seed)
    if eos == "einstein":
        kw.update(eos=1)
        eps0 = float(O.eos_energy(O.make_params(2, [L] * 3, eos=1), 1.0)[0])
    else:
        eps0 = 100.0
    q, p, e = W.equilibrium_state(N, [L] * 3, eps0=eps0, seed=2000 + seed)
    P = O.make_params(N, [L] * 3, **kw)
    t0 = time.perf_counter()
    S = O.State(P, q, p, e)
    rc, _ = S.step(RELAX)
    if rc != 0:
        raise RuntimeError(f"oracle relaxation failed ({rc}) for {eos} dt={dt} seed={seed}")
    E0 = S.energies()
    rc, rec = S.step(STEPS, record=True)
    if rc != 0:
        raise RuntimeError(f"oracle run failed ({rc}) for {eos} dt={dt} seed={seed}")
    wall = time.perf_counter() - t0
    out = {"eos": eos, "dt": dt, "seed": seed,
           "drift_per_1e4": slope_per_1e4(np.concatenate([[E0[3]], rec[:, 3]])),
           "end_to_end_rel": float((rec[-1, 3] - E0[3]) / abs(E0[3])),
           "Tkin": float(rec[:, 7].mean()), "Tint": float(rec[:, 8].mean()),
           "seconds": wall, "particle_steps_per_s": N * (RELAX + STEPS) / wall}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f)
    os.replace(tmp, path)
    print(f"done {eos} dt={dt} seed={seed}: drift {out['drift_per_1e4']:.3e} "
          f"in {wall:.0f} s", flush=True)
    return out


def mean_se(x):
    x = np.asarray(x, dtype=float)
    return [float(x.mean()), float(x.std(ddof=1) / np.sqrt(len(x))) if len(x) > 1 else 0.0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--cache", default=os.path.join("/tmp", "dpde_oracle_drift"))
    args = ap.parse_args()
    os.makedirs(args.cache, exist_ok=True)
    jobs = [(eos, dt, s, args.cache) for eos, dt in JOBS for s in SEEDS]
    t0 = time.time()
    with mp.Pool(args.procs) as pool:
        runs = pool.map(run_one, jobs, chunksize=1)
    res = {}
    for eos, dt in JOBS:
        rs = [r for r in runs if r["eos"] == eos and r["dt"] == dt]
        res[f"{eos}_dt{dt}"] = {
            "drift_per_1e4": mean_se([r["drift_per_1e4"] for r in rs]),
            "Tkin": mean_se([r["Tkin"] for r in rs]), "Tint": mean_se([r["Tint"] for r in rs]),
            "per_seed": rs}
    cpu = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"what": "CPU FP64 oracle, energy drift per 10^4 steps and temperatures",
           "n": N, "density": 3.0, "relaxation_steps": RELAX, "steps": STEPS,
           "seeds": list(SEEDS), "init_seed": "2000 + seed", "results": res,
           "host": {"cpu": cpu, "worker_processes": args.procs, "wall_seconds": time.time() - t0},
           "script": "tests/golden/make_oracle_drift.py"}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
