"""Throughput of the DPDE VV+SER step on one MI355X.

Default workload: the learned-EOS system, N = 1,048,576 particles at number
density 3 in a periodic cube (side 70.4411, 70^3 cells), soft DPD force
a = 25, gamma = 4.5, kT = 1, Einstein internal EOS (n = 50, w = 2, c0 = 10)
inverted by the surrogate network (trained on the GPU first) with Newton
outside its range, dt = 0.005, FP64 pair terms.  Inputs are synthetic
(uniform positions, Maxwell momenta, theta_i = 1) and resident in HBM before
the timed region.

One JSON line on stdout: metric, value (particle-steps/s), roofline of the
dominant kernel (per-kernel HIP-event times over a profiled stretch of the
same run), the CPU oracle timed on a bounded sample of the same workload, and
the other variants of the same geometry.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one lane-operation per lane per clock; FP64 FMA counts once)
ALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU lane-operations of one directed SER pair term of sweep 1,
# counted from the formulas as implemented: Philox-4x32-10 45 (two 32x32->64
# products and two three-way xors per round), FP64 Box-Muller 173 (two
# logarithms 38 each, two square roots 8 each, two sine/cosine pairs 36 each,
# uniforms and products 9), pair geometry, weight and increment 63,
# accumulation 3
PAIR_TERM_LANE_OPS = 284
FP64_VECTOR_PEAK_TFLOPS = 78.6
N_1M = 1_048_576


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_system(dp, W, n, *, eos, theta_mode, precision, dt, seed=7, init_seed=20260101):
    L = W.cubic_side(n)
    box = [L, L, L]
    cfg = dp.Config(n=n, box=box, dt=dt, eos=eos, theta_mode=theta_mode, precision=precision,
                    seed=seed)
    if eos == dp.EOS_EINSTEIN:
        # eps_i = eps(theta = 1) from the library's own EOS (a small helper handle)
        nh = 200
        Lh = W.cubic_side(nh)
        qh, ph, eh = W.equilibrium_state(nh, [Lh] * 3, eps0=10.0, seed=1)
        helper = dp.System(dp.Config(n=nh, box=[Lh] * 3, eos=eos), qh, ph, eh)
        import torch
        eps0 = float(helper.eos_energy(torch.ones(1, dtype=torch.float64)).cpu()[0])
        helper.close()
    else:
        eps0 = cfg.cv * 1.0
    q, p, e = W.equilibrium_state(n, box, eps0=eps0, seed=init_seed)
    return dp.System(cfg, q, p, e), cfg, (q, p, e), eps0


def timed(sysm, steps, warmup):
    import torch
    sysm.step(warmup)
    sysm.history()  # drop warm-up records
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, sysm.history()


def timed_graph(sysm, steps, warmup, g=100):
    """Like timed(), with the timed steps run as replays of one captured
    g-step graph (dpde_step_graph); the capture and its first replay belong
    to the warm-up.  A remainder that is not a multiple of g runs eagerly."""
    import torch
    g = max(2, min(g, steps - steps % 2))
    reps, rem = divmod(steps, g)
    sysm.step(warmup)
    sysm.step_graph(g, 1)
    sysm.history()  # drop warm-up records
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step_graph(g, reps)
    if rem:
        sysm.step(rem)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, sysm.history()


def drift_per_1e4(hist):
    """Slope of (E_n - E_0)/|E_0| per 10^4 steps over a timed run.  The timed
    runs start from the synthetic (unrelaxed) state, so this includes the
    relaxation transient; the drift measurement proper is `drift_gpu` and
    `drift_vs_oracle`, which relax first."""
    E = hist[:, 3]
    if len(E) < 3:
        return None
    n = np.arange(len(E), dtype=float)
    s = np.polyfit(n, (E - E[0]) / abs(E[0]), 1)[0]
    return float(1e4 * s)


def drift_fit(E):
    """Least-squares slope of (E_n - E_0)/|E_0| against n, times 10^4
    (the linear fit of Sec. 4.2.1, eq. E_drift, per 10^4 steps)."""
    E = np.asarray(E, dtype=float)
    n = np.arange(len(E), dtype=float)
    return float(1e4 * np.polyfit(n, (E - E[0]) / abs(E[0]), 1)[0])


def mean_se(x):
    x = np.asarray(x, dtype=float)
    return float(x.mean()), float(x.std(ddof=1) / math.sqrt(len(x))) if len(x) > 1 else 0.0


def drift_vs_oracle(dp, W, seeds, n=1000, steps=1000, dt=0.01):
    """Small equilibrium system (N=1000, density 3, dt=0.01, 1000 steps):
    GPU and CPU oracle run the same seeds; drift per 10^4 steps and the
    kinetic/internal temperatures, mean +- standard error over seeds."""
    import oracle as O
    L = W.cubic_side(n)
    g_d, o_d, g_tk, g_ti, o_tk, o_ti = [], [], [], [], [], []
    t_cpu = 0.0
    for sd in seeds:
        q, p, e = W.equilibrium_state(n, [L] * 3, eps0=100.0, seed=1000 + sd)
        s = dp.System(dp.Config(n=n, box=[L] * 3, dt=dt, seed=sd), q, p, e)
        E0 = s.energies()
        s.step(steps)
        h = s.history()
        s.close()
        Eg = np.concatenate([[E0[3]], h[:, 3]])
        g_d.append(drift_fit(Eg))
        g_tk.append(h[steps // 2:, 7].mean())
        g_ti.append(h[steps // 2:, 8].mean())
        P = O.make_params(n, [L] * 3, dt=dt, seed=sd)
        t0 = time.perf_counter()
        S = O.State(P, q, p, e)
        E0o = S.energies()
        rc, rec = S.step(steps, record=True)
        t_cpu += time.perf_counter() - t0
        Eo = np.concatenate([[E0o[3]], rec[:, 3]])
        o_d.append(drift_fit(Eo))
        o_tk.append(rec[steps // 2:, 7].mean())
        o_ti.append(rec[steps // 2:, 8].mean())
    gm, gs = mean_se(g_d)
    om, os_ = mean_se(o_d)
    return {"workload": f"N={n} density 3, dt={dt}, {steps} steps, {len(seeds)} seeds, FP64",
            "gpu_drift_per_1e4": [gm, gs], "oracle_drift_per_1e4": [om, os_],
            "diff_over_combined_se": abs(gm - om) / max(1e-300, math.hypot(gs, os_)),
            "gpu_Tkin_Tint": [mean_se(g_tk)[0], mean_se(g_ti)[0]],
            "oracle_Tkin_Tint": [mean_se(o_tk)[0], mean_se(o_ti)[0]],
            "oracle_seconds": t_cpu}


GOLDEN_DRIFT = os.path.join(ROOT, "tests", "golden", "oracle_drift_n65536.json")


def _eps_theta1(dp, W):
    """eps(theta = 1) of the Einstein EOS from the library's own EOS kernel."""
    import torch
    nh = 200
    Lh = W.cubic_side(nh)
    qh, ph, eh = W.equilibrium_state(nh, [Lh] * 3, eps0=10.0, seed=1)
    helper = dp.System(dp.Config(n=nh, box=[Lh] * 3, eos=dp.EOS_EINSTEIN), qh, ph, eh)
    eps0 = float(helper.eos_energy(torch.ones(1, dtype=torch.float64)).cpu()[0])
    helper.close()
    return eps0


def drift_gpu(dp, W, n=65536, steps=10000, seeds=(1, 2, 3, 4), mlp_iters=20000):
    """Equilibrium energy drift and temperatures on the GPU at N = 65,536
    (density 3): 10^4 steps after 1000 relaxation steps, the protocol of the
    stored oracle runs (same initial states and noise seeds), with the linear
    EOS (FP64 and FP32 pair terms, dt 0.005 and 0.01) and the Einstein EOS at
    dt 0.005 (FP64 with Newton, FP64 with the surrogate, FP32 with the
    surrogate) and 0.0025 (FP64 with Newton, FP32 with the surrogate).  Each
    FP64 result with a stored oracle run is set against it, in combined
    standard errors of the seed means."""
    L = W.cubic_side(n)
    golden = json.load(open(GOLDEN_DRIFT))["results"] if os.path.exists(GOLDEN_DRIFT) else {}
    eps_e = _eps_theta1(dp, W)
    legs = [("fp64_linear_dt0.005", dp.EOS_LINEAR, dp.THETA_NEWTON, dp.FP64, 0.005, "linear_dt0.005"),
            ("fp64_linear_dt0.01", dp.EOS_LINEAR, dp.THETA_NEWTON, dp.FP64, 0.01, "linear_dt0.01"),
            ("fp32_linear_dt0.005", dp.EOS_LINEAR, dp.THETA_NEWTON, dp.FP32, 0.005, None),
            ("fp32_linear_dt0.01", dp.EOS_LINEAR, dp.THETA_NEWTON, dp.FP32, 0.01, None),
            ("fp64_newton_einstein_dt0.005", dp.EOS_EINSTEIN, dp.THETA_NEWTON, dp.FP64, 0.005,
             "einstein_dt0.005"),
            ("fp64_mlp_einstein_dt0.005", dp.EOS_EINSTEIN, dp.THETA_MLP, dp.FP64, 0.005, None),
            ("fp32_mlp_einstein_dt0.005", dp.EOS_EINSTEIN, dp.THETA_MLP, dp.FP32, 0.005, None),
            # the Einstein EOS at half the step, where the drift of both forms
            # falls below 1e-6 per 10^4 steps
            ("fp64_newton_einstein_dt0.0025", dp.EOS_EINSTEIN, dp.THETA_NEWTON, dp.FP64, 0.0025,
             None),
            ("fp32_mlp_einstein_dt0.0025", dp.EOS_EINSTEIN, dp.THETA_MLP, dp.FP32, 0.0025, None)]
    weights = None
    out = {}
    for name, eos, tm, prec, dt, gkey in legs:
        dr, tk, ti = [], [], []
        for sd in seeds:
            eps0 = eps_e if eos == dp.EOS_EINSTEIN else 100.0
            q, p, e = W.equilibrium_state(n, [L] * 3, eps0=eps0, seed=2000 + sd)
            s = dp.System(dp.Config(n=n, box=[L] * 3, dt=dt, seed=sd, eos=eos, theta_mode=tm,
                                    precision=prec), q, p, e)
            if tm != dp.THETA_NEWTON:
                if weights is None:
                    s.mlp_train(nsamples=10**6, iters=mlp_iters, batch=4096, lr=3e-3)
                    weights = s.mlp_get()
                else:
                    s.mlp_set(*weights)
            # relax the random initial packing before measuring
            s.step_graph(100, 10)
            s.history()
            E0 = s.energies()
            s.step_graph(100, steps // 100)
            h = s.history()
            s.close()
            dr.append(drift_fit(np.concatenate([[E0[3]], h[:, 3]])))
            tk.append(h[:, 7].mean())
            ti.append(h[:, 8].mean())
        r = {"drift_per_1e4": list(mean_se(dr)), "Tkin": list(mean_se(tk)),
             "Tint": list(mean_se(ti)), "dt": dt}
        if gkey and gkey in golden:
            g = golden[gkey]
            r["oracle_drift_per_1e4"] = g["drift_per_1e4"]
            r["oracle_Tkin"] = g["Tkin"]
            r["oracle_Tint"] = g["Tint"]
            r["drift_diff_over_combined_se"] = abs(r["drift_per_1e4"][0] - g["drift_per_1e4"][0]) / \
                max(1e-300, math.hypot(r["drift_per_1e4"][1], g["drift_per_1e4"][1]))
        out[name] = r
        log(f"[bench]   drift {name}: {r['drift_per_1e4'][0]:.3e} +- {r['drift_per_1e4'][1]:.1e}")
    return {"workload": f"N={n} density 3, {steps} steps after 1000 relaxation steps, "
                        f"{len(seeds)} seeds (noise seeds {list(seeds)}, initial states seeded "
                        f"2000 + seed), drift = 10^4 x slope of (E_n - E_0)/|E_0|",
            "oracle": "tests/golden/oracle_drift_n65536.json (CPU FP64 oracle, same protocol)",
            "results": out}


def kernel_profile(sysm, steps):
    sysm.profile(True)
    sysm.step(steps)
    prof = sysm.profile_read()
    sysm.profile(False)
    return {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in prof.items()}


def mean_neighbours(sysm, n):
    pr = sysm.debug_pairs()
    return 2.0 * len(pr) / n


# Algorithmic HBM bytes per particle of the pair kernels: every per-particle
# array the step of the method reads or writes, once (q, p, 1/T, id, eps, F,
# dp_i at 8 B per double, 4 B per id); neighbour gathers, neighbour lists and
# the stored increments dp_ij are this implementation's choices and are not
# counted.
ALGO_BYTES = {
    "pass_a": 24 + 24 + 24 + 24,          # q, p' in | F, p~ out  (96)
    "pass_b": 24 + 24 + 8 + 4 + 24,       # q, p~, 1/T, id in | dp_i out  (84)
    "pass_c": 24 + 24 + 8 + 4 + 24 + 8 + 24 + 8 + 8,  # q, p~, 1/T, id, dp_i, eps | p, eps, 1/T (132)
}
# The end of the step inside the tile sweep 2 (the observables' sums and the
# next step's kick and drift): F, U and Laplacian shares in | q out (64); the
# build-time position the list-build decision compares with is the lists'
# machinery, not counted
TAIL_BYTES = 24 + 8 + 8 + 24


def pair_kernel_bytes(name, tail=False):
    for k, v in ALGO_BYTES.items():
        if name.startswith(k):
            return float(v) + (TAIL_BYTES if tail and k == "pass_c" else 0.0)
    return None


def pair_kernel_list_bytes(name, nwork, nskin, tail=False):
    """The same plus the neighbour-list words (4 B per entry and per count):
    the skin list read and the work list written by pass A, the work list read
    by the sweeps."""
    b = pair_kernel_bytes(name, tail)
    if b is None:
        return None
    work = 4.0 + 4.0 * nwork
    if name.startswith("pass_a"):
        return b + 4.0 + 4.0 * nskin + work
    return b + work


PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "learned_eos_n1m_traffic.txt")
KERNEL_SOURCES = ["common.h", "bin.h", "pairs.h", "eos.h", "mlp.h", "hybrid.h", "api.hip"]


def _profile_lines():
    """Lines of the committed counter summary, or None when the kernel
    sources have changed since the counters were taken."""
    import hashlib
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1507_06643_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    lines = open(PROFILE_TRAFFIC).read().splitlines()
    sha = [l.split()[1] for l in lines if l.startswith("source_sha256")]
    if not sha or sha[0] != h.hexdigest():
        return None
    return lines


# The pair kernels of the headline workload as rocprofv3 names them (batch,
# precision, model and, for sweep 2, the surrogate fused in: the learned EOS).
PAIR_KERNEL_SYMBOLS = {"pass_a_forces": "k_pass_a_uniq<false, 0, false>",
                       "pass_b_ser": "k_pass_b_uniq<false, 0, 0>",
                       "pass_c_ser": "k_pass_c_uniq<false, 0, 0, 0, 1>"}


def counter_traffic(kernel):
    """HBM bytes per launch (read, write) of a kernel from the committed
    rocprofv3 counter summary (None if stale)."""
    lines = _profile_lines()
    for l in lines or []:
        parts = l.rsplit(" ", 2)
        if len(parts) == 3 and parts[0] == kernel:
            return float(parts[1]), float(parts[2])
    return None


def counter_valu(kernel):
    """Issued VALU wave-instructions per launch from the committed summary."""
    lines = _profile_lines()
    for l in lines or []:
        if l.startswith("valu "):
            name, v = l[5:].rsplit(" ", 1)
            if name == kernel:
                return float(v)
    return None


def batched_leg(dp, W, nrep=256, steps=2000, graph_steps=100, tune_steps=10):
    """Independent replicas of uneven size in one handle, advanced by replays
    of one captured graph, block sizes chosen by the library's autotuner."""
    import torch
    sizes, seeds = W.replica_sizes(nrep, 500, 8000, seed=20260103)
    cfgs, qs, ps, es = [], [], [], []
    for r, (nr, sd) in enumerate(zip(sizes, seeds)):
        L = W.cubic_side(int(nr))
        q, p, e = W.equilibrium_state(int(nr), [L] * 3, seed=30000 + r)
        cfgs.append(dp.Config(n=int(nr), box=[L] * 3, dt=0.01, seed=int(sd), replica=r))
        qs.append(q); ps.append(p); es.append(e)
    s = dp.System(cfgs, np.concatenate(qs), np.concatenate(ps), np.concatenate(es))
    _, _, tune_ms = s.autotune(tune_steps)
    shape = s.get_shape()
    s.step_graph(graph_steps, 1)  # capture and warm up
    s.history()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_graph(graph_steps, steps // graph_steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    hist = s.history(cap=steps)  # (steps, nrep, record)
    drifts = np.array([drift_fit(hist[:, r, 3]) for r in range(nrep)])
    ntot = int(sizes.sum())
    s.close()
    return {"workload": f"{nrep} replicas, N uniform in [500, 8000] (total {ntot}), density 3, "
                        f"dt=0.01, {steps} steps as {steps // graph_steps} replays of a "
                        f"{graph_steps}-step graph, FP64",
            "value": ntot * steps / secs, "unit": "particle-steps/s",
            "ms_per_step": 1e3 * secs / steps,
            "autotuned": {"shape": shape, "trial_ms_per_step": tune_ms},
            "drift_per_1e4": [float(drifts.mean()), float(drifts.std(ddof=1) / np.sqrt(nrep))]}


def shock_leg(dp, W, steps=5000, graph_steps=100, nslab=20):
    """Symmetric impact in a 400 x 20 x 20 box (free along x): throughput,
    energy conservation and the kinetic/internal temperature profiles."""
    import torch
    box = (400.0, 20.0, 20.0)
    q, p, e = W.shock_state(box)
    n = len(q)
    cfg = dp.Config(n=n, box=list(box), periodic=(0, 1, 1), dt=0.005, precision=dp.FP32)
    s = dp.System(cfg, q, p, e)
    E0 = s.energies()[3]
    s.step_graph(graph_steps, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_graph(graph_steps, steps // graph_steps - 1)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    E1 = s.energies()[3]
    qg, pg, eg, st = s.get_state()
    qg, pg, eg = qg.cpu().numpy(), pg.cpu().numpy(), eg.cpu().numpy()
    s.close()

    def profile(qx, pp, ee):
        edges = np.linspace(0.0, box[0], nslab + 1)
        idx = np.clip(np.digitize(qx, edges) - 1, 0, nslab - 1)
        tk, ti, ux = [], [], []
        for b in range(nslab):
            m = idx == b
            if m.sum() < 2:
                tk.append(None); ti.append(None); ux.append(None)
                continue
            v = pp[m] / cfg.mass
            vbar = v.mean(axis=0)
            tk.append(float(cfg.mass * ((v - vbar) ** 2).sum() / (3 * (m.sum() - 1))))
            ti.append(float((ee[m] / cfg.cv).mean()))
            ux.append(float(vbar[0]))
        return {"T_kin": tk, "T_int": ti, "u_x": ux}
    return {"workload": f"shock, N={n}, box 400x20x20 (free along x), +-2 bulk velocity, "
                        f"dt=0.005, {steps} steps, FP32 pair terms, FP64 energies",
            "value": n * (steps - graph_steps) / secs, "unit": "particle-steps/s",
            "ms_per_step": 1e3 * secs / (steps - graph_steps),
            "energy_rel_change": float((E1 - E0) / abs(E0)), "final_step": int(st),
            "slabs": nslab, "initial_profile": profile(q[:, 0], p, e),
            "final_profile": profile(qg[:, 0], pg, eg)}


def next_rows_leg(dp, W, n=N_1M, steps=100, warmup=20, only=None):
    """Throughput at N = 1M of the schemes beyond plain SER: SEM with the
    internal-energy projection (Sec. 4.2), friction and noise along e_ij,
    the splined LJ at the paper's density (eq. Ep), and Hybrid with 32^3
    domains (Sec. 3.2.2)."""
    out = {}
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=20260101)
    cases = [
        ("sem_projected", dict(scheme=dp.SCHEME_SEM, project=True, dt=0.005)),
        ("projected_model_ser", dict(model=dp.MODEL_PROJECTED, dt=0.005)),
        ("hybrid_32cubed_domains", dict(scheme=dp.SCHEME_HYBRID, ndom=(32, 32, 32), dt=0.005)),
    ]
    for name, kw in cases:
        if only is not None and name != only:
            continue
        log(f"[bench] next rows: {name}")
        s = dp.System(dp.Config(n=n, box=[L] * 3, **kw), q, p, e)
        secs, h = timed(s, steps, warmup)
        out[name] = {"value": n * steps / secs, "ms_per_step": 1e3 * secs / steps,
                     "timed_run_energy_slope_per_1e4": drift_per_1e4(h)}
        s.close()
    if only is not None and only != "lj_density_0.8095":
        return out
    side = int(round(n ** (1.0 / 3.0)))
    ql, pl, el, box = W.lattice_state(side, 0.8095, eps0=50.0, seed=20260105)
    log(f"[bench] next rows: lj_density_0.8095 (N={side ** 3})")
    s = dp.System(dp.Config(n=side ** 3, box=box, potential=dp.POT_LJ, rc=2.5, cv=50.0, gamma=8.0,
                            dt=0.002, neighbor_cap=128, project=True), ql, pl, el)
    secs, h = timed(s, steps, warmup)
    out["lj_density_0.8095"] = {"value": side ** 3 * steps / secs,
                                "ms_per_step": 1e3 * secs / steps, "n": side ** 3,
                                "T_kin": float(h[:, 7].mean()),
                                "T_pot": float(h[:, 10].mean() / h[:, 11].mean()),
                                "T_int": float(h[:, 8].mean())}
    s.close()
    return out


def oracle_worker(n, steps, eos, dt, eps0, seed):
    """One single-threaded oracle run (a child process of cpu_baseline):
    prints its step rate as one JSON line."""
    import oracle as O
    import workloads as W
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, eps0=eps0, seed=seed)
    P = O.make_params(n, [L] * 3, dt=dt, eos=eos)
    t0 = time.perf_counter()
    S = O.State(P, q, p, e)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    rc, _ = S.step(steps)
    t_run = time.perf_counter() - t0
    print(json.dumps({"rate": n * steps / t_run, "seconds": t_run, "init_seconds": t_init,
                      "rc": rc}), flush=True)


def cpu_baseline(n, steps, eos, dt, eps0, max_procs=16):
    """The CPU oracle on every host core available to this process (at most
    max_procs): one single-threaded oracle process per core, each running
    `steps` steps of its own copy of the workload after its initialisation;
    the throughput is the sum of their step rates.  The oracle is the same
    plain C code the tests pin (not tuned for speed)."""
    import subprocess
    cores = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-worker",
           json.dumps([n, steps, eos, dt, eps0])]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    t0 = time.perf_counter()
    procs = [subprocess.Popen(cmd + [str(20260101 + k)], stdout=subprocess.PIPE, env=env,
                              text=True) for k in range(cores)]
    outs = []
    for pr in procs:
        so, _ = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"oracle worker failed with {pr.returncode}")
        outs.append(json.loads(so.strip().splitlines()[-1]))
    wall = time.perf_counter() - t0
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    rates = [o["rate"] for o in outs]
    return {"value": float(sum(rates)), "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{cores} single-threaded oracle processes in parallel (one per core), "
                      f"each {steps} steps of its own N={n} learned-EOS system (Newton "
                      f"inversion, dt={dt}) after initialisation; step rates summed "
                      f"(per process {min(rates):.3g}-{max(rates):.3g} particle-steps/s, "
                      f"{wall:.0f} s wall)",
            "per_core_rate": float(np.mean(rates)), "rc": [o["rc"] for o in outs],
            "cpu_model": model, "host_cpus_available": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--n", type=int, default=N_1M)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--tuning-table",
                    default=os.path.join(ROOT, "paper_1507_06643_amd", "tuning_gfx950.txt"),
                    help="launch-shape table loaded before any system is made (if present)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default block sizes (profiling runs: no tuning trials)")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--mlp-iters", type=int, default=20000)
    ap.add_argument("--no-drift", action="store_true", help="skip the energy-drift legs")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the batched-replica and shock legs")
    ap.add_argument("--drift-seeds", type=int, default=8)
    ap.add_argument("--next-row", default=None,
                    choices=["sem_projected", "projected_model_ser", "hybrid_32cubed_domains",
                             "lj_density_0.8095"],
                    help="only time one of the next-row workloads at N = 1M and print its "
                         "figures (profiling runs)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only time the batched-replica workload and print its figures "
                         "(profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--oracle-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("worker_seed", nargs="?", type=int, default=20260101, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_worker:
        n_w, steps_w, eos_w, dt_w, eps_w = json.loads(args.oracle_worker)
        oracle_worker(n_w, steps_w, eos_w, dt_w, eps_w, args.worker_seed)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU slab decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 3}))
        return

    import paper_1507_06643_amd as dp
    import workloads as W

    torch.cuda.set_device(0)
    table = args.tuning_table if args.tuning_table and os.path.exists(args.tuning_table) else None
    if table:
        dp.tuning_load(table)
    if args.next_row:
        print(json.dumps(next_rows_leg(dp, W, only=args.next_row)), flush=True)
        return
    if args.batched_only:
        print(json.dumps(batched_leg(dp, W)), flush=True)
        return
    n = args.n
    dt = 0.005
    log(f"[bench] learned-EOS workload N={n}: init")
    sysm, cfg, _, eps0 = make_system(dp, W, n, eos=dp.EOS_EINSTEIN, theta_mode=dp.THETA_MLP,
                                     precision=dp.FP64, dt=dt)
    t0 = time.perf_counter()
    curve = sysm.mlp_train(nsamples=10**6, iters=args.mlp_iters, batch=4096, lr=3e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[bench] surrogate trained in {t_train:.2f} s, final loss {curve[-1]:.3e}")
    if not args.no_autotune:
        sysm.autotune(20)
    shape = sysm.get_shape()
    log(f"[bench] launch shape: {shape} ({'autotuned' if not args.no_autotune else 'table' if table else 'default'})")
    graph_len = max(2, min(100, args.steps - args.steps % 2))
    log(f"[bench] timing {args.steps} steps ({graph_len}-step graph replays) after "
        f"{args.warmup} warm-up")
    secs, hist = timed_graph(sysm, args.steps, args.warmup, g=graph_len)
    value = n * args.steps / secs
    ms_step = 1e3 * secs / args.steps
    log(f"[bench] {value:.4e} particle-steps/s ({ms_step:.3f} ms/step)")
    secs_e, _ = timed(sysm, 100, 0)
    eager_ms = 1e3 * secs_e / 100
    prof = kernel_profile(sysm, args.profile_steps)
    nbar = mean_neighbours(sysm, n)
    nwork = sysm.mean_work_list()
    # skin-list length from the density of the uniform fluid: the list's own
    # pairs (all of them, or a tile's inner pairs once) within rc + skin
    nskin = nwork * ((cfg.rc + cfg.skin) / cfg.rc) ** 3
    b0 = sysm.list_builds()
    sysm.step(100)
    builds_per_step = (sysm.list_builds() - b0) / 100.0
    symbols = PAIR_KERNEL_SYMBOLS
    unique_pairs = 0.5 * nbar * n
    # the step's end runs inside sweep 2 when the kick is launched less often
    # than the sweep (once per call rather than once per step)
    tail = prof.get("kick", {"launches": 0})["launches"] < prof["pass_c_ser"]["launches"]
    pair_roofs = {}
    for k in [k for k in prof if k in symbols]:
        bpp_k = pair_kernel_bytes(k, tail)
        t_k = prof[k]["avg_ms"] * 1e-3
        tr = counter_traffic(symbols[k])
        vi = counter_valu(symbols[k])
        r = {"avg_launch_ms": prof[k]["avg_ms"], "algorithmic_bytes_per_particle": bpp_k,
             "algorithmic_bytes": bpp_k * n, "hbm_GBps": bpp_k * n / t_k / 1e9,
             "hbm_frac": bpp_k * n / t_k / 1e9 / HBM_PEAK_GBS,
             "with_lists_bytes_per_particle": pair_kernel_list_bytes(k, nwork, nskin, tail),
             "with_lists_hbm_frac": pair_kernel_list_bytes(k, nwork, nskin, tail) * n / t_k /
             1e9 / HBM_PEAK_GBS,
             "counter_bytes": None if tr is None else tr[0] + tr[1],
             "counter_GBps": None if tr is None else (tr[0] + tr[1]) / t_k / 1e9,
             "issued_valu_frac": None if vi is None else vi * 64 / t_k / ALU_PEAK_LANE_OPS}
        if k.startswith("pass_b"):
            # secondary: the noise and increment of every unique pair, once
            ops = PAIR_TERM_LANE_OPS * unique_pairs
            r.update({"unique_pairs": unique_pairs, "algorithmic_lane_ops": ops,
                      "alu_lane_ops_per_s": ops / t_k, "alu_frac": ops / t_k / ALU_PEAK_LANE_OPS})
        pair_roofs[k] = r
    dom = max(pair_roofs, key=lambda k: pair_roofs[k]["avg_launch_ms"])
    d = pair_roofs[dom]
    roof = {"kernel": dom, "symbol": symbols[dom], "bound": "hbm", "achieved": d["hbm_GBps"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["hbm_frac"],
            "traffic": d["counter_bytes"],
            # the kernel's measured HBM traffic (counters) against the same peak
            "traffic_frac": None if d["counter_GBps"] is None else d["counter_GBps"] / HBM_PEAK_GBS,
            "bytes_per_particle": d["algorithmic_bytes_per_particle"],
            "n": n, "avg_launch_ms": d["avg_launch_ms"], "step_end_in_sweep_2": tail,
            "mean_neighbours": nbar,
            "mean_work_list": nwork, "skin_list_estimate": nskin, "pair_kernels": pair_roofs}
    if "alu_frac" in d:
        roof["secondary_alu"] = {"achieved": d["alu_lane_ops_per_s"], "peak": ALU_PEAK_LANE_OPS,
                                 "unit": "lane-op/s", "frac": d["alu_frac"],
                                 "lane_ops_per_unique_pair": PAIR_TERM_LANE_OPS}
    line = {
        "metric": "particle-steps/s at N=1M",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "learned-EOS N=1,048,576 density 3, Einstein EOS (n=50, w=2, c0=10) "
                               "via BF16 surrogate + Newton fallback, dt=0.005, FP64 pair terms",
                   "n": n, "dt": dt, "precision": "fp64", "theta": "mlp+newton-fallback",
                   "skin": cfg.skin, "list_builds_per_step": builds_per_step,
                   "execution": f"replays of a captured {graph_len}-step graph",
                   "shape": shape, "autotuned": not args.no_autotune,
                   "tuning_table": os.path.relpath(table, ROOT) if table else None},
        "eager_ms_per_step": eager_ms,
        "roofline": roof,
        "kernels_ms": {k: round(v["avg_ms"], 5) for k, v in prof.items()},
        "timed_run_energy_slope_per_1e4": drift_per_1e4(hist),
        "surrogate_train_s": t_train,
    }
    sysm.close()
    if not args.no_variants:
        variants = {}
        for name, eos, tm, prec, vdt in [
                ("plain_fp64_linear_eos", dp.EOS_LINEAR, dp.THETA_NEWTON, dp.FP64, 0.005),
                ("fp32_pairs_learned_eos", dp.EOS_EINSTEIN, dp.THETA_MLP, dp.FP32, 0.005),
                ("fp64_newton_learned_eos", dp.EOS_EINSTEIN, dp.THETA_NEWTON, dp.FP64, 0.005),
                # at half the step, where both forms drift below 1e-6 per 10^4 steps
                ("fp32_pairs_learned_eos_dt0.0025", dp.EOS_EINSTEIN, dp.THETA_MLP, dp.FP32, 0.0025),
                ("fp64_newton_learned_eos_dt0.0025", dp.EOS_EINSTEIN, dp.THETA_NEWTON, dp.FP64,
                 0.0025)]:
            log(f"[bench] variant {name}")
            s2, _, _, _ = make_system(dp, W, n, eos=eos, theta_mode=tm, precision=prec, dt=vdt)
            if tm != dp.THETA_NEWTON:
                s2.mlp_train(nsamples=10**6, iters=args.mlp_iters, batch=4096, lr=3e-3)
            if not args.no_autotune:
                s2.autotune(20)
            sec2, h2 = timed_graph(s2, max(50, args.steps // 2), 10)
            p2 = kernel_profile(s2, args.profile_steps)
            variants[name] = {"value": n * max(50, args.steps // 2) / sec2,
                              "ms_per_step": 1e3 * sec2 / max(50, args.steps // 2),
                              "kernels_ms": {k: round(v["avg_ms"], 5) for k, v in p2.items()},
                              "timed_run_energy_slope_per_1e4": drift_per_1e4(h2)}
            s2.close()
        line["variants"] = variants
        # speed of the FP32-pair-term + surrogate form relative to plain FP64
        # (linear EOS) and to FP64 with Newton on the same EOS; the drift legs
        # give both precisions' drift at dt = 0.005 and 0.0025
        v32 = variants["fp32_pairs_learned_eos"]["value"]
        line["fp32_surrogate_speedup"] = {
            "vs_plain_fp64_linear_eos": v32 / variants["plain_fp64_linear_eos"]["value"],
            "vs_fp64_newton_same_eos": v32 / variants["fp64_newton_learned_eos"]["value"],
            "vs_fp64_surrogate_same_eos": v32 / value,
            "vs_fp64_newton_same_eos_dt0.0025":
                variants["fp32_pairs_learned_eos_dt0.0025"]["value"] /
                variants["fp64_newton_learned_eos_dt0.0025"]["value"]}
    if not args.no_legs:
        log("[bench] batched replicas: 256 systems, one captured graph, autotuned blocks")
        line["batched_replicas"] = batched_leg(dp, W)
        log("[bench] shock: N=480000, 5000 steps, FP32 pair terms")
        line["shock"] = shock_leg(dp, W)
        line["next_rows"] = next_rows_leg(dp, W)
    if not args.no_drift:
        log("[bench] energy drift: GPU vs oracle, N=1000")
        line["drift_vs_oracle"] = drift_vs_oracle(dp, W, list(range(1, args.drift_seeds + 1)))
        log("[bench] energy drift: GPU, N=65536, 10^4 steps")
        line["drift_gpu"] = drift_gpu(dp, W, mlp_iters=args.mlp_iters)
        sp = line.get("fp32_surrogate_speedup")
        res = line["drift_gpu"]["results"]
        if sp is not None:
            # the speedup stated next to the drift of both forms on the same
            # EOS and dt, and their difference in combined standard errors
            for dtk in ("0.005", "0.0025"):
                a = res[f"fp32_mlp_einstein_dt{dtk}"]
                b = res[f"fp64_newton_einstein_dt{dtk}"]
                sfx = "" if dtk == "0.005" else "_dt0.0025"
                sp[f"drift_per_1e4_fp32_surrogate{sfx}"] = a["drift_per_1e4"]
                sp[f"drift_per_1e4_fp64_newton{sfx}"] = b["drift_per_1e4"]
                sp[f"drift_diff_over_combined_se{sfx}"] = \
                    abs(a["drift_per_1e4"][0] - b["drift_per_1e4"][0]) / \
                    max(1e-300, math.hypot(a["drift_per_1e4"][1], b["drift_per_1e4"][1]))
    if not args.no_cpu:
        log(f"[bench] CPU oracle: {args.cpu_steps} steps at N={n}")
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_steps, 1, dt, eps0)
    # the paper's only timing of SER (its benchmark table in the section on
    # equilibrium simulations): context, not a target -- another potential,
    # another workload and one core of an unstated CPU
    line["paper_context"] = {
        "value": 1.0 / 7.85e-5, "unit": "particle-steps/s per core",
        "hardware": "one CPU core, model not stated",
        "workload": "SER with projection, splined LJ, density 0.8095, C_v 10, sigma 2, "
                    "N = 144,000 over 8 processors",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
