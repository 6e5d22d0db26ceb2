"""Build the tuning table of launch shapes on this GPU.

Runs the library's autotuner on one system of each size class of the
workloads, in FP64 and FP32, and writes the table that dpde_tuning_load reads
(one line per size class, replica class and precision):

    python -m paper_1507_06643_amd.tune --out paper_1507_06643_amd/tuning_gfx950.txt

The systems are the synthetic workloads: plain DPDE at density 3 with
N = 1000 and 65,536, the shock box 400 x 20 x 20 (N = 480,000), the learned
EOS at N = 1,048,576 and 256 replicas of 500..8000 particles.  Tuning leaves
every trajectory as the chosen shape would give it, so the table only decides
speed.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

import paper_1507_06643_amd as dp

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import workloads as W  # noqa: E402


def _einstein_eps0():
    """eps(theta = 1) from the library's Einstein EOS (a small helper handle)."""
    nh = 200
    Lh = W.cubic_side(nh)
    q, p, e = W.equilibrium_state(nh, [Lh] * 3, eps0=10.0, seed=1)
    h = dp.System(dp.Config(n=nh, box=[Lh] * 3, eos=dp.EOS_EINSTEIN), q, p, e)
    eps0 = float(h.eos_energy(torch.ones(1, dtype=torch.float64)).cpu()[0])
    h.close()
    return eps0


def _cases(precisions):
    for prec in precisions:
        for n, dt in ((1000, 0.01), (65536, 0.005)):
            L = W.cubic_side(n)
            q, p, e = W.equilibrium_state(n, [L] * 3, seed=n)
            yield (f"plain N={n}", prec,
                   lambda n=n, L=L, q=q, p=p, e=e, dt=dt, prec=prec: dp.System(
                       dp.Config(n=n, box=[L] * 3, dt=dt, precision=prec), q, p, e))
        q, p, e = W.shock_state()
        yield ("shock N=480000", prec, lambda q=q, p=p, e=e, prec=prec: dp.System(
            dp.Config(n=len(q), box=[400.0, 20.0, 20.0], periodic=[0, 1, 1], dt=0.005,
                      precision=prec), q, p, e))

        def learned(prec=prec):
            n = 1_048_576
            L = W.cubic_side(n)
            q, p, e = W.equilibrium_state(n, [L] * 3, eps0=_einstein_eps0())
            s = dp.System(dp.Config(n=n, box=[L] * 3, dt=0.005, eos=dp.EOS_EINSTEIN,
                                    theta_mode=dp.THETA_MLP, precision=prec), q, p, e)
            s.mlp_train(nsamples=10**6, iters=2000, batch=4096, lr=3e-3)
            return s
        yield ("learned EOS N=1048576", prec, learned)

        def batched(prec=prec):
            sizes, seeds = W.replica_sizes(256, 500, 8000, seed=20260103)
            cfgs, qs, ps, es = [], [], [], []
            for r, (nr, sd) in enumerate(zip(sizes, seeds)):
                L = W.cubic_side(int(nr))
                q, p, e = W.equilibrium_state(int(nr), [L] * 3, seed=30000 + r)
                cfgs.append(dp.Config(n=int(nr), box=[L] * 3, dt=0.01, seed=int(sd), replica=r,
                                      precision=prec))
                qs.append(q); ps.append(p); es.append(e)
            return dp.System(cfgs, np.concatenate(qs), np.concatenate(ps), np.concatenate(es))
        yield ("256 replicas", prec, batched)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tuning_gfx950.txt"))
    ap.add_argument("--steps", type=int, default=20, help="timed steps per candidate shape")
    ap.add_argument("--fp64-only", action="store_true")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    dp.tuning_clear()
    precs = (dp.FP64,) if args.fp64_only else (dp.FP64, dp.FP32)
    for name, prec, make in _cases(precs):
        t0 = time.perf_counter()
        s = make()
        s.step(10)
        s.autotune(args.steps)
        sh = s.get_shape()
        got = dp.tuning_lookup(s.n, s.nrep, prec)
        s.close()
        print(f"[tune] {name} {'fp64' if prec == dp.FP64 else 'fp32'}: {sh} "
              f"{got[1]:.4f} ms/step ({time.perf_counter() - t0:.1f} s)", flush=True)
    dp.tuning_save(args.out)
    print(f"[tune] table written to {args.out}", flush=True)


if __name__ == "__main__":
    main()
