"""Seeded synthetic inputs for the DPDE workloads.

This module only draws random numbers and lays them out.  It contains none of
the method's arithmetic (no forces, no equation of state, no integrator), so
both the CPU oracle and the GPU library can be fed from it without sharing any
code with each other.

Recipe (one function per workload):
  * positions uniform in the box, momenta Maxwellian N(0, m kT) per component
    with the mean removed (zero total momentum, no rescaling), internal energy
    the same value for every particle (the caller supplies it: eps = C_v*theta
    for the linear EOS, or the nonlinear EOS evaluated at theta = 1);
  * shock: the same, plus a bulk x-velocity +u on the left half (x < Lx/2) and
    -u on the right half, added after the mean removal;
  * replicas: sizes drawn uniformly in [n_lo, n_hi], one seed per replica.
All generators use numpy's PCG64 through default_rng(seed).
"""
from __future__ import annotations

import numpy as np

DENSITY = 3.0


def cubic_side(n: int, density: float = DENSITY) -> float:
    """Side of the cube holding n particles at the given number density."""
    return float((n / density) ** (1.0 / 3.0))


def equilibrium_state(n: int, box, *, kT: float = 1.0, mass: float = 1.0, eps0: float = 100.0,
                      seed: int = 20260101):
    """Uniform positions in [0,box), Maxwell momenta with zero mean, eps_i = eps0.

    Returns (q, p, eps) as float64 arrays of shapes (n,3), (n,3), (n,).
    """
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64).reshape(3)
    q = rng.random((n, 3)) * box
    # guard against the (measure-zero) rounding of u*L up to L
    q = np.where(q >= box, 0.0, q)
    p = rng.normal(0.0, np.sqrt(mass * kT), size=(n, 3))
    p -= p.mean(axis=0, keepdims=True)
    eps = np.full(n, float(eps0), dtype=np.float64)
    return q.astype(np.float64), p.astype(np.float64), eps


def shock_state(box=(400.0, 20.0, 20.0), *, density: float = DENSITY, u: float = 2.0,
                kT: float = 1.0, mass: float = 1.0, eps0: float = 100.0, seed: int = 20260102):
    """Symmetric impact: left half +u, right half -u along x (the long axis)."""
    box = np.asarray(box, dtype=np.float64)
    n = int(round(density * box.prod()))
    q, p, eps = equilibrium_state(n, box, kT=kT, mass=mass, eps0=eps0, seed=seed)
    left = q[:, 0] < 0.5 * box[0]
    p[:, 0] += np.where(left, mass * u, -mass * u)
    return q, p, eps


def lattice_state(n_side: int, density: float, *, kT: float = 1.0, mass: float = 1.0,
                  eps0: float = 50.0, jitter: float = 0.05, seed: int = 20260105):
    """Simple cubic lattice of n_side^3 particles filling a cubic box at the
    given density, each site displaced uniformly by up to +-jitter lattice
    spacings (a crystal to melt, for the LJ potential); Maxwell momenta with
    zero mean; eps_i = eps0."""
    rng = np.random.default_rng(seed)
    n = n_side ** 3
    L = (n / density) ** (1.0 / 3.0)
    a = L / n_side
    g = (np.arange(n_side) + 0.5) * a
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    q = q + rng.uniform(-jitter * a, jitter * a, size=q.shape)
    q = np.mod(q, L)
    p = rng.normal(0.0, np.sqrt(mass * kT), size=(n, 3))
    p -= p.mean(axis=0)
    eps = np.full(n, float(eps0))
    return q, p, eps, [L, L, L]


def replica_sizes(nrep: int, n_lo: int = 500, n_hi: int = 8000, seed: int = 20260103):
    """Replica sizes uniform in [n_lo, n_hi] and one 64-bit RNG seed per replica."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=nrep)
    seeds = rng.integers(1, 2**63 - 1, size=nrep, dtype=np.int64).astype(np.uint64)
    return sizes.astype(np.int64), seeds


def theta_samples(n: int, lo: float = 0.2, hi: float = 20.0, seed: int = 20260104):
    """Training temperatures for the EOS surrogate: log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def random_pairs(n: int, npairs: int, seed: int = 5):
    """Random ordered id pairs lo < hi (for RNG word checks)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, size=npairs, dtype=np.int64)
    b = rng.integers(0, n - 1, size=npairs, dtype=np.int64)
    b = np.where(b >= a, b + 1, b)
    lo = np.minimum(a, b).astype(np.uint32)
    hi = np.maximum(a, b).astype(np.uint32)
    return lo, hi
