"""ctypes view of the C oracle plus a few pure-numpy helpers.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  Nothing in the product package imports it.

All arrays are float64 in particle-ID order: q and p of shape (n,3), eps (n,).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import build as _build

OR_OK, OR_EINVAL, OR_EBOX, OR_ENOMEM, OR_ENEG_EINT, OR_EEOS = 0, -1, -2, -3, -5, -6


class OrParams(C.Structure):
    _fields_ = [
        ("box", C.c_double * 3),
        ("mass", C.c_double), ("rc", C.c_double), ("a", C.c_double), ("gamma", C.c_double),
        ("kT_ref", C.c_double), ("dt", C.c_double),
        ("cv", C.c_double), ("eos_n", C.c_double), ("eos_omega", C.c_double), ("eos_c0", C.c_double),
        ("n", C.c_int64), ("step", C.c_int64), ("seed", C.c_uint64),
        ("periodic", C.c_int32 * 3),
        ("eos", C.c_int32), ("replica", C.c_int32), ("scheme", C.c_int32),
        ("project", C.c_int32), ("model", C.c_int32), ("potential", C.c_int32),
        ("pad_", C.c_int32),
        ("E0", C.c_double), ("eps_lj", C.c_double), ("r_lj", C.c_double),
        ("ndom", C.c_int32 * 3), ("pad2_", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        u32p = C.POINTER(C.c_uint32)
        P = C.POINTER(OrParams)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_pair_words.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32, C.c_uint32, u32p]
        L.or_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32, C.c_uint32, dp]
        L.or_wrap.argtypes = [C.c_double, C.c_double]
        L.or_wrap.restype = C.c_double
        L.or_cell_index.argtypes = [P, dp]
        L.or_cell_index.restype = C.c_int64
        L.or_check_box.argtypes = [P]
        for f in (L.or_pairs_brute, L.or_pairs_cells):
            f.argtypes = [P, dp, i64p, i32p, C.c_int64]
        L.or_forces.argtypes = [P, dp, dp, dp]
        L.or_forces_pairs.argtypes = [P, dp, i32p, C.c_int64, dp, dp]
        L.or_eos_energy.argtypes = [P, C.c_double]
        L.or_eos_energy.restype = C.c_double
        L.or_eos_cv.argtypes = [P, C.c_double]
        L.or_eos_cv.restype = C.c_double
        L.or_theta_newton.argtypes = [P, C.c_double, C.POINTER(C.c_int)]
        L.or_theta_newton.restype = C.c_double
        L.or_inv_temperature.argtypes = [P, dp, dp]
        L.or_fd_pairs.argtypes = [P, dp, dp, dp, i32p, C.c_int64, dp]
        L.or_fd.argtypes = [P, dp, dp, dp, dp]
        L.or_step.argtypes = [P, dp, dp, dp, dp, dp]
        L.or_run.argtypes = [P, dp, dp, dp, dp, dp, C.c_int64, dp]
        L.or_energies.argtypes = [P, dp, dp, C.c_double, dp]
        L.or_project.argtypes = [P, dp, C.c_double, C.c_double]
        L.or_pair_potential.argtypes = [P, C.c_double, dp, dp, dp]
        L.or_config_temperature.argtypes = [P, dp, dp, dp]
        L.or_mlp_nparam.restype = C.c_int
        L.or_mlp_forward.argtypes = [dp, dp, dp, C.c_int64]
        L.or_mlp_loss_grad.argtypes = [dp, dp, dp, C.c_int64, dp]
        L.or_mlp_loss_grad.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(n, box, *, periodic=(1, 1, 1), mass=1.0, rc=1.0, a=25.0, gamma=4.5, kT_ref=1.0,
                dt=0.01, eos=0, cv=100.0, eos_n=50.0, eos_omega=2.0, eos_c0=10.0, seed=7, step=0,
                replica=0, scheme=0, project=0, E0=0.0, model=0, potential=0, eps_lj=1.0,
                r_lj=1.0, ndom=(1, 1, 1)) -> OrParams:
    P = OrParams()
    P.box = (C.c_double * 3)(*[float(x) for x in box])
    P.mass, P.rc, P.a, P.gamma, P.kT_ref, P.dt = mass, rc, a, gamma, kT_ref, dt
    P.cv, P.eos_n, P.eos_omega, P.eos_c0 = cv, eos_n, eos_omega, eos_c0
    P.n, P.step, P.seed = int(n), int(step), int(seed)
    P.periodic = (C.c_int32 * 3)(*[int(x) for x in periodic])
    P.eos, P.replica, P.scheme = int(eos), int(replica), int(scheme)
    P.project, P.model, P.potential = int(project), int(model), int(potential)
    P.E0, P.eps_lj, P.r_lj = float(E0), float(eps_lj), float(r_lj)
    P.ndom = (C.c_int32 * 3)(*[int(x) for x in ndom])
    return P


def check(rc, what="oracle"):
    if rc != OR_OK:
        raise RuntimeError(f"{what} failed with code {rc}")


# ---- RNG ---------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return list(o)


def pair_words(seed, replica, step, lo, hi):
    o = (C.c_uint32 * 4)()
    lib().or_pair_words(seed, replica, step, lo, hi, o)
    return list(o)


def gauss3(seed, replica, step, lo, hi):
    g = (C.c_double * 3)()
    lib().or_gauss3(seed, replica, step, lo, hi, g)
    return np.array(list(g))


# ---- geometry ----------------------------------------------------------------
def cell_index(P, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    return np.array([lib().or_cell_index(C.byref(P), _d(q[i])) for i in range(q.shape[0])],
                    dtype=np.int64)


def pairs(P, q, method="cells"):
    q = np.ascontiguousarray(q, dtype=np.float64)
    f = lib().or_pairs_cells if method == "cells" else lib().or_pairs_brute
    cap = 16 * q.shape[0] + 64
    while True:
        buf = np.zeros((cap, 2), dtype=np.int32)
        m = C.c_int64(0)
        rc = f(C.byref(P), _d(q), C.byref(m), buf.ctypes.data_as(C.POINTER(C.c_int32)), cap)
        if rc == OR_ENOMEM and m.value > cap:
            cap = m.value + 64
            continue
        check(rc, "pairs")
        out = buf[: m.value].copy()
        if method != "cells":
            out = out[np.lexsort((out[:, 1], out[:, 0]))]
        return out


# ---- dynamics ----------------------------------------------------------------
def forces(P, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    F = np.zeros_like(q)
    U = C.c_double(0.0)
    check(lib().or_forces(C.byref(P), _d(q), _d(F), C.byref(U)), "forces")
    return F, U.value


def fd(P, q, p, eps):
    """FD sub-step alone at fixed q; returns new (p, eps, dp)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    p = np.array(p, dtype=np.float64, copy=True)
    eps = np.array(eps, dtype=np.float64, copy=True)
    dp = np.zeros_like(p)
    rc = lib().or_fd(C.byref(P), _d(q), _d(p), _d(eps), _d(dp))
    return rc, p, eps, dp


class State:
    """Oracle trajectory state in ID order (q, p, eps, F, U, step).  With
    P.project set, the target energy E0 of the projection is the energy of the
    initial state (Sec. 4.2)."""

    def __init__(self, P, q, p, eps):
        self.P = P
        self.q = np.array(q, dtype=np.float64, copy=True)
        self.p = np.array(p, dtype=np.float64, copy=True)
        self.eps = np.array(eps, dtype=np.float64, copy=True)
        self.F, self.U = forces(P, self.q)
        if P.project:
            P.E0 = self.energies()[3]

    def step(self, nsteps=1, record=False):
        rec = np.zeros((nsteps, 10)) if record else None
        U = C.c_double(self.U)
        rc = lib().or_run(C.byref(self.P), _d(self.q), _d(self.p), _d(self.eps), _d(self.F),
                          C.byref(U), int(nsteps), _d(rec) if record else None)
        self.U = U.value
        return rc, rec

    def energies(self):
        out = np.zeros(10)
        check(lib().or_energies(C.byref(self.P), _d(self.p), _d(self.eps), C.c_double(self.U),
                                _d(out)), "energies")
        return out


def pair_potential(P, r):
    """(v, v', v'') of the pair potential at distance r."""
    v, dv, d2v = C.c_double(), C.c_double(), C.c_double()
    lib().or_pair_potential(C.byref(P), float(r), C.byref(v), C.byref(dv), C.byref(d2v))
    return v.value, dv.value, d2v.value


def config_temperature_terms(P, q):
    """(|grad U|^2, Laplacian of U) for the configurational temperature."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    g, l = C.c_double(), C.c_double()
    check(lib().or_config_temperature(C.byref(P), _d(q), C.byref(g), C.byref(l)), "config T")
    return g.value, l.value


def energies(P, p, eps, U):
    out = np.zeros(10)
    p = np.ascontiguousarray(p, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    check(lib().or_energies(C.byref(P), _d(p), _d(eps), C.c_double(U), _d(out)), "energies")
    return out


# ---- equation of state ---------------------------------------------------------
def eos_energy(P, theta):
    return np.array([lib().or_eos_energy(C.byref(P), float(t)) for t in np.atleast_1d(theta)])


def eos_cv(P, theta):
    return np.array([lib().or_eos_cv(C.byref(P), float(t)) for t in np.atleast_1d(theta)])


def theta_newton(P, eps):
    out = np.zeros(len(np.atleast_1d(eps)))
    its = np.zeros(len(out), dtype=np.int64)
    for k, e in enumerate(np.atleast_1d(eps)):
        it = C.c_int(0)
        out[k] = lib().or_theta_newton(C.byref(P), float(e), C.byref(it))
        its[k] = it.value
    return out, its


# ---- surrogate MLP (FP64) --------------------------------------------------------
MLP_H = 32


def mlp_nparam():
    return lib().or_mlp_nparam()


def mlp_forward(w, x):
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    lib().or_mlp_forward(_d(w), _d(x), _d(y), len(x))
    return y


def mlp_loss_grad(w, x, t):
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    g = np.zeros_like(w)
    loss = lib().or_mlp_loss_grad(_d(w), _d(x), _d(t), len(x), _d(g))
    return loss, g


def sigma_of(P):
    """sigma = sqrt(2 gamma kT_ref) (eq. alternative_FDR with k_B = 1)."""
    return math.sqrt(2.0 * P.gamma * P.kT_ref)
