"""Python face of libdpde.so: a handle object whose methods mirror the C ABI.

Only marshalling happens here (torch tensors <-> device pointers, ctypes
structures); all arithmetic of the method runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


@dataclass
class Config:
    """Parameters of one system (fields of struct dpde_params)."""
    n: int
    box: Sequence[float]
    periodic: Sequence[int] = (1, 1, 1)
    mass: float = 1.0
    rc: float = 1.0
    a: float = 25.0
    gamma: float = 4.5
    kT_ref: float = 1.0
    dt: float = 0.01
    eos: int = L.EOS_LINEAR
    cv: float = 100.0
    eos_n: float = 50.0
    eos_omega: float = 2.0
    eos_c0: float = 10.0
    skin: float = 0.3
    model: int = L.MODEL_VECTOR
    potential: int = L.POT_SOFT
    eps_lj: float = 1.0
    r_lj: float = 1.0
    project: bool = False
    ndom: Sequence[int] = (1, 1, 1)
    precision: int = L.FP64
    theta_mode: int = L.THETA_NEWTON
    scheme: int = L.SCHEME_SER
    seed: int = 7
    step0: int = 0
    replica: int = 0
    neighbor_cap: int = 0

    def to_c(self) -> L.Params:
        P = L.Params()
        P.n = int(self.n)
        P.box = (C.c_double * 3)(*[float(x) for x in self.box])
        P.mass, P.rc, P.a, P.gamma = self.mass, self.rc, self.a, self.gamma
        P.kT_ref, P.dt, P.cv = self.kT_ref, self.dt, self.cv
        P.eos_n, P.eos_omega, P.eos_c0 = self.eos_n, self.eos_omega, self.eos_c0
        P.skin = float(self.skin)
        P.eps_lj, P.r_lj = float(self.eps_lj), float(self.r_lj)
        P.model, P.potential = int(self.model), int(self.potential)
        P.seed, P.step0 = int(self.seed) & (2**64 - 1), int(self.step0)
        P.periodic = (C.c_int32 * 3)(*[int(x) for x in self.periodic])
        P.eos, P.precision, P.theta_mode, P.scheme = (int(self.eos), int(self.precision),
                                                       int(self.theta_mode), int(self.scheme))
        P.replica, P.neighbor_cap = int(self.replica), int(self.neighbor_cap)
        P.flags = L.DPDE_FLAG_PROJECT_EINT if self.project else 0
        P.ndom = (C.c_int32 * 3)(*[int(x) for x in self.ndom])
        return P


def _dev(x, dtype=torch.float64):
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.asarray(x))
    return x.to(device="cuda", dtype=dtype).contiguous()


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class System:
    """One dpde_handle (a single system or a batch of replicas)."""

    def __init__(self, cfg, q, p, eps, offsets=None):
        lib = L.load()
        self._lib = lib
        self.h = C.c_void_p()
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        qd, pd, ed = _dev(q), _dev(p), _dev(eps)
        if isinstance(cfg, (list, tuple)):
            cfgs = list(cfg)
            self.nrep = len(cfgs)
            arr = (L.Params * self.nrep)(*[c.to_c() for c in cfgs])
            offs = np.zeros(self.nrep + 1, dtype=np.int64)
            offs[1:] = np.cumsum([c.n for c in cfgs])
            self.offsets = offs
            o = (C.c_int64 * (self.nrep + 1))(*[int(v) for v in offs])
            L.check(lib.dpde_init_batch(arr, self.nrep, o, _ptr(qd), _ptr(pd), _ptr(ed), stream,
                                        C.byref(self.h)))
            self.n = int(offs[-1])
        else:
            self.nrep = 1
            self.n = int(cfg.n)
            self.offsets = np.array([0, self.n], dtype=np.int64)
            P = cfg.to_c()
            L.check(lib.dpde_init(C.byref(P), _ptr(qd), _ptr(pd), _ptr(ed), stream,
                                  C.byref(self.h)))
        self.cfg = cfg

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if self.h:
            self._lib.dpde_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping -------------------------------------------------------------
    def step(self, nsteps: int = 1) -> int:
        return L.check(self._lib.dpde_step(self.h, int(nsteps)))

    def step_raw(self, nsteps: int = 1) -> int:
        """dpde_step returning the error code instead of raising."""
        return self._lib.dpde_step(self.h, int(nsteps))

    def step_graph(self, nsteps: int, reps: int = 1) -> int:
        return L.check(self._lib.dpde_step_graph(self.h, int(nsteps), int(reps)))

    def list_builds(self) -> int:
        b = C.c_int64(0)
        L.check(self._lib.dpde_list_builds(self.h, C.byref(b)))
        return b.value

    def set_tuning(self, pair_block: int, aux_block: int = 256):
        L.check(self._lib.dpde_set_tuning(self.h, int(pair_block), int(aux_block)))

    def get_shape(self) -> dict:
        sh = L.Shape()
        L.check(self._lib.dpde_get_shape(self.h, C.byref(sh)))
        return {"pair_block": sh.pair_block, "aux_block": sh.aux_block, "pairs": sh.pairs,
                "order_block": sh.order_block}

    def set_shape(self, pair_block=None, aux_block=None, pairs=None, order_block=None):
        cur = self.get_shape()
        pick = lambda v, k: int(v if v is not None else cur[k])
        sh = L.Shape(pick(pair_block, "pair_block"), pick(aux_block, "aux_block"),
                     pick(pairs, "pairs"), pick(order_block, "order_block"))
        L.check(self._lib.dpde_set_shape(self.h, C.byref(sh)))

    def autotune(self, steps: int = 20):
        """Pick the fastest launch shape (state restored) and record it in the
        library's tuning table; returns (pair block, aux block, ms/step) (the
        full shape: get_shape())."""
        pb, ab, ms = C.c_int32(0), C.c_int32(0), C.c_double(0.0)
        L.check(self._lib.dpde_autotune(self.h, int(steps), C.byref(pb), C.byref(ab), C.byref(ms)))
        return pb.value, ab.value, ms.value

    @property
    def stream_ptr(self) -> int:
        return self._lib.dpde_stream(self.h) or 0

    # -- observables ------------------------------------------------------------
    def energies(self) -> np.ndarray:
        if self.nrep > 1:
            out = np.zeros((self.nrep, L.REC_LEN))
            L.check(self._lib.dpde_energies_batch(self.h, out.ctypes.data_as(C.POINTER(C.c_double))))
            return out
        out = np.zeros(L.REC_LEN)
        L.check(self._lib.dpde_energies(self.h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def history(self, cap: int = 1 << 16) -> np.ndarray:
        out = np.zeros((cap, self.nrep, L.REC_LEN))
        cnt = C.c_int64(0)
        L.check(self._lib.dpde_history(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), cap,
                                       C.byref(cnt)))
        out = out[: cnt.value]
        return out[:, 0, :] if self.nrep == 1 else out

    def get_state(self):
        q = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        p = torch.empty_like(q)
        e = torch.empty(self.n, dtype=torch.float64, device="cuda")
        step = C.c_int64(0)
        L.check(self._lib.dpde_get_state(self.h, _ptr(q), _ptr(p), _ptr(e), C.byref(step)))
        return q, p, e, step.value

    def set_state(self, q, p, eps, step: int):
        qd, pd, ed = _dev(q), _dev(p), _dev(eps)
        torch.cuda.synchronize()
        L.check(self._lib.dpde_set_state(self.h, _ptr(qd), _ptr(pd), _ptr(ed), int(step)))

    def forces(self):
        F = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        U = C.c_double(0.0)
        L.check(self._lib.dpde_forces(self.h, _ptr(F), C.byref(U)))
        return F, U.value

    # -- profiling ----------------------------------------------------------------
    def profile(self, enable: bool):
        L.check(self._lib.dpde_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self, nmax: int = 64):
        names = C.create_string_buffer(32 * nmax)
        ms = np.zeros(nmax)
        cnt = np.zeros(nmax, dtype=np.int64)
        k = self._lib.dpde_profile_read(self.h, names, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                        cnt.ctypes.data_as(C.POINTER(C.c_int64)), nmax)
        if k < 0:
            L.check(k)
        raw = names.raw
        out = {}
        for i in range(k):
            nm = raw[32 * i: 32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(cnt[i]))
        return out

    # -- equation of state and surrogate --------------------------------------------
    def theta(self, eps, mode: int = L.THETA_NEWTON):
        e = _dev(eps)
        th = torch.empty_like(e)
        it = torch.empty(e.shape, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        L.check(self._lib.dpde_theta(self.h, _ptr(e), _ptr(th), _ptr(it), e.numel(), int(mode)))
        return th, it

    def eos_energy(self, theta):
        th = _dev(theta)
        e = torch.empty_like(th)
        torch.cuda.synchronize()
        L.check(self._lib.dpde_eos_energy(self.h, _ptr(th), _ptr(e), th.numel()))
        return e

    def mlp_train(self, theta_lo=0.2, theta_hi=20.0, nsamples=10**6, iters=4000, batch=4096,
                  lr=3e-3, seed=11):
        cfg = L.MlpCfg(theta_lo, theta_hi, int(nsamples), int(iters), int(batch), 0, float(lr),
                       int(seed))
        curve = np.zeros(max(1, iters), dtype=np.float32)
        L.check(self._lib.dpde_mlp_train(self.h, C.byref(cfg),
                                         curve.ctypes.data_as(C.POINTER(C.c_float))))
        return curve[:iters]

    def mlp_get(self):
        w = np.zeros(L.MLP_NPARAM, dtype=np.float32)
        norm = np.zeros(4)
        L.check(self._lib.dpde_mlp_get(self.h, w.ctypes.data_as(C.POINTER(C.c_float)),
                                       norm.ctypes.data_as(C.POINTER(C.c_double))))
        return w, norm

    def mlp_set(self, w, norm):
        w = np.ascontiguousarray(w, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float64)
        L.check(self._lib.dpde_mlp_set(self.h, w.ctypes.data_as(C.POINTER(C.c_float)),
                                       norm.ctypes.data_as(C.POINTER(C.c_double))))

    def mlp_grad(self, x, t):
        xd = _dev(x, torch.float32)
        td = _dev(t, torch.float32)
        loss = C.c_float(0.0)
        g = np.zeros(L.MLP_NPARAM, dtype=np.float32)
        torch.cuda.synchronize()
        L.check(self._lib.dpde_mlp_grad(self.h, _ptr(xd), _ptr(td), xd.numel(), C.byref(loss),
                                        g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def mlp_grad_noalloc(self, x, t):
        """dpde_mlp_grad_noalloc: the gradient with the library's static buffer."""
        xd = _dev(x, torch.float32)
        td = _dev(t, torch.float32)
        loss = C.c_float(0.0)
        g = np.zeros(L.MLP_NPARAM, dtype=np.float32)
        torch.cuda.synchronize()
        L.check(self._lib.dpde_mlp_grad_noalloc(self.h, _ptr(xd), _ptr(td), xd.numel(),
                                                C.byref(loss),
                                                g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def mlp_eval(self, x):
        xd = _dev(x, torch.float32)
        y = torch.empty_like(xd)
        torch.cuda.synchronize()
        L.check(self._lib.dpde_mlp_eval(self.h, _ptr(xd), _ptr(y), xd.numel()))
        return y

    # -- test hooks -------------------------------------------------------------------
    def debug_cells(self):
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        L.check(self._lib.dpde_debug_cells(self.h, _ptr(out)))
        return out

    def debug_order(self):
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        L.check(self._lib.dpde_debug_order(self.h, _ptr(out)))
        return out

    def debug_inv_temperature(self):
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        L.check(self._lib.dpde_debug_inv_temperature(self.h, _ptr(out)))
        return out

    def debug_list_lengths(self):
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        L.check(self._lib.dpde_debug_list_lengths(self.h, _ptr(out)))
        return out

    def mean_work_list(self) -> float:
        return float(self.debug_list_lengths().double().mean().item())

    def debug_pairs(self, cap=None):
        cap = cap if cap is not None else 40 * self.n
        out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
        cnt = C.c_int64(0)
        L.check(self._lib.dpde_debug_pairs(self.h, _ptr(out), cap, C.byref(cnt)))
        if cnt.value > cap:
            return self.debug_pairs(cnt.value + 16)
        pr = out[: cnt.value].cpu().numpy()
        order = np.lexsort((pr[:, 1], pr[:, 0]))
        return pr[order]


def debug_rng(seed: int, replica: int, step: int, lo, hi):
    """Philox words and normals of pairs (lo[k], hi[k]) computed on the GPU."""
    lib = L.load()
    lo_d = _dev(lo, torch.int32).view(torch.int32)
    hi_d = _dev(hi, torch.int32).view(torch.int32)
    n = lo_d.numel()
    raw = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    g = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    g32 = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    L.check(lib.dpde_debug_rng(int(seed) & (2**64 - 1), int(replica), int(step), _ptr(lo_d),
                               _ptr(hi_d), n, _ptr(raw), _ptr(g), _ptr(g32)))
    return (raw.cpu().numpy().view(np.uint32), g.cpu().numpy(), g32.cpu().numpy())


def tuning_load(path: str) -> None:
    """Merge a tuning-table file into the library's table."""
    lib = L.load()
    L.check(lib.dpde_tuning_load(os.fsencode(path)))


def tuning_save(path: str) -> None:
    """Write the library's tuning table."""
    lib = L.load()
    L.check(lib.dpde_tuning_save(os.fsencode(path)))


def tuning_clear() -> None:
    L.check(L.load().dpde_tuning_clear())


def tuning_lookup(n: int, nrep: int, precision: int):
    """The recorded shape for this size class, as (shape dict, ms/step), or None."""
    sh, ms, found = L.Shape(), C.c_double(0.0), C.c_int32(0)
    L.check(L.load().dpde_tuning_lookup(int(n), int(nrep), int(precision), C.byref(sh),
                                        C.byref(ms), C.byref(found)))
    if not found.value:
        return None
    return ({"pair_block": sh.pair_block, "aux_block": sh.aux_block, "pairs": sh.pairs,
             "order_block": sh.order_block}, ms.value)
