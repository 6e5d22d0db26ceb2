"""ctypes binding of libdpde.so: the same entry points as include/dpde.h.

Argument marshalling only.  Device arrays are torch CUDA tensors (float64,
contiguous); every computation happens in the HIP library.  Importing this
module without the built library raises immediately: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpde.so")

DPDE_OK, DPDE_EINVAL, DPDE_EBOX, DPDE_ENOMEM, DPDE_EHIP = 0, -1, -2, -3, -4
DPDE_ENEG_EINT, DPDE_EEOS, DPDE_EOVERFLOW, DPDE_ENONFINITE = -5, -6, -7, -8
DPDE_ERANGE = -9
DPDE_EIO = -10
FP64, FP32 = 0, 1
EOS_LINEAR, EOS_EINSTEIN = 0, 1
THETA_NEWTON, THETA_MLP, THETA_MLP_NEWTON = 0, 1, 2
SCHEME_SER, SCHEME_SEM, SCHEME_HYBRID = 0, 1, 2
MODEL_VECTOR, MODEL_PROJECTED = 0, 1
POT_SOFT, POT_LJ = 0, 1
DPDE_FLAG_REGENERATE_NOISE = 1
DPDE_FLAG_PROJECT_EINT = 2
REC_LEN = 12
MLP_NPARAM = 1153

ERROR_NAMES = {
    DPDE_EINVAL: "DPDE_EINVAL", DPDE_EBOX: "DPDE_EBOX", DPDE_ENOMEM: "DPDE_ENOMEM",
    DPDE_EHIP: "DPDE_EHIP", DPDE_ENEG_EINT: "DPDE_ENEG_EINT", DPDE_EEOS: "DPDE_EEOS",
    DPDE_EOVERFLOW: "DPDE_EOVERFLOW", DPDE_ENONFINITE: "DPDE_ENONFINITE",
    DPDE_ERANGE: "DPDE_ERANGE", DPDE_EIO: "DPDE_EIO",
}


class Params(C.Structure):
    """Mirror of struct dpde_params."""
    _fields_ = [
        ("n", C.c_int64),
        ("box", C.c_double * 3),
        ("mass", C.c_double), ("rc", C.c_double), ("a", C.c_double), ("gamma", C.c_double),
        ("kT_ref", C.c_double), ("dt", C.c_double), ("cv", C.c_double),
        ("eos_n", C.c_double), ("eos_omega", C.c_double), ("eos_c0", C.c_double),
        ("eps_lj", C.c_double), ("r_lj", C.c_double),
        ("skin", C.c_double),
        ("seed", C.c_uint64), ("step0", C.c_int64),
        ("periodic", C.c_int32 * 3),
        ("eos", C.c_int32), ("precision", C.c_int32), ("theta_mode", C.c_int32),
        ("scheme", C.c_int32), ("model", C.c_int32), ("potential", C.c_int32),
        ("replica", C.c_uint32), ("neighbor_cap", C.c_int32),
        ("flags", C.c_int32),
        ("ndom", C.c_int32 * 3),
    ]


class Shape(C.Structure):
    """Mirror of struct dpde_shape."""
    _fields_ = [("pair_block", C.c_int32), ("aux_block", C.c_int32), ("pairs", C.c_int32),
                ("order_block", C.c_int32)]


PAIRS_BOTH_SIDES, PAIRS_ONCE_PER_TILE = 0, 1


class MlpCfg(C.Structure):
    """Mirror of struct dpde_mlp_cfg."""
    _fields_ = [
        ("theta_lo", C.c_double), ("theta_hi", C.c_double),
        ("nsamples", C.c_int64), ("iters", C.c_int64),
        ("batch", C.c_int32), ("pad", C.c_int32),
        ("lr", C.c_double), ("seed", C.c_uint64),
    ]


class DpdeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


# (name, restype, argtypes) of every exported entry point
_vp = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int32
_dp = C.POINTER(C.c_double)
SIGNATURES = [
    ("dpde_init", C.c_int, [C.POINTER(Params), _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
    ("dpde_step", C.c_int, [_vp, _i64]),
    ("dpde_energies", C.c_int, [_vp, _dp]),
    ("dpde_history", C.c_int, [_vp, _dp, _i64, C.POINTER(_i64)]),
    ("dpde_get_state", C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(_i64)]),
    ("dpde_set_state", C.c_int, [_vp, _vp, _vp, _vp, _i64]),
    ("dpde_forces", C.c_int, [_vp, _vp, _dp]),
    ("dpde_free", C.c_int, [_vp]),
    ("dpde_list_builds", C.c_int, [_vp, C.POINTER(_i64)]),
    ("dpde_last_error", C.c_char_p, []),
    ("dpde_stream", _vp, [_vp]),
    ("dpde_init_batch", C.c_int, [C.POINTER(Params), _i32, C.POINTER(_i64), _vp, _vp, _vp, _vp,
                                  C.POINTER(_vp)]),
    ("dpde_energies_batch", C.c_int, [_vp, _dp]),
    ("dpde_step_graph", C.c_int, [_vp, _i64, _i64]),
    ("dpde_set_tuning", C.c_int, [_vp, _i32, _i32]),
    ("dpde_get_shape", C.c_int, [_vp, C.POINTER(Shape)]),
    ("dpde_set_shape", C.c_int, [_vp, C.POINTER(Shape)]),
    ("dpde_autotune", C.c_int, [_vp, _i32, C.POINTER(_i32), C.POINTER(_i32), _dp]),
    ("dpde_tuning_load", C.c_int, [C.c_char_p]),
    ("dpde_tuning_save", C.c_int, [C.c_char_p]),
    ("dpde_tuning_clear", C.c_int, []),
    ("dpde_tuning_lookup", C.c_int, [_i64, _i32, _i32, C.POINTER(Shape), _dp,
                                     C.POINTER(_i32)]),
    ("dpde_profile_enable", C.c_int, [_vp, _i32]),
    ("dpde_profile_read", C.c_int, [_vp, C.c_char_p, _dp, C.POINTER(_i64), _i32]),
    ("dpde_theta", C.c_int, [_vp, _vp, _vp, _vp, _i64, _i32]),
    ("dpde_eos_energy", C.c_int, [_vp, _vp, _vp, _i64]),
    ("dpde_mlp_train", C.c_int, [_vp, C.POINTER(MlpCfg), C.POINTER(C.c_float)]),
    ("dpde_mlp_get", C.c_int, [_vp, C.POINTER(C.c_float), _dp]),
    ("dpde_mlp_set", C.c_int, [_vp, C.POINTER(C.c_float), _dp]),
    ("dpde_mlp_grad", C.c_int, [_vp, _vp, _vp, _i64, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    ("dpde_mlp_grad_noalloc", C.c_int, [_vp, _vp, _vp, _i64, C.POINTER(C.c_float),
                                        C.POINTER(C.c_float)]),
    ("dpde_mlp_eval", C.c_int, [_vp, _vp, _vp, _i64]),
    ("dpde_debug_cells", C.c_int, [_vp, _vp]),
    ("dpde_debug_order", C.c_int, [_vp, _vp]),
    ("dpde_debug_inv_temperature", C.c_int, [_vp, _vp]),
    ("dpde_debug_list_lengths", C.c_int, [_vp, _vp]),
    ("dpde_debug_pairs", C.c_int, [_vp, _vp, _i64, C.POINTER(_i64)]),
    ("dpde_debug_rng", C.c_int, [C.c_uint64, C.c_uint32, _i64, _vp, _vp, _i64, _vp, _vp, _vp]),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libdpde.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; "
                          f"g.build()'` (or python paper_1507_06643_amd/build.py)")
    L = C.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc: int):
    if rc != DPDE_OK:
        raise DpdeError(rc, load().dpde_last_error().decode())
    return rc
