"""The C ABI: every function declared in include/dpde.h is exported by
libdpde.so and bound by the Python layer, and the ctypes structures have the
C layout (checked by compiling a probe against the header with gcc)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpde.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpde_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_core_boundary():
    names = _declared()
    for core in ("dpde_init", "dpde_step", "dpde_energies", "dpde_free", "dpde_last_error"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1507_06643_amd import _lib as L
    lib = L.load()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (dpde_[a-z0-9_]+)", out))
    declared = set(_declared())
    assert declared <= exported, declared - exported
    bound = {name for name, _, _ in L.SIGNATURES}
    assert declared == bound, declared ^ bound
    for name in declared:
        assert getattr(lib, name) is not None


def test_struct_layouts_match_c(tmp_path):
    from paper_1507_06643_amd import _lib as L
    fields = [f for f, _ in L.Params._fields_]
    mfields = [f for f, _ in L.MlpCfg._fields_ if f != "pad"]
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){",
             'printf("%zu %zu\\n", sizeof(dpde_params), sizeof(dpde_mlp_cfg));']
    for f in fields:
        lines.append(f'printf("P {f} %zu\\n", offsetof(dpde_params, {f}));')
    for f in mfields:
        lines.append(f'printf("M {f} %zu\\n", offsetof(dpde_mlp_cfg, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sp, sm = map(int, out[0].split())
    assert sp == C.sizeof(L.Params) and sm == C.sizeof(L.MlpCfg)
    for line in out[1:]:
        if not line:
            continue
        kind, f, off = line.split()
        cls = L.Params if kind == "P" else L.MlpCfg
        assert getattr(cls, f).offset == int(off), f


def test_errors_without_gpu_are_reported_not_raised():
    """Calls that fail validation return codes (no GPU work is issued)."""
    from paper_1507_06643_amd import _lib as L
    lib = L.load()
    h = C.c_void_p()
    P = L.Params()
    P.n = 1  # n < 2
    rc = lib.dpde_init(C.byref(P), None, None, None, None, C.byref(h))
    assert rc == L.DPDE_EINVAL
    assert b"n = 1" in lib.dpde_last_error()
    assert lib.dpde_step(None, 1) == L.DPDE_EINVAL
    assert lib.dpde_free(None) == L.DPDE_OK


def test_box_rule_reported():
    from paper_1507_06643_amd import _lib as L
    lib = L.load()
    h = C.c_void_p()
    P = L.Params()
    P.n, P.mass, P.rc, P.dt, P.kT_ref, P.cv, P.gamma, P.a = 10, 1.0, 1.0, 0.01, 1.0, 100.0, 4.5, 25.0
    P.box = (C.c_double * 3)(2.5, 5.0, 5.0)
    P.periodic = (C.c_int32 * 3)(1, 1, 1)
    dummy = C.c_void_p(16)  # never dereferenced: the box check fails first
    rc = lib.dpde_init(C.byref(P), dummy, dummy, dummy, None, C.byref(h))
    assert rc == L.DPDE_EBOX, lib.dpde_last_error()


def test_build_script_loads_without_the_built_library():
    """build() must work in a fresh checkout, where libdpde.so does not exist
    yet: it loads the HIP build script by path, and that import does not pull
    in the package (whose import loads the library)."""
    code = ("import sys, __graft_entry__ as g; "
            "m = g._load_file('_b', 'paper_1507_06643_amd/build.py'); "
            "assert callable(m.build) and m.LIB.endswith('libdpde.so'); "
            "assert 'paper_1507_06643_amd' not in sys.modules")
    subprocess.run(["python3", "-c", code], cwd=ROOT, check=True)
