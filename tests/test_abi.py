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


def test_tuning_table_round_trip(tmp_path):
    """The tuning table is host-side: load, look up, save and reload without
    a GPU; malformed or out-of-range files are rejected and leave it as it was."""
    from paper_1507_06643_amd import _lib as L
    lib = L.load()
    assert lib.dpde_tuning_clear() == L.DPDE_OK
    good = tmp_path / "t.txt"
    good.write_text("# nclass rclass precision pair_block aux_block pairs order_block ms\n"
                    "20 0 0 256 512 1 2 0.655\n"
                    "  16 0 1 128 256 0 1 0.041\n"
                    "20 9 0 64 128 1 3 0.91\n")
    assert lib.dpde_tuning_load(str(good).encode()) == L.DPDE_OK

    def lookup(n, nrep, prec):
        sh, ms, found = L.Shape(), C.c_double(), C.c_int32()
        assert lib.dpde_tuning_lookup(n, nrep, prec, C.byref(sh), C.byref(ms),
                                      C.byref(found)) == L.DPDE_OK
        if not found.value:
            return None
        return (sh.pair_block, sh.aux_block, sh.pairs, sh.order_block), ms.value

    # N = 2^20 .. 2^21 - 1 is class 20; 256 replicas are class 1 + 8 = 9
    assert lookup(1_048_576, 1, 0) == ((256, 512, 1, 2), 0.655)
    assert lookup(2_097_151, 1, 0) == ((256, 512, 1, 2), 0.655)
    assert lookup(65_536, 1, 1) == ((128, 256, 0, 1), 0.041)
    assert lookup(1_100_000, 256, 0) == ((64, 128, 1, 3), 0.91)
    assert lookup(1_048_576, 1, 1) is None
    assert lookup(2_097_152, 1, 0) is None
    saved = tmp_path / "s.txt"
    assert lib.dpde_tuning_save(str(saved).encode()) == L.DPDE_OK
    assert lib.dpde_tuning_clear() == L.DPDE_OK
    assert lookup(1_048_576, 1, 0) is None
    assert lib.dpde_tuning_load(str(saved).encode()) == L.DPDE_OK
    assert lookup(65_536, 1, 1) == ((128, 256, 0, 1), 0.041)
    # rejected files leave the table unchanged
    bad = tmp_path / "b.txt"
    bad.write_text("20 0 0 256 512 1 2\n")
    assert lib.dpde_tuning_load(str(bad).encode()) == L.DPDE_EIO
    bad.write_text("12 0 0 256 512 1 9 0.1\n")  # order_block 9
    assert lib.dpde_tuning_load(str(bad).encode()) == L.DPDE_EINVAL
    bad.write_text("12 0 0 96 512 1 2 0.1\n")  # block not a multiple of 64
    assert lib.dpde_tuning_load(str(bad).encode()) == L.DPDE_EINVAL
    assert lookup(4096, 1, 0) is None
    assert lib.dpde_tuning_load(str(tmp_path / "missing.txt").encode()) == L.DPDE_EIO
    assert lib.dpde_tuning_clear() == L.DPDE_OK


def test_committed_tuning_table_parses():
    from paper_1507_06643_amd import _lib as L
    path = os.path.join(ROOT, "paper_1507_06643_amd", "tuning_gfx950.txt")
    if not os.path.exists(path):
        pytest.skip("no tuning table committed")
    lib = L.load()
    assert lib.dpde_tuning_load(path.encode()) == L.DPDE_OK, lib.dpde_last_error()
    assert lib.dpde_tuning_clear() == L.DPDE_OK


def test_shape_layout_matches_c(tmp_path):
    from paper_1507_06643_amd import _lib as L
    fields = [f for f, _ in L.Shape._fields_]
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){",
             'printf("%zu\\n", sizeof(dpde_shape));']
    lines += [f'printf("{f} %zu\\n", offsetof(dpde_shape, {f}));' for f in fields]
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    assert int(out[0]) == C.sizeof(L.Shape)
    for line in out[1:]:
        if line:
            f, off = line.split()
            assert getattr(L.Shape, f).offset == int(off), f
