"""Host logic of bench.py (no GPU): the algorithmic bytes behind the
roofline, the energy-drift fit, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_particle():
    # q, p in / F, p out; q, p, 1/T, id in / dp_i out; the sweep-2 set
    assert bench.pair_kernel_bytes("pass_a_forces") == 96.0
    assert bench.pair_kernel_bytes("pass_b_ser") == 84.0
    assert bench.pair_kernel_bytes("pass_c_ser") == 132.0
    # with the step's end inside sweep 2: F, U, Laplacian in, q out
    assert bench.pair_kernel_bytes("pass_c_ser", tail=True) == 132.0 + 64.0
    assert bench.pair_kernel_bytes("pass_a_forces", tail=True) == 96.0
    assert bench.pair_kernel_bytes("kick") is None
    # list words: 4 B per entry and per count
    assert bench.pair_kernel_list_bytes("pass_b_ser", 8.0, 18.0) == 84.0 + 4.0 + 32.0
    assert bench.pair_kernel_list_bytes("pass_a_forces", 8.0, 18.0) == 96.0 + 4.0 + 72.0 + 36.0


def test_drift_fit_is_the_relative_slope_per_1e4_steps():
    E0, slope = -1234.5, 3e-9  # relative drift per step
    n = np.arange(2001)
    rng = np.random.default_rng(0)
    E = E0 * (1.0 - slope * n) + rng.normal(0.0, 1e-9, n.size)
    got = bench.drift_fit(E)
    assert abs(got - 1e4 * slope) < 1e-7
    hist = np.zeros((n.size, 12))
    hist[:, 3] = E
    assert abs(bench.drift_per_1e4(hist) - got) < 1e-12


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_pair_kernel_symbols_are_in_the_profile_summaries():
    """The names the bench looks up in the committed rocprofv3 summaries are
    the ones rocprofv3 reported, so no counter figure drops out silently."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    stats = open(os.path.join(root, "profiles", "learned_eos_n1m_kernel_stats.md")).read()
    traffic = open(bench.PROFILE_TRAFFIC).read().splitlines()
    named = {l.rsplit(" ", 2)[0] for l in traffic if l.startswith("k_")}
    for sym in bench.PAIR_KERNEL_SYMBOLS.values():
        assert f"| {sym} |" in stats, sym
        assert sym in named, sym
