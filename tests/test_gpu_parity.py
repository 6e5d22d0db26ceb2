"""GPU path vs CPU oracle, through the C ABI.

Integers (RNG words, cell indices, pair lists) must match bit for bit from
identical inputs; FP64 state must match to 1e-12 relative per step with the
scales L (positions, compared modulo L), sqrt(m kT) (momenta) and the mean
internal energy (internal energies).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def dp():
    import torch
    assert torch.cuda.is_available()
    import paper_1507_06643_amd as m
    return m


def _cfg(dp, n, box, **kw):
    return dp.Config(n=n, box=list(box), **kw)


def _oparams(n, box, **kw):
    return O.make_params(n, box, **kw)


def _state_errors(box, periodic, got, want, eps_scale):
    qg, pg, eg = got
    qo, po, eo = want
    dq = qg - qo
    for k in range(3):
        if periodic[k]:
            dq[:, k] -= box[k] * np.rint(dq[:, k] / box[k])
    eq = np.abs(dq).max() / max(box)
    ep = np.abs(pg - po).max()
    ee = np.abs(eg - eo).max() / eps_scale
    return eq, ep, ee


def _gpu_state(sysm):
    q, p, e, step = sysm.get_state()
    return q.cpu().numpy(), p.cpu().numpy(), e.cpu().numpy(), step


# ---------------------------------------------------------------------------
# Counter-based RNG: words bit-exact, normals to rounding.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,replica,step", [(7, 0, 0), (2**64 - 1, 3, 12345),
                                               (0xDEADBEEF12345678, 255, 2**33 + 7)])
def test_rng_words_and_normals(dp, seed, replica, step):
    lo, hi = W.random_pairs(2**31 - 1, 4099, seed=seed % 1000)
    raw, g, g32 = dp.debug_rng(seed, replica, step, lo, hi)
    for k in range(0, len(lo), 97):
        assert list(raw[k]) == O.pair_words(seed, replica, step, int(lo[k]), int(hi[k]))
        go = O.gauss3(seed, replica, step, int(lo[k]), int(hi[k]))
        assert np.abs(g[k] - go).max() <= 1e-14 * max(1.0, np.abs(go).max())
        assert np.abs(g32[k] - go).max() <= 2e-5 * max(1.0, np.abs(go).max())


# ---------------------------------------------------------------------------
# Cells and pairs: bit-exact from identical positions.
# ---------------------------------------------------------------------------
def _adversarial(n, box, seed):
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=float)
    nc = np.floor(box).astype(int)
    q = rng.random((n, 3)) * box
    m = n // 5
    for k in range(3):
        q[:m, k] = rng.integers(0, nc[k], size=m) * (box[k] / nc[k])
    q[m:m + 7, 0] = 0.0
    q[m + 7:m + 14, 1] = np.nextafter(box[1], 0.0)
    q[m + 14:m + 21, 2] = np.nextafter(box[2], 0.0)
    base = q[m + 21].copy()
    for t in range(4):
        q[m + 21 + t] = base
        q[m + 21 + t, 0] = (base[0] + t * 1.0) % box[0]
    return q


CASES = [
    (1000, None, (1, 1, 1), 1),
    (3001, None, (1, 1, 1), 2),        # ragged
    (2400, (20.0, 6.5, 6.2), (0, 1, 1), 3),  # free boundaries along x
    (5000, (12.3, 11.7, 11.9), (1, 1, 1), 4),
    (180, (3.95, 3.95, 3.95), (1, 1, 1), 5),  # 3 cells per side: every stencil wraps
]


@pytest.mark.parametrize("skin", [0.0, 0.3])
@pytest.mark.parametrize("n,box,periodic,seed", CASES)
def test_cells_and_pairs_bit_exact(dp, n, box, periodic, seed, skin):
    if box is None:
        L = W.cubic_side(n)
        box = (L, L, L)
    q = _adversarial(n, box, seed)
    _, p, e = W.equilibrium_state(n, box, seed=seed)
    sysm = dp.System(_cfg(dp, n, box, periodic=periodic, skin=skin), q, p, e)
    P = _oparams(n, box, periodic=periodic)
    # cells have side rc + skin (the reach of the neighbour lists)
    Pc = _oparams(n, box, periodic=periodic, rc=1.0 + skin)
    cells = sysm.debug_cells().cpu().numpy()
    assert np.array_equal(cells, O.cell_index(Pc, q))
    got = sysm.debug_pairs()
    want = O.pairs(P, q, "cells")
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    sysm.close()


def _check_cell_order(sysm, offsets):
    """The memory order of the last list build: a permutation of the
    identifier rows in which every cell's particles fill consecutive slots in
    increasing identifier order.  Cells are taken from the current positions,
    so the positions must be those of the build."""
    rows = sysm.debug_order().cpu().numpy().astype(np.int64)
    cells = sysm.debug_cells().cpu().numpy().astype(np.int64)  # by identifier row
    assert np.array_equal(np.sort(rows), np.arange(len(rows)))
    rep = np.searchsorted(np.asarray(offsets), rows, side="right") - 1
    key = rep * (cells.max() + 1) + cells[rows]
    same = np.diff(key) == 0
    assert np.count_nonzero(~same) + 1 == len(np.unique(key))  # one run per cell
    assert (np.diff(rows)[same] > 0).all()  # increasing identifiers inside it


@pytest.mark.parametrize("case", ["uniform", "clustered", "blocked", "batch"])
def test_memory_order_is_identifier_order_within_cells(dp, case):
    """The reorder ranks each particle in its cell by identifier, from the
    other lanes where the cell lies within one wave's 64 slots and from
    memory otherwise (a cell of 300 particles, cells across wave ends): after
    the set-up build and after a step that rebuilds (skin 0), each cell's
    particles sit in consecutive slots in increasing identifier order.  The
    clustered state is checked after the set-up build only: at a hundred
    times the workload's density one step drives internal energies negative,
    which the step reports as an error."""
    if case == "batch":
        sizes = [700, 100, 533]
        cfgs, qs, ps, es = [], [], [], []
        for r, nr in enumerate(sizes):
            L = W.cubic_side(nr) if nr != 100 else 3.95
            q, p, e = W.equilibrium_state(nr, [L] * 3, seed=900 + r)
            cfgs.append(_cfg(dp, nr, [L] * 3, skin=0.0, seed=3 + r, replica=r))
            qs.append(q); ps.append(p); es.append(e)
        sysm = dp.System(cfgs, np.vstack(qs), np.vstack(ps), np.concatenate(es))
        offsets = sysm.offsets
    else:
        n = 3001
        L = W.cubic_side(n)
        q, p, e = W.equilibrium_state(n, [L] * 3, seed=77)
        cap = 0
        if case == "clustered":  # 300 particles in one cell (side L / 10 > 1.0)
            rng = np.random.default_rng(78)
            q[:300] = 2.2 + 0.5 * rng.random((300, 3))
            cap = 512
        sysm = dp.System(_cfg(dp, n, [L] * 3, skin=0.0, neighbor_cap=cap), q, p, e)
        if case == "blocked":
            sysm.set_shape(order_block=2)
        offsets = [0, n]
    _check_cell_order(sysm, offsets)
    if case != "clustered":
        sysm.step(1)
        _check_cell_order(sysm, offsets)
    sysm.close()


@pytest.mark.parametrize("order_block", [2, 3])
@pytest.mark.parametrize("n,box,periodic,seed", [CASES[2], CASES[4]])
def test_pairs_bit_exact_in_blocked_cell_order(dp, n, box, periodic, seed, order_block):
    """The same pair set in blocked cell order, where a stencil row is several
    runs of memory and some runs are reached across a periodic face."""
    q = _adversarial(n, box, seed)
    _, p, e = W.equilibrium_state(n, box, seed=seed)
    sysm = dp.System(_cfg(dp, n, box, periodic=periodic, skin=0.3), q, p, e)
    sysm.set_shape(order_block=order_block)
    got = sysm.debug_pairs()
    want = O.pairs(_oparams(n, box, periodic=periodic), q, "cells")
    assert np.array_equal(got, want)
    sysm.close()


@pytest.mark.parametrize("skin", [0.0, 0.3])
def test_pairs_far_outside_free_boundary(dp, skin):
    """Particles far outside a free boundary (clamped into the end cells)
    keep every pair.  The list build compares FP32 distances against a radius
    widened by a bound on their rounding, which grows with the largest
    coordinate: at x ~ 900 a pair at r = rc - 1e-6 rounds to r = rc in FP32,
    so without the widening it would be lost (skin 0: the list radius is rc)."""
    box = (24.0, 8.0, 8.0)
    n = 1200
    q, p, e = W.equilibrium_state(n, box, seed=31)
    rng = np.random.default_rng(5)
    q[:40] = np.array([900.0, 4.0, 4.0]) + rng.random((40, 3)) * 1.5
    q[40:80] = np.array([-300.0, 4.0, 4.0]) + rng.random((40, 3)) * 1.5
    q[80] = (900.0, 2.0, 2.0)
    q[81] = (900.0 + 1.0 - 1e-6, 2.0, 2.0)
    q[82] = (-300.0, 6.0, 6.0)
    q[83] = (-300.0 - 1.0 + 1e-6, 6.0, 6.0)
    sysm = dp.System(_cfg(dp, n, box, periodic=(0, 1, 1), skin=skin), q, p, e)
    P = _oparams(n, box, periodic=(0, 1, 1))
    got = sysm.debug_pairs()
    assert np.array_equal(got, O.pairs(P, q, "brute"))
    assert {(80, 81), (82, 83)} <= {tuple(x) for x in got.tolist()}
    S = O.State(P, q, p, e)
    rc, _ = S.step(1)
    assert rc == 0
    sysm.step(1)
    qg, pg, eg, _ = _gpu_state(sysm)
    errs = _state_errors(box, (0, 1, 1), (qg, pg, eg), (S.q, S.p, S.eps), np.abs(S.eps).mean())
    assert max(errs) < TOL, errs
    sysm.close()


def test_pairs_of_evolved_state_match_brute_force(dp):
    n = 600
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=9)
    sysm = dp.System(_cfg(dp, n, [L] * 3), q, p, e)
    sysm.step(25)
    qg, _, _, _ = _gpu_state(sysm)
    P = _oparams(n, [L] * 3)
    assert np.array_equal(sysm.debug_pairs(), O.pairs(P, qg, "brute"))
    Pc = _oparams(n, [L] * 3, rc=1.0 + sysm.cfg.skin)
    assert np.array_equal(sysm.debug_cells().cpu().numpy(), O.cell_index(Pc, qg))


# ---------------------------------------------------------------------------
# Forces and energies at initialisation.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1000, 20000])
def test_forces_and_energies(dp, n):
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=n)
    sysm = dp.System(_cfg(dp, n, [L] * 3), q, p, e)
    F, U = sysm.forces()
    Fo, Uo = O.forces(_oparams(n, [L] * 3), q)
    assert np.abs(F.cpu().numpy() - Fo).max() <= TOL * max(1.0, np.abs(Fo).max())
    assert abs(U - Uo) <= TOL * abs(Uo)
    en = sysm.energies()
    eo = O.energies(_oparams(n, [L] * 3), p, e, Uo)
    assert np.allclose(en[[0, 1, 2, 3, 7, 8, 9]], eo[[0, 1, 2, 3, 7, 8, 9]], rtol=TOL, atol=0)
    assert np.abs(en[4:7] - eo[4:7]).max() < 1e-10
    sysm.close()


# ---------------------------------------------------------------------------
# One step from a GPU state, replayed by the oracle.
# ---------------------------------------------------------------------------
def _step_parity(dp, n, box, periodic=(1, 1, 1), nsteps_before=(0, 7), **kw):
    q, p, e = W.equilibrium_state(n, box, seed=n + 1, eps0=kw.get("cv", 100.0))
    sysm = dp.System(_cfg(dp, n, box, periodic=periodic, **kw), q, p, e)
    worst = 0.0
    done = 0
    for nb in nsteps_before:
        sysm.step(nb - done)
        done = nb
        qs, ps, es, step = _gpu_state(sysm)
        P = _oparams(n, box, periodic=periodic, step=step, **kw)
        S = O.State(P, qs, ps, es)
        rc, _ = S.step(1)
        assert rc == 0
        sysm.step(1)
        done += 1
        qg, pg, eg, step1 = _gpu_state(sysm)
        assert step1 == step + 1
        errs = _state_errors(box, periodic, (qg, pg, eg), (S.q, S.p, S.eps), np.abs(S.eps).mean())
        worst = max(worst, max(errs))
        en = sysm.energies()
        eo = S.energies()
        assert abs(en[3] - eo[3]) <= 1e-12 * abs(eo[3])
        assert abs(en[8] - eo[8]) <= 1e-12 * abs(eo[8])
    sysm.close()
    return worst


def test_step_parity_config0(dp):
    n = 1000
    L = W.cubic_side(n)
    assert _step_parity(dp, n, [L] * 3, dt=0.01) < TOL


def test_step_parity_65536(dp):
    n = 65536
    L = W.cubic_side(n)
    assert _step_parity(dp, n, [L] * 3, dt=0.005, nsteps_before=(0, 3)) < TOL


def test_step_parity_free_x_boundaries(dp):
    box = (24.0, 8.0, 8.0)
    n = int(3 * np.prod(box))
    assert _step_parity(dp, n, box, periodic=(0, 1, 1), dt=0.005) < TOL


def test_step_parity_mass_and_ragged(dp):
    box = (9.3, 8.1, 7.7)
    n = 1733
    assert _step_parity(dp, n, box, dt=0.004, mass=2.5, gamma=3.0, kT_ref=1.3, a=18.0) < TOL


def test_two_particles_and_n_below_two(dp):
    """The smallest systems: one interacting pair, and two particles out of
    range of each other (no pair: momenta and internal energies stay exactly
    as they were, positions drift).  n = 1 is rejected."""
    box = [4.0] * 3
    p = np.array([[0.3, -0.2, 0.1], [-0.3, 0.2, -0.1]])
    e = np.array([100.0, 97.0])
    for q, pair in ((np.array([[1.0, 1.0, 1.0], [1.5, 1.2, 1.1]]), True),
                    (np.array([[0.5, 0.5, 0.5], [2.5, 2.5, 2.5]]), False)):
        sysm = dp.System(_cfg(dp, 2, box, dt=0.01), q, p, e)
        S = O.State(_oparams(2, box, dt=0.01), q, p, e)
        for _ in range(5):
            rc, _ = S.step(1)
            assert rc == 0
            sysm.step(1)
            qg, pg, eg, _ = _gpu_state(sysm)
            errs = _state_errors(box, (1, 1, 1), (qg, pg, eg), (S.q, S.p, S.eps), 100.0)
            assert max(errs) < TOL, (pair, errs)
        if pair:
            assert np.abs(pg - p).max() > 1e-3
        else:
            assert np.array_equal(pg, p) and np.array_equal(eg, e)
        sysm.close()
    with pytest.raises(dp.DpdeError) as ex:
        dp.System(_cfg(dp, 1, box), q[:1], p[:1], e[:1])
    assert ex.value.code == dp._lib.DPDE_EINVAL


# ---------------------------------------------------------------------------
# Conservation and determinism on the GPU.
# ---------------------------------------------------------------------------
def test_energy_conserved_without_conservative_force(dp):
    n = 4000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=5)
    sysm = dp.System(_cfg(dp, n, [L] * 3, a=0.0), q, p, e)
    E0 = sysm.energies()[3]
    sysm.step(500)
    h = sysm.history()
    assert h.shape[0] == 500
    assert np.abs(h[:, 3] - E0).max() < 1e-12 * E0
    assert np.abs(h[:, 4:7]).max() < 1e-10
    sysm.close()


def test_bit_reproducible_and_resumable(dp):
    n = 3000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=6)
    a = dp.System(_cfg(dp, n, [L] * 3), q, p, e)
    a.step(20)
    sa = _gpu_state(a)
    b = dp.System(_cfg(dp, n, [L] * 3), q, p, e)
    b.step(10)
    qb, pb, eb, st = b.get_state()
    c = dp.System(_cfg(dp, n, [L] * 3, step0=st), qb, pb, eb)
    c.step(10)
    sc = _gpu_state(c)
    for x, y in zip(sa[:3], sc[:3]):
        assert np.array_equal(x, y)
    assert sa[3] == sc[3] == 20
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("case", ["periodic", "free_x", "batch", "batch_small_replica"])
def test_step_end_in_sweep_two_equals_separate_passes(dp, case):
    """Within one call of several steps the tile sweep 2 also takes the
    step's observables and the next step's kick and drift; a call of one step
    runs them as separate passes.  Twelve one-step calls and one twelve-step
    call give the same states, records and list builds bit for bit (a
    ragged last tile; with a free x boundary particles leave the box, which
    the kick reports to the list build; a batch's tiles span two replicas; a
    replica smaller than a tile keeps the separate passes)."""
    if case in ("periodic", "free_x"):
        n = 6007
        L = W.cubic_side(n)
        box, per = [L] * 3, [1, 1, 1]
        if case == "free_x":
            box, per = [1.6 * L, L / 1.25, L / 1.3], [0, 1, 1]
        q, p, e = W.equilibrium_state(n, box, seed=313)
        cfg = _cfg(dp, n, box, periodic=per, dt=0.01, seed=5)
    else:
        sizes = [700, 1290, 533, 1800] if case == "batch" else [700, 100, 533]
        cfg, qs, ps, es = [], [], [], []
        for r, nr in enumerate(sizes):
            L = W.cubic_side(nr)
            box, per = [L] * 3, [1, 1, 1]
            if r == 1 and case == "batch":
                box, per = [1.6 * L, L / 1.25, L / 1.3], [0, 1, 1]
            elif r == 1:
                box = [3.95] * 3  # the smallest periodic box of three cells
            q, p, e = W.equilibrium_state(nr, box, seed=700 + r)
            cfg.append(_cfg(dp, nr, box, periodic=per, dt=0.01, seed=31 + r, replica=r))
            qs.append(q); ps.append(p); es.append(e)
        q, p, e = np.vstack(qs), np.vstack(ps), np.concatenate(es)
    a = dp.System(cfg, q, p, e)
    b = dp.System(cfg, q, p, e)
    a.step(12)
    for _ in range(12):
        b.step(1)
    sa, sb = _gpu_state(a), _gpu_state(b)
    for x, y in zip(sa[:3], sb[:3]):
        assert np.array_equal(x, y)
    assert sa[3] == sb[3] == 12
    assert np.array_equal(a.history(), b.history())
    assert np.array_equal(a.energies(), b.energies())
    assert a.list_builds() == b.list_builds() > 1
    if case == "free_x":
        assert (np.abs(sa[0][:, 0] - box[0] / 2) > box[0] / 2).any()  # outside the box
    a.close()
    b.close()


def test_trajectory_independent_of_skin(dp):
    """Neighbour lists built every step (skin 0) and Verlet lists with a skin
    rebuilt on displacement give the same trajectory bit for bit: the lists
    are filtered to r < rc in neighbour-id order every step."""
    n = 5000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=91)
    states, builds, records = [], [], []
    for skin in (0.0, 0.2, 0.5):
        s = dp.System(_cfg(dp, n, [L] * 3, skin=skin, dt=0.01), q, p, e)
        s.step(60)
        states.append(_gpu_state(s))
        builds.append(s.list_builds())
        records.append(s.history())
        s.close()
    for st, rec in zip(states[1:], records[1:]):
        for x, y in zip(states[0][:3], st[:3]):
            assert np.array_equal(x, y)
        # observables are fixed-point sums: independent of the memory order
        assert np.array_equal(records[0], rec)
    assert builds[0] == 61                 # initial build + one per step
    assert 1 < builds[2] < builds[1] < 61  # fewer rebuilds with a larger skin


def test_stored_increments_equal_regenerated_noise(dp):
    """Sweep 2 reading back the stored dp_ij and sweep 2 regenerating G_ij^n
    from (ids, n) as the paper does give the same trajectory bit for bit."""
    from paper_1507_06643_amd import _lib as L
    n = 4000
    L_ = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L_] * 3, seed=81)
    for prec in (dp.FP64, dp.FP32):
        a = dp.System(_cfg(dp, n, [L_] * 3, precision=prec), q, p, e)
        cfg = _cfg(dp, n, [L_] * 3, precision=prec)
        P = cfg.to_c()
        P.flags = L.DPDE_FLAG_REGENERATE_NOISE
        import ctypes as C
        import torch
        h = C.c_void_p()
        qd = torch.as_tensor(q, device="cuda").contiguous()
        pd = torch.as_tensor(p, device="cuda").contiguous()
        ed = torch.as_tensor(e, device="cuda").contiguous()
        torch.cuda.synchronize()
        lib = L.load()
        L.check(lib.dpde_init(C.byref(P), C.c_void_p(qd.data_ptr()), C.c_void_p(pd.data_ptr()),
                              C.c_void_p(ed.data_ptr()), None, C.byref(h)))
        a.step(12)
        L.check(lib.dpde_step(h, 12))
        qo = torch.empty_like(qd); po = torch.empty_like(pd); eo = torch.empty_like(ed)
        st = C.c_int64(0)
        L.check(lib.dpde_get_state(h, C.c_void_p(qo.data_ptr()), C.c_void_p(po.data_ptr()),
                                   C.c_void_p(eo.data_ptr()), C.byref(st)))
        sa = _gpu_state(a)
        assert np.array_equal(sa[0], qo.cpu().numpy())
        assert np.array_equal(sa[1], po.cpu().numpy())
        assert np.array_equal(sa[2], eo.cpu().numpy())
        lib.dpde_free(h)
        a.close()


def _run_form(dp, cfgs, q, p, e, pairs, steps):
    s = dp.System(cfgs, q, p, e)
    s.set_shape(pairs=pairs)
    assert s.get_shape()["pairs"] == pairs
    s.step(steps)
    out = _gpu_state(s), s.history()
    s.close()
    return out


def _forms_agree(box, periodic, a, b, ha, hb, eps_scale):
    eq, ep, ee = _state_errors(box, periodic, a[:3], b[:3], eps_scale)
    assert max(eq, ep, ee) < 1e-12, (eq, ep, ee)
    assert a[3] == b[3]
    # observables: energies to rounding, momentum sums to rounding
    assert np.allclose(ha[:, :4], hb[:, :4], rtol=1e-12, atol=0)
    assert np.abs(ha[:, 4:7] - hb[:, 4:7]).max() < 1e-9


@pytest.mark.parametrize("case", ["fp64", "fp32", "projected", "lj_long_lists", "free_x",
                                  "regenerated"])
def test_pair_forms_agree(dp, case):
    """The SER sweeps with each pair inside a 128-particle tile evaluated once
    (fixed-point per-particle sums) and with every pair term evaluated on both
    particles' lanes (FP64 sums in identifier order) give the same trajectory
    to rounding: the same pair terms (exact negatives), summed in two
    arithmetics.  The LJ case has ~53 neighbours per particle (lists longer
    than the LDS staging of pass A); n is not a multiple of the tile."""
    from paper_1507_06643_amd import _lib as L
    kw, n, dens = {}, 4001, 3.0
    if case == "fp32":
        kw = dict(precision=dp.FP32)
    elif case == "projected":
        kw = dict(model=dp.MODEL_PROJECTED)
    elif case == "lj_long_lists":
        kw = dict(potential=dp.POT_LJ, rc=2.5, eps_lj=1.0, r_lj=1.0, dt=0.002, cv=50.0,
                  neighbor_cap=128)
        dens = 0.8095
    L_ = W.cubic_side(n, dens)
    box, per = [L_] * 3, (1, 1, 1)
    if case == "free_x":
        box, per = [3 * L_, L_ / 1.8, L_ / 1.8], (0, 1, 1)
    q, p, e = W.equilibrium_state(n, box, seed=83, eps0=kw.get("cv", 100.0))
    if case == "lj_long_lists":
        # a jittered lattice (no overlapping LJ cores) with 95 sites left empty
        ql, _, _, box = W.lattice_state(16, dens, seed=84)
        q = ql[:n]
    cfg = _cfg(dp, n, box, periodic=list(per), **kw)
    steps = 4
    if case == "regenerated":
        import ctypes as C
        import torch
        lib = L.load()
        out = []
        for pairs in (dp.PAIRS_BOTH_SIDES, dp.PAIRS_ONCE_PER_TILE):
            P = cfg.to_c()
            P.flags = L.DPDE_FLAG_REGENERATE_NOISE
            h = C.c_void_p()
            qd, pd, ed = (torch.as_tensor(x, device="cuda").contiguous() for x in (q, p, e))
            torch.cuda.synchronize()
            L.check(lib.dpde_init(C.byref(P), C.c_void_p(qd.data_ptr()),
                                  C.c_void_p(pd.data_ptr()), C.c_void_p(ed.data_ptr()), None,
                                  C.byref(h)))
            sh = L.Shape(256, 256, pairs, 1)
            L.check(lib.dpde_set_shape(h, C.byref(sh)))
            L.check(lib.dpde_step(h, steps))
            qo, po, eo = torch.empty_like(qd), torch.empty_like(pd), torch.empty_like(ed)
            st = C.c_int64(0)
            L.check(lib.dpde_get_state(h, C.c_void_p(qo.data_ptr()), C.c_void_p(po.data_ptr()),
                                       C.c_void_p(eo.data_ptr()), C.byref(st)))
            out.append((qo.cpu().numpy(), po.cpu().numpy(), eo.cpu().numpy(), st.value))
            lib.dpde_free(h)
        eq, ep, ee = _state_errors(box, per, out[0][:3], out[1][:3], e.mean())
        assert max(eq, ep, ee) < 1e-12, (eq, ep, ee)
        return
    (sa, ha) = _run_form(dp, cfg, q, p, e, dp.PAIRS_BOTH_SIDES, steps)
    (sb, hb) = _run_form(dp, cfg, q, p, e, dp.PAIRS_ONCE_PER_TILE, steps)
    _forms_agree(box, per, sa, sb, ha, hb, e.mean())


def test_pair_forms_agree_batched(dp):
    """The same for uneven batched replicas (tiles straddle replica borders)."""
    sizes = [517, 1203, 200, 2900]
    cfgs, qs, ps, es = [], [], [], []
    for r, nr in enumerate(sizes):
        L = W.cubic_side(nr)
        q, p, e = W.equilibrium_state(nr, [L] * 3, seed=700 + r)
        cfgs.append(_cfg(dp, nr, [L] * 3, seed=11 + r, replica=r))
        qs.append(q); ps.append(p); es.append(e)
    q, p, e = np.vstack(qs), np.vstack(ps), np.concatenate(es)
    (sa, ha) = _run_form(dp, cfgs, q, p, e, dp.PAIRS_BOTH_SIDES, 4)
    (sb, hb) = _run_form(dp, cfgs, q, p, e, dp.PAIRS_ONCE_PER_TILE, 4)
    ep = np.abs(sa[1] - sb[1]).max()
    ee = np.abs(sa[2] - sb[2]).max() / np.abs(sa[2]).mean()
    assert max(ep, ee) < 1e-12, (ep, ee)
    assert np.allclose(ha[:, :, :4], hb[:, :, :4], rtol=1e-12, atol=0)


@pytest.mark.parametrize("pairs", [0, 1])
def test_cell_block_order_leaves_trajectory_unchanged(dp, pairs):
    """The memory order of the cells (row-major, or blocks of 2^3, 3^3, 5^3
    cells, the blocks at the high faces cut short) changes which particles
    share a tile and a cache line, not the result: the pair set is the
    stencil's and every per-particle sum is order independent, so the states
    after 6 steps are equal bit for bit.  Uneven batched replicas, one with a
    free x boundary and cell counts that no block edge divides."""
    sizes = [1517, 3203, 900]
    cfgs, qs, ps, es = [], [], [], []
    for r, nr in enumerate(sizes):
        L = W.cubic_side(nr)
        box, per = [L] * 3, [1, 1, 1]
        if r == 1:
            box, per = [2.2 * L, L / 1.45, L / 1.5], [0, 1, 1]
        q, p, e = W.equilibrium_state(nr, box, seed=900 + r)
        cfgs.append(_cfg(dp, nr, box, periodic=per, seed=21 + r, replica=r))
        qs.append(q); ps.append(p); es.append(e)
    q, p, e = np.vstack(qs), np.vstack(ps), np.concatenate(es)
    ref = None
    for ob in (1, 2, 3, 5):
        s = dp.System(cfgs, q, p, e)
        s.set_shape(pairs=pairs, order_block=ob)
        assert s.get_shape()["order_block"] == ob
        s.step(3)
        s.set_shape(order_block=1 + ob % 3)  # a change of order mid-run
        s.step(3)
        out = _gpu_state(s), s.history()
        s.close()
        if ref is None:
            ref = out
            continue
        for a, b in zip(ref[0][:3], out[0][:3]):
            assert np.array_equal(a, b), ob
        assert np.array_equal(ref[1], out[1]), ob


def test_invalid_order_block_rejected(dp):
    n = 1000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=86)
    s = dp.System(_cfg(dp, n, [L] * 3), q, p, e)
    for ob in (0, 9, -1):
        with pytest.raises(RuntimeError):
            s.set_shape(order_block=ob)
    assert s.get_shape()["order_block"] == 1
    s.close()


def test_pair_term_range_is_reported(dp):
    """A pair increment beyond the range of the fixed-point sums fails the
    step with DPDE_ERANGE rather than wrapping: one particle at 2e4 lands
    among its new neighbours with a friction increment gamma_ij chi v dt of
    up to 4.5 * 2e4 * 0.01 = 900."""
    n = 2000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=85)
    p[0] = [2e4, 0.0, 0.0]
    s = dp.System(_cfg(dp, n, [L] * 3, a=0.0, skin=0.0), q, p, e)
    assert s.get_shape()["pairs"] == dp.PAIRS_ONCE_PER_TILE
    rc = s.step_raw(1)
    assert rc == dp._lib.DPDE_ERANGE
    s.close()


def test_dense_region_uses_the_list_fallback(dp):
    """A blob at ~11x the density gives some particles several hundred
    neighbours (lists of capacity 512, beyond the register sort widths, which
    take the in-place insertion sort, and beyond the wave-tile sweep, which
    falls back to lane pairs); pairs and one step still match the oracle."""
    rng = np.random.default_rng(17)
    L = 20.0
    base = 3 * int(L ** 3)
    q = np.vstack([rng.random((base, 3)) * L, 8.0 + rng.random((2000, 3)) * 4.0])
    n = len(q)
    _, p, e = W.equilibrium_state(n, [L] * 3, seed=18)
    cfg = dict(dt=0.002, neighbor_cap=512)
    sysm = dp.System(_cfg(dp, n, [L] * 3, **cfg), q, p, e)
    P = _oparams(n, [L] * 3, dt=0.002)
    assert np.array_equal(sysm.debug_pairs(), O.pairs(P, q, "cells"))
    sysm.step(2)
    qs, ps, es, st = _gpu_state(sysm)
    S = O.State(_oparams(n, [L] * 3, dt=0.002, step=st), qs, ps, es)
    rc, _ = S.step(1)
    assert rc == 0
    sysm.step(1)
    qg, pg, eg, _ = _gpu_state(sysm)
    errs = _state_errors([L] * 3, (1, 1, 1), (qg, pg, eg), (S.q, S.p, S.eps), np.abs(S.eps).mean())
    assert max(errs) < TOL, errs
    sysm.close()
