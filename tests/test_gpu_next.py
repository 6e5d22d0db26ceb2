"""GPU path vs oracle for the next rows: the projection on the internal
energies (Sec. 4.2), friction and noise along e_ij (the original DPDE model,
Sec. 2.1), the splined LJ potential (eq. Ep) and the configurational
temperature (eq. Tcon)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
LJ = dict(potential=1, rc=2.5, eps_lj=1.0, r_lj=1.0)


@pytest.fixture(scope="module")
def dp():
    import torch
    assert torch.cuda.is_available()
    import paper_1507_06643_amd as m
    return m


def _gpu_state(s):
    q, p, e, st = s.get_state()
    return q.cpu().numpy(), p.cpu().numpy(), e.cpu().numpy(), st


def _errs(box, qg, pg, eg, S):
    dq = qg - S.q
    for k in range(3):
        dq[:, k] -= box[k] * np.rint(dq[:, k] / box[k])
    return (np.abs(dq).max() / max(box), np.abs(pg - S.p).max(),
            np.abs(eg - S.eps).max() / np.abs(S.eps).mean())


def _step_vs_oracle(dp, q, p, e, box, cfg_kw, okw, prime=3, project=False):
    n = len(q)
    s = dp.System(dp.Config(n=n, box=list(box), project=project, **cfg_kw), q, p, e)
    E0 = s.energies()[3]
    s.step(prime)
    qs, ps, es, st = _gpu_state(s)
    P = O.make_params(n, box, step=st, project=int(project), **okw)
    S = O.State(P, qs, ps, es)
    P.E0 = E0  # the GPU's target: the energy of its initial state
    rc, _ = S.step(1)
    assert rc == 0
    s.step(1)
    qg, pg, eg, _ = _gpu_state(s)
    errs = _errs(box, qg, pg, eg, S)
    en, eo = s.energies(), S.energies()
    hist = s.history()
    s.close()
    return errs, en, eo, E0, hist


# ---------------------------------------------------------------------------
# Projection on the internal energies
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", [0, 1])
def test_projection_step_parity(dp, scheme):
    n = 3000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=41)
    errs, en, eo, E0, hist = _step_vs_oracle(dp, q, p, e, [L] * 3,
                                             dict(dt=0.02, scheme=scheme),
                                             dict(dt=0.02, scheme=scheme), project=True)
    assert max(errs) < TOL, errs
    assert abs(en[3] - eo[3]) <= TOL * abs(eo[3])
    assert np.abs(hist[:, 3] - E0).max() < 1e-12 * abs(E0)


def test_sem_drifts_ser_conserves_projection_restores(dp):
    n = 4000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=42)
    drift = {}
    for name, scheme, proj in (("sem", 1, False), ("ser", 0, False), ("sem_proj", 1, True)):
        s = dp.System(dp.Config(n=n, box=[L] * 3, dt=0.02, scheme=scheme, project=proj), q, p, e)
        E0 = s.energies()[3]
        s.step(1000)
        h = s.history()
        drift[name] = np.abs(h[:, 3] - E0).max() / abs(E0)
        s.close()
    assert drift["sem_proj"] < 1e-12
    assert drift["sem"] > 10 * drift["ser"], drift


# ---------------------------------------------------------------------------
# Friction and noise along e_ij
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", [0, 1])
def test_projected_model_step_parity(dp, scheme):
    n = 4000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=43)
    kw = dict(dt=0.01, scheme=scheme, model=1)
    errs, en, eo, _, _ = _step_vs_oracle(dp, q, p, e, [L] * 3, kw, kw)
    assert max(errs) < TOL, errs
    assert abs(en[3] - eo[3]) <= TOL * abs(eo[3])
    assert np.abs(en[4:7] - eo[4:7]).max() < 1e-10


def test_projected_model_fp32(dp):
    n = 4000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=44)
    errs, en, eo, _, _ = _step_vs_oracle(dp, q, p, e, [L] * 3,
                                         dict(dt=0.005, model=1, precision=dp.FP32),
                                         dict(dt=0.005, model=1))
    assert errs[0] < 1e-9 and errs[1] < 2e-5 and errs[2] < 2e-7, errs


# ---------------------------------------------------------------------------
# Splined LJ and the configurational temperature
# ---------------------------------------------------------------------------
def _lj_state(n_side=16, seed=45):
    q, p, e, box = W.lattice_state(n_side, 0.8095, eps0=50.0, seed=seed)
    return q, p, e, box


def test_lj_forces_energy_and_config_terms(dp):
    q, p, e, box = _lj_state()
    n = len(q)
    s = dp.System(dp.Config(n=n, box=box, cv=50.0, neighbor_cap=128, **LJ), q, p, e)
    F, U = s.forces()
    P = O.make_params(n, box, cv=50.0, **LJ)
    Fo, Uo = O.forces(P, q)
    assert np.abs(F.cpu().numpy() - Fo).max() <= TOL * np.abs(Fo).max()
    assert abs(U - Uo) <= TOL * abs(Uo)
    g2, lap = O.config_temperature_terms(P, q)
    en = s.energies()
    assert abs(en[10] - g2) <= 1e-11 * g2
    assert abs(en[11] - lap) <= 1e-11 * abs(lap)
    s.close()


def test_lj_step_parity(dp):
    q, p, e, box = _lj_state(seed=46)
    kw = dict(dt=0.002, cv=50.0, gamma=8.0, **LJ)
    errs, en, eo, _, _ = _step_vs_oracle(dp, q, p, e, box, dict(neighbor_cap=128, **kw), kw)
    assert max(errs) < TOL, errs
    assert abs(en[3] - eo[3]) <= TOL * abs(eo[3])


def test_soft_config_terms(dp):
    n = 3000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=47)
    s = dp.System(dp.Config(n=n, box=[L] * 3), q, p, e)
    g2, lap = O.config_temperature_terms(O.make_params(n, [L] * 3), q)
    en = s.energies()
    assert abs(en[10] - g2) <= 1e-11 * g2
    assert abs(en[11] - lap) <= 1e-11 * abs(lap)
    s.close()


# ---------------------------------------------------------------------------
# Hybrid (Sec. 3.2.2): SSA inside spatial domains, SER across them
# ---------------------------------------------------------------------------
# domains of ~3000, ~100 and ~47 particles sweep in the particle arrays (the
# last mixed with LDS lanes); ~24, ~6 and ~3 keep their state in LDS pools of
# the three sizes
@pytest.mark.parametrize("ndom", [(1, 1, 1), (4, 4, 4), (3, 2, 5), (5, 5, 5), (8, 8, 8),
                                  (10, 10, 10)])
def test_hybrid_step_parity(dp, ndom):
    n = 3000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=51)
    kw = dict(dt=0.01, scheme=2, ndom=ndom)
    errs, en, eo, _, _ = _step_vs_oracle(dp, q, p, e, [L] * 3, kw, kw)
    assert max(errs) < TOL, errs
    assert abs(en[3] - eo[3]) <= TOL * abs(eo[3])


def test_hybrid_step_parity_nonlinear_eos(dp):
    """Hybrid with the Einstein EOS: every SSA pair takes gamma_ij from
    temperatures found by Newton on the current internal energies."""
    n = 3000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=54)
    kw = dict(dt=0.01, scheme=2, ndom=(6, 6, 6), eos=1)
    errs, en, eo, _, _ = _step_vs_oracle(dp, q, p, e, [L] * 3, kw, kw)
    assert max(errs) < TOL, errs
    assert abs(en[3] - eo[3]) <= TOL * abs(eo[3])


def test_batched_hybrid_replicas_match_single_systems(dp):
    """Replicas with different domain decompositions in one handle: each
    equals its own single run bit for bit, stepped eagerly and by graph
    replay."""
    sizes, seeds = W.replica_sizes(4, 500, 3000, seed=79)
    ndoms = [(2, 2, 2), (3, 3, 3), (1, 2, 3), (5, 5, 5)]
    cfgs, qs, ps, es = [], [], [], []
    for r, (nr, sd) in enumerate(zip(sizes, seeds)):
        L = W.cubic_side(int(nr))
        q, p, e = W.equilibrium_state(int(nr), [L] * 3, seed=3000 + r)
        cfgs.append(dp.Config(n=int(nr), box=[L] * 3, seed=int(sd), replica=r, scheme=2,
                              ndom=ndoms[r]))
        qs.append(q); ps.append(p); es.append(e)
    Q, Pm, E = np.concatenate(qs), np.concatenate(ps), np.concatenate(es)
    b = dp.System(cfgs, Q, Pm, E)
    b.step(6)
    qb, pb, eb, _ = _gpu_state(b)
    enb = b.energies()
    for r in range(len(cfgs)):
        s = dp.System(cfgs[r], qs[r], ps[r], es[r])
        s.step(6)
        q1, p1, e1, _ = _gpu_state(s)
        lo, hi = b.offsets[r], b.offsets[r + 1]
        assert np.array_equal(qb[lo:hi], q1)
        assert np.array_equal(pb[lo:hi], p1)
        assert np.array_equal(eb[lo:hi], e1)
        assert np.array_equal(enb[r], s.energies())
        s.close()
    g = dp.System(cfgs, Q, Pm, E)
    g.step_graph(2, 3)
    assert np.array_equal(g.energies(), enb)
    g.close()
    b.close()


def test_hybrid_with_fine_domains_equals_ser(dp):
    n = 3000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=52)
    fine = [int(np.ceil(L / 0.05))] * 3
    a = dp.System(dp.Config(n=n, box=[L] * 3, scheme=2, ndom=fine), q, p, e)
    b = dp.System(dp.Config(n=n, box=[L] * 3, scheme=0), q, p, e)
    # the SER sweeps in the form Hybrid runs (FP64 sums in identifier order)
    b.set_shape(pairs=dp.PAIRS_BOTH_SIDES)
    a.step(3)
    b.step(3)
    qa, pa, ea, _ = _gpu_state(a)
    qb, pb, eb, _ = _gpu_state(b)
    # domains of side 0.05 hold two particles with probability ~1e-7 each
    assert np.array_equal(pa, pb) and np.array_equal(ea, eb)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_hybrid_conserves_energy(dp, precision):
    """SSA steps (FP64) and SER across domains (FP64 or FP32 pair terms, FP64
    reinjection) conserve energy to round-off without conservative forces."""
    n = 4000
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=53)
    s = dp.System(dp.Config(n=n, box=[L] * 3, a=0.0, scheme=2, ndom=(3, 3, 3),
                            precision=precision), q, p, e)
    E0 = s.energies()[3]
    s.step(200)
    h = s.history()
    s.close()
    assert np.abs(h[:, 3] - E0).max() < 1e-12 * abs(E0)
    assert np.abs(h[:, 4:7]).max() < 1e-10


# ---------------------------------------------------------------------------
# Batched replicas with the next rows' options: every replica equals its own
# single run bit for bit (per-replica E0 for the projection, per-replica
# geometry for the LJ lattices).
# ---------------------------------------------------------------------------
def _batch_equals_singles(dp, cfgs, qs, ps, es, steps):
    Q, P, E = np.concatenate(qs), np.concatenate(ps), np.concatenate(es)
    # the same batch replayed from a captured graph (steps / 2 replays of 2)
    g = dp.System(cfgs, Q, P, E)
    g.step_graph(2, steps // 2)
    eng = g.energies()
    g.close()
    b = dp.System(cfgs, Q, P, E)
    b.step(steps)
    assert np.array_equal(eng, b.energies())
    qb, pb, eb, _ = _gpu_state(b)
    enb = b.energies()
    for r in range(len(cfgs)):
        s = dp.System(cfgs[r], qs[r], ps[r], es[r])
        s.step(steps)
        q1, p1, e1, _ = _gpu_state(s)
        lo, hi = b.offsets[r], b.offsets[r + 1]
        assert np.array_equal(qb[lo:hi], q1), r
        assert np.array_equal(pb[lo:hi], p1), r
        assert np.array_equal(eb[lo:hi], e1), r
        assert np.array_equal(enb[r], s.energies()), r
        s.close()
    b.close()


@pytest.mark.parametrize("kw", [dict(project=True), dict(project=True, scheme=1),
                                dict(model=1), dict(model=1, precision=1)])
def test_batched_next_rows_match_single_systems(dp, kw):
    sizes, seeds = W.replica_sizes(4, 500, 3000, seed=81)
    cfgs, qs, ps, es = [], [], [], []
    for r, (nr, sd) in enumerate(zip(sizes, seeds)):
        L = W.cubic_side(int(nr))
        q, p, e = W.equilibrium_state(int(nr), [L] * 3, seed=5000 + r)
        cfgs.append(dp.Config(n=int(nr), box=[L] * 3, seed=int(sd), replica=r, dt=0.01, **kw))
        qs.append(q); ps.append(p); es.append(e)
    _batch_equals_singles(dp, cfgs, qs, ps, es, 6)


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_lj_replicas_match_single_systems(dp, precision):
    cfgs, qs, ps, es = [], [], [], []
    for r, side in enumerate((8, 9, 10)):
        q, p, e, box = W.lattice_state(side, 0.8095, eps0=50.0, seed=6000 + r)
        cfgs.append(dp.Config(n=side ** 3, box=list(box), seed=11 + r, replica=r, dt=0.002,
                              cv=50.0, gamma=8.0, neighbor_cap=128, precision=precision,
                              **LJ))
        qs.append(q); ps.append(p); es.append(e)
    _batch_equals_singles(dp, cfgs, qs, ps, es, 6)


@pytest.mark.parametrize("case", ["sem_projected", "hybrid", "lj"])
def test_cell_block_order_leaves_other_schemes_unchanged(dp, case):
    """SEM with the projection, Hybrid (SSA inside domains) and the splined
    LJ potential run the both-sides form; their trajectories too are the same
    bit for bit in row-major and blocked cell order (B = 2 and 3)."""
    n = 3000
    kw = dict(dt=0.01)
    dens = 3.0
    if case == "sem_projected":
        kw.update(scheme=1, project=True)
    elif case == "hybrid":
        kw.update(scheme=2, ndom=(4, 3, 5))
    else:
        kw.update(potential=dp.POT_LJ, rc=2.5, dt=0.002, cv=50.0, neighbor_cap=128)
        dens = 0.8095
    if case == "lj":
        q, p, e, box = W.lattice_state(14, dens, eps0=50.0, seed=61)
        n = len(q)
    else:
        L = W.cubic_side(n, dens)
        box = [L] * 3
        q, p, e = W.equilibrium_state(n, box, seed=62)
    ref = None
    for ob in (1, 2, 3):
        s = dp.System(dp.Config(n=n, box=list(box), **kw), q, p, e)
        s.set_shape(order_block=ob)
        s.step(6)
        out = _gpu_state(s), s.history()
        s.close()
        if ref is None:
            ref = out
            continue
        for a, b in zip(ref[0][:3], out[0][:3]):
            assert np.array_equal(a, b), (case, ob)
        assert np.array_equal(ref[1], out[1]), (case, ob)
