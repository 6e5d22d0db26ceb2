"""Pins of the oracle's next-row features against what the paper and the
mathematics fix, independent of the oracle's own formulas:

- projection on the internal energies (Sec. 4.2): the projected step has total
  energy E0, leaves q and p untouched and shifts every eps_i by the same
  amount; without it SEM drifts;
- friction and noise projected on e_ij (the original DPDE model, Sec. 2.1):
  the pair increment is parallel to e_ij, momentum and (SER) energy are
  conserved, and SEM with the one-dimensional Ito term keeps T_int near T_kin;
- splined LJ (eq. Ep): v(rc) = v'(rc) = 0 seen through finite differences of
  U, F = -grad U and the Laplacian of U by central differences, and the
  textbook minimum of the unshifted LJ potential;
- the configurational temperature terms (eq. Tcon) against finite differences.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _state(n, seed, box=None, **kw):
    L = W.cubic_side(n)
    box = box or [L] * 3
    q, p, e = W.equilibrium_state(n, box, seed=seed)
    return box, q, p, e


# ---------------------------------------------------------------------------
# Projection (Sec. 4.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", [0, 1])
def test_projection_restores_energy_and_only_shifts_eps(scheme):
    n = 400
    box, q, p, e = _state(n, 3)
    Pp = O.make_params(n, box, dt=0.02, scheme=scheme, project=1)
    Pu = O.make_params(n, box, dt=0.02, scheme=scheme, project=0)
    Sp = O.State(Pp, q, p, e)
    Su = O.State(Pu, q, p, e)
    E0 = Sp.energies()[3]
    assert Pp.E0 == E0
    assert Sp.step(1)[0] == 0 and Su.step(1)[0] == 0
    assert np.array_equal(Sp.q, Su.q) and np.array_equal(Sp.p, Su.p)
    shift = Sp.eps - Su.eps
    Eu = Su.energies()[3]
    assert np.abs(shift - shift.mean()).max() < 1e-12 * np.abs(e).mean()
    assert abs(shift.mean() + (Eu - E0) / n) < 1e-12 * abs(E0) / n
    assert abs(Sp.energies()[3] - E0) < 1e-12 * abs(E0)


def test_sem_drifts_without_projection_and_not_with_it():
    n = 300
    box, q, p, e = _state(n, 4)
    drift = {}
    for proj in (0, 1):
        P = O.make_params(n, box, dt=0.03, scheme=1, project=proj)
        S = O.State(P, q, p, e)
        E0 = S.energies()[3]
        rc, rec = S.step(200, record=True)
        assert rc == 0
        drift[proj] = np.abs(rec[:, 3] - E0).max() / abs(E0)
    assert drift[1] < 1e-12
    assert drift[0] > 1e-6


# ---------------------------------------------------------------------------
# Friction and noise along e_ij (model 1)
# ---------------------------------------------------------------------------
def test_projected_increment_is_parallel_to_the_separation():
    box = [6.0, 6.0, 6.0]
    q = np.array([[1.0, 1.0, 1.0], [1.5, 1.3, 0.8]])
    p = np.array([[0.7, -0.2, 0.4], [-0.3, 0.5, 0.1]])
    e = np.array([100.0, 90.0])
    P = O.make_params(2, box, a=0.0, model=1, dt=0.01)
    p0 = p.copy()
    S = O.State(P, q, p, e)
    rc, _ = S.step(1)
    assert rc == 0
    dp0 = S.p[0] - p0[0]
    # no conservative force and no drift of the pair direction within the
    # step beyond dt*v: compare with the separation after the drift
    dnew = S.q[0] - S.q[1]
    cross = np.cross(dp0, dnew)
    assert np.linalg.norm(cross) < 1e-12 * np.linalg.norm(dp0) * np.linalg.norm(dnew)
    assert np.abs(S.p.sum(axis=0) - p0.sum(axis=0)).max() < 1e-14


@pytest.mark.parametrize("model", [0, 1])
def test_momentum_and_energy_conserved_by_the_ser_step(model):
    n = 500
    box, q, p, e = _state(n, 8)
    P = O.make_params(n, box, a=0.0, model=model, dt=0.01)
    S = O.State(P, q, p, e)
    E0 = S.energies()[3]
    P0 = S.p.sum(axis=0)
    rc, rec = S.step(20, record=True)
    assert rc == 0
    assert np.abs(rec[:, 3] - E0).max() < 1e-12 * abs(E0)
    assert np.abs(S.p.sum(axis=0) - P0).max() < 1e-11


def test_projected_model_sem_keeps_temperatures_together():
    """With the one-dimensional Ito term sigma^2/m of the projected model,
    SEM at small dt keeps T_int and T_kin within a few percent; the vector
    model's 3 sigma^2/m would push T_int away by tens of percent."""
    n = 300
    box, q, p, e = _state(n, 11)
    P = O.make_params(n, box, model=1, scheme=1, dt=0.005, cv=10.0)
    e = np.full(n, 10.0)
    S = O.State(P, q, p, e)
    rc, rec = S.step(1500, record=True)
    assert rc == 0
    tk = rec[500:, 7].mean()
    ti = rec[500:, 8].mean()
    assert abs(tk - ti) / ti < 0.06


# ---------------------------------------------------------------------------
# Splined LJ (eq. Ep) and the configurational temperature (eq. Tcon)
# ---------------------------------------------------------------------------
LJ = dict(potential=1, rc=2.5, eps_lj=1.0, r_lj=1.0)


def _lj_cluster(seed, n=20, box=10.0):
    rng = np.random.default_rng(seed)
    q = []
    while len(q) < n:
        x = rng.random(3) * box
        ok = True
        for y in q:
            d = x - y
            d -= box * np.rint(d / box)
            if np.linalg.norm(d) < 0.95:
                ok = False
                break
        if ok:
            q.append(x)
    return np.array(q), [box] * 3


def _U(P, q):
    return O.forces(P, q)[1]


def test_lj_textbook_minimum():
    P = O.make_params(2, [10.0] * 3, **LJ)
    rmin = 2.0 ** (1.0 / 6.0)
    # the splined potential differs from 4(r^-12 - r^-6) by a + b r; remove
    # it with two far points: the unshifted minimum value is -eps
    v = lambda r: O.pair_potential(P, r)[0]
    r1, r2 = 2.0, 2.4
    # linear part through the two far points of (v - v_LJ) = -(c0 + c1 (r - rc))
    vlj = lambda r: 4.0 * (r ** -12 - r ** -6)
    c1 = ((v(r2) - vlj(r2)) - (v(r1) - vlj(r1))) / (r2 - r1)
    c0 = (v(r1) - vlj(r1)) - c1 * r1
    assert abs(v(rmin) - (c0 + c1 * rmin) - (-1.0)) < 1e-12
    # and the derivative of the unshifted part vanishes there
    h = 1e-5
    dv = (v(rmin + h) - v(rmin - h)) / (2 * h) - c1
    assert abs(dv) < 1e-7  # central difference, h^2 v''' / 6


def test_lj_vanishes_smoothly_at_the_cutoff():
    P = O.make_params(2, [10.0] * 3, **LJ)
    for h in (1e-2, 5e-3, 2.5e-3):
        q = np.array([[1.0, 1.0, 1.0], [1.0 + 2.5 - h, 1.0, 1.0]])
        U = _U(P, q)
        # v(rc) = v'(rc) = 0: U(rc - h) = O(h^2) with the curvature v''(rc)/2
        v2 = 4.0 * (156 * 2.5 ** -14 - 42 * 2.5 ** -8)
        assert abs(U - 0.5 * v2 * h * h) < 2.0 * abs(v2) * h ** 3 + 1e-15


@pytest.mark.parametrize("seed", [1, 2])
def test_lj_force_is_minus_gradient(seed):
    q, box = _lj_cluster(seed)
    P = O.make_params(len(q), box, **LJ)
    F, U = O.forces(P, q)
    h = 1e-6
    for i in range(len(q)):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, c] += h
            qm[i, c] -= h
            g = (_U(P, qp) - _U(P, qm)) / (2 * h)
            assert abs(F[i, c] + g) < 1e-5 * max(1.0, abs(g))


@pytest.mark.parametrize("potential", [0, 1])
def test_config_temperature_terms_against_finite_differences(potential):
    if potential == 1:
        q, box = _lj_cluster(5)
        P = O.make_params(len(q), box, **LJ)
    else:
        rng = np.random.default_rng(6)
        box = [5.0] * 3
        q = rng.random((60, 3)) * 5.0
        P = O.make_params(len(q), box)
    g2, lap = O.config_temperature_terms(P, q)
    h = 1e-4
    U0 = _U(P, q)
    lap_fd = 0.0
    grad = np.zeros_like(q)
    for i in range(len(q)):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, c] += h
            qm[i, c] -= h
            Up, Um = _U(P, qp), _U(P, qm)
            lap_fd += (Up - 2 * U0 + Um) / (h * h)
            grad[i, c] = (Up - Um) / (2 * h)
    assert abs(g2 - (grad ** 2).sum()) < 1e-5 * g2
    assert abs(lap - lap_fd) < 1e-3 * abs(lap)


# ---------------------------------------------------------------------------
# Hybrid (Sec. 3.2.2): SSA inside domains, SER across them
# ---------------------------------------------------------------------------
def test_hybrid_with_single_particle_domains_is_ser():
    """Domains too small to hold two interacting particles leave every pair
    to SER: the Hybrid step equals the SER step bit for bit."""
    n = 300
    box, q, p, e = _state(n, 21)
    fine = [int(np.ceil(b / 0.05)) for b in box]
    Ph = O.make_params(n, box, scheme=2, ndom=fine)
    Ps = O.make_params(n, box, scheme=0)
    # domains of side < 0.05 hold two particles with probability ~1e-7 each
    Sh, Ss = O.State(Ph, q, p, e), O.State(Ps, q, p, e)
    Sh.step(1)
    Ss.step(1)
    qq = Sh.q
    dom = np.stack([np.minimum((qq[:, d] * fine[d] / box[d]).astype(int), fine[d] - 1)
                    for d in range(3)], axis=1)
    pairs = O.pairs(Ph, qq, "cells")
    same = (dom[pairs[:, 0]] == dom[pairs[:, 1]]).all(axis=1)
    if same.any():
        pytest.skip("a pair fell inside one fine domain")
    assert np.array_equal(Sh.p, Ss.p) and np.array_equal(Sh.eps, Ss.eps)


@pytest.mark.parametrize("ndom", [(1, 1, 1), (2, 2, 2), (3, 1, 2)])
def test_hybrid_conserves_energy_and_momentum(ndom):
    n = 400
    box, q, p, e = _state(n, 22)
    P = O.make_params(n, box, a=0.0, scheme=2, ndom=ndom, dt=0.01)
    S = O.State(P, q, p, e)
    E0 = S.energies()[3]
    P0 = S.p.sum(axis=0)
    rc, rec = S.step(20, record=True)
    assert rc == 0
    assert np.abs(rec[:, 3] - E0).max() < 1e-12 * abs(E0)
    assert np.abs(S.p.sum(axis=0) - P0).max() < 1e-11


def test_ssa_pair_update_is_the_exact_ornstein_uhlenbeck_step():
    """Two particles alone: one SSA update at fixed gamma_ij must sample the
    exact solution of d p_ij = -(2 gamma chi/m) p_ij dt + 2 sigma sqrt(chi) dW,
    mean e^{-a} p_ij and variance (sigma^2 m / gamma)(1 - e^{-2a}) per
    component with a = (2 gamma chi/m) dt (Sec. 3.1.2 with the sign of a
    fixed); a sign error or a lost factor 2 fails the moments."""
    box = [6.0, 6.0, 6.0]
    q = np.array([[1.0, 1.0, 1.0], [1.3, 1.1, 1.0]])
    p0 = np.array([[1.5, -0.5, 0.2], [-0.7, 0.4, 0.3]])
    e0 = np.array([100.0, 100.0])
    r = np.linalg.norm(q[0] - q[1])
    gamma, kT, m, dt = 4.5, 1.0, 1.0, 0.05
    chi = (1 - r) ** 2
    gij = gamma * kT / 2 * (1 / 1.0 + 1 / 1.0)  # T_i = eps/cv = 1
    a = 2 * gij / m * chi * dt
    sigma2 = 2 * gamma * kT
    out = []
    for step in range(6000):
        P = O.make_params(2, box, a=0.0, scheme=2, ndom=(1, 1, 1), dt=dt, gamma=gamma, step=step)
        rc, pp, ee, _ = O.fd(P, q, p0, e0)
        assert rc == 0
        out.append((pp[0] - pp[1]))
    out = np.array(out)
    pij0 = p0[0] - p0[1]
    mean_exp = np.exp(-a) * pij0
    var_exp = sigma2 * m / gij * (1 - np.exp(-2 * a))
    se = np.sqrt(var_exp / len(out))
    assert np.abs(out.mean(axis=0) - mean_exp).max() < 5 * se
    assert np.abs(out.var(axis=0) / var_exp - 1).max() < 0.08
