"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these tests re-derives a value by retyping the oracle's own formula:
each checks the oracle against a library routine, a closed form, an invariant
the paper states, a brute-force enumeration, or a statistical law of the
continuous dynamics.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
import workloads as W


# ---------------------------------------------------------------------------
# Counter-based RNG: the Philox round and key schedule of Salmon et al.
# (SC'11), written here generically over the word width.  The 64-bit instance
# is pinned bit-for-bit against numpy's Philox-4x64-10 bit generator; the
# 32-bit instance (published constants) must then equal the oracle's C code.
# ---------------------------------------------------------------------------
def _philox_generic(ctr, key, width, mults, weyl, rounds=10):
    mask = (1 << width) - 1
    x = list(ctr)
    k = list(key)
    for r in range(rounds):
        if r:
            k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
        a = mults[0] * x[0]
        b = mults[1] * x[2]
        x = [(b >> width) ^ x[1] ^ k[0], b & mask, (a >> width) ^ x[3] ^ k[1], a & mask]
    return x


M64, W64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157), (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
M32, W32 = (0xD2511F53, 0xCD9E8D57), (0x9E3779B9, 0xBB67AE85)


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((123456789, 2**63 + 5), (7, 2**64 - 2, 3, 0))])
def test_philox_structure_matches_numpy_4x64(key, ctr):
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = [int(v) for v in g.random_raw(4)]
    # numpy advances the 256-bit counter by one before producing a block
    c = list(ctr)
    c[0] = (c[0] + 1) & (2**64 - 1)
    if c[0] == 0:
        c[1] = (c[1] + 1) & (2**64 - 1)
    assert _philox_generic(c, key, 64, M64, W64) == raw


def test_oracle_philox4x32_equals_published_definition():
    rng = np.random.default_rng(1)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**32, size=4)]
        key = [int(v) for v in rng.integers(0, 2**32, size=2)]
        assert O.philox4x32_10(ctr, key) == _philox_generic(ctr, key, 32, M32, W32)
    # edge counters
    for ctr in ([0, 0, 0, 0], [2**32 - 1] * 4):
        for key in ([0, 0], [2**32 - 1, 2**32 - 1]):
            assert O.philox4x32_10(ctr, key) == _philox_generic(ctr, key, 32, M32, W32)


def test_pair_words_key_and_counter_layout():
    seed = (0xABCDEF01 << 32) | 0x12345678
    step = (3 << 32) | 17
    got = O.pair_words(seed, 5, step, 11, 42)
    want = _philox_generic([11, 42, 17, 3], [0x12345678, 0xABCDEF01 ^ 5], 32, M32, W32)
    assert got == want


def test_gauss3_is_standard_normal():
    n = 60000
    lo, hi = W.random_pairs(10**6, n, seed=3)
    g = np.array([O.gauss3(99, 0, 12345, int(a), int(b)) for a, b in zip(lo, hi)])
    for c in range(3):
        assert stats.kstest(g[:, c], "norm").pvalue > 1e-3
        assert abs(g[:, c].mean()) < 5.0 / math.sqrt(n)
        assert abs(g[:, c].var() - 1.0) < 6.0 * math.sqrt(2.0 / n)
    cor = np.corrcoef(g.T)
    assert np.all(np.abs(cor - np.eye(3)) < 5.0 / math.sqrt(n))


def test_gauss3_depends_on_every_key_and_counter_field():
    base = O.gauss3(7, 0, 10, 1, 2)
    for args in [(8, 0, 10, 1, 2), (7, 1, 10, 1, 2), (7, 0, 11, 1, 2), (7, 0, 10, 3, 2),
                 (7, 0, 10, 1, 4), (7 + (1 << 32), 0, 10, 1, 2), (7, 0, 10 + (1 << 32), 1, 2)]:
        assert not np.array_equal(O.gauss3(*args), base)


# ---------------------------------------------------------------------------
# Pair set: cell list == brute force == an independent numpy enumeration.
# ---------------------------------------------------------------------------
def _numpy_pairs(q, box, periodic, rc):
    d = q[:, None, :] - q[None, :, :]
    for k in range(3):
        if periodic[k]:
            d[..., k] -= box[k] * np.rint(d[..., k] / box[k])
    r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    i, j = np.nonzero(np.triu(r2 < rc * rc, k=1))
    return np.stack([i, j], axis=1).astype(np.int32)


def _adversarial_positions(box, rc, rng, n):
    nc = np.floor(np.asarray(box) / rc).astype(int)
    q = rng.random((n, 3)) * box
    m = n // 4
    # exactly on cell faces
    for k in range(3):
        q[:m, k] = rng.integers(0, nc[k], size=m) * (box[k] / nc[k])
    # at 0 and just below L
    q[m:m + 8, 0] = 0.0
    q[m + 8:m + 16, 1] = np.nextafter(box[1], 0.0)
    # a chain of points exactly rc apart along x (r^2 == rc^2 is excluded)
    base = q[m + 16].copy()
    for t in range(4):
        q[m + 16 + t] = base
        q[m + 16 + t, 0] = (base[0] + t * rc) % box[0]
    return q


@pytest.mark.parametrize("n,periodic,seed", [(100, (1, 1, 1), 0), (250, (1, 1, 1), 1),
                                             (200, (0, 1, 1), 2), (150, (1, 0, 1), 3)])
def test_pairs_cells_equal_brute_force(n, periodic, seed):
    L = W.cubic_side(n)
    box = [L * 1.3, L, L * 0.9] if L * 0.9 >= 3 else [L, L, L]
    rng = np.random.default_rng(seed)
    q = _adversarial_positions(box, 1.0, rng, n)
    P = O.make_params(n, box, periodic=periodic)
    a = O.pairs(P, q, "cells")
    b = O.pairs(P, q, "brute")
    c = _numpy_pairs(q, np.asarray(box), periodic, 1.0)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


def test_box_too_small_rejected():
    P = O.make_params(10, [2.5, 5.0, 5.0])
    assert O.lib().or_check_box(P) == O.OR_EBOX


def test_cell_index_definition():
    L = 7.0
    P = O.make_params(10, [L, L, L])  # nc = 7, side 1
    q = np.array([[0.0, 0.0, 0.0], [np.nextafter(L, 0), 0.5, 6.5], [1.0, 2.0, 3.0], [-1e-300, 0, 0]])
    want = [0, 6 + 7 * (0 + 7 * 6), 1 + 7 * (2 + 7 * 3), 0]
    assert list(O.cell_index(P, q)) == want


def test_wrap_edge_cases():
    L = 6.9336
    assert O.lib().or_wrap(-1e-300, L) == 0.0          # -tiny + L rounds to L -> 0
    assert O.lib().or_wrap(L, L) == 0.0
    assert O.lib().or_wrap(-0.25, L) == L - 0.25
    assert O.lib().or_wrap(L + 0.5, L) == pytest.approx(0.5, abs=1e-15)
    x = 3.0
    assert O.lib().or_wrap(x, L) == x


# ---------------------------------------------------------------------------
# Conservative part: F = -grad U, Newton's third law, VV reversibility.
# ---------------------------------------------------------------------------
def test_forces_are_minus_gradient_of_potential():
    n = 100
    L = W.cubic_side(n)
    q, _, _ = W.equilibrium_state(n, [L] * 3, seed=11)
    P = O.make_params(n, [L] * 3)
    F, _ = O.forces(P, q)
    rng = np.random.default_rng(0)
    h = 1e-6
    for i in rng.choice(n, 10, replace=False):
        for k in range(3):
            qp = q.copy(); qp[i, k] += h
            qm = q.copy(); qm[i, k] -= h
            dU = (O.forces(P, qp)[1] - O.forces(P, qm)[1]) / (2 * h)
            assert F[i, k] == pytest.approx(-dU, abs=1e-6 * max(1.0, abs(F[i, k])))


def test_forces_sum_to_zero():
    n = 400
    L = W.cubic_side(n)
    q, _, _ = W.equilibrium_state(n, [L] * 3, seed=12)
    F, U = O.forces(O.make_params(n, [L] * 3), q)
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).sum()
    assert U > 0


def test_pure_verlet_is_time_reversible_and_keeps_eps():
    """gamma = 0 removes the FD part: the scheme is velocity-Verlet, which is
    time reversible (run n steps, flip p, run n steps -> start)."""
    n = 200
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=13)
    P = O.make_params(n, [L] * 3, gamma=0.0, dt=0.005)
    S = O.State(P, q, p, e)
    S.step(50)
    assert np.array_equal(S.eps, e)
    S.p = -S.p
    S.step(50)
    dq = S.q - q
    dq -= L * np.rint(dq / L)
    assert np.abs(dq).max() < 1e-9
    assert np.abs(S.p + p).max() < 1e-9


def test_pure_verlet_energy_error_is_second_order():
    n = 200
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=14, kT=0.2)
    errs = []
    for dt in (0.004, 0.002):
        P = O.make_params(n, [L] * 3, gamma=0.0, dt=dt)
        S = O.State(P, q, p, e)
        E0 = S.energies()[3]
        _, rec = S.step(int(round(0.2 / dt)), record=True)
        errs.append(np.abs(rec[:, 3] - E0).max())
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.5, ratio


# ---------------------------------------------------------------------------
# Fluctuation/dissipation by SER: exact energy and momentum conservation of
# the sub-step (Sec. 3.2.1), the two-particle reduction to the pairwise
# reinjection rule of eq. SSA_ij, and the noise law of eq. DPDE.
# ---------------------------------------------------------------------------
def _kinetic(p, m=1.0):
    return float((p * p).sum() / (2.0 * m))


@pytest.mark.parametrize("dt,mass", [(0.01, 1.0), (0.05, 2.5)])
def test_ser_fd_conserves_energy_and_momentum(dt, mass):
    n = 600
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=15, mass=mass)
    P = O.make_params(n, [L] * 3, dt=dt, mass=mass)
    rc, p1, e1, dp = O.fd(P, q, p, e)
    assert rc == 0
    dK = _kinetic(p1, mass) - _kinetic(p, mass)
    dE = e1.sum() - e.sum()
    scale = np.abs(dp).sum() * np.abs(p).max() / mass
    assert abs(dK + dE) < 1e-13 * scale + 1e-12 * abs(e.sum()) * 1e-2
    assert abs(dK) > 1e3 * abs(dK + dE)          # a real exchange took place
    assert np.abs(dp.sum(axis=0)).max() < 1e-13 * np.abs(dp).sum()


def test_sem_does_not_conserve_energy():
    n = 600
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=15)
    P = O.make_params(n, [L] * 3, dt=0.02, scheme=1)
    rc, p1, e1, dp = O.fd(P, q, p, e)
    dK = _kinetic(p1) - _kinetic(p)
    dE = e1.sum() - e.sum()
    assert abs(dK + dE) > 1e-6 * abs(dK)


def test_two_particles_reduce_to_pairwise_reinjection():
    """With one interacting pair, SER gives dp_2 = -dp_1 and
    d eps_1 = d eps_2 = -dK/2, the reinjection rule of eq. SSA_ij."""
    box = [3.0, 3.0, 3.0]
    q = np.array([[1.0, 1.0, 1.0], [1.3, 1.2, 0.9]])
    p = np.array([[0.7, -0.2, 0.1], [-0.4, 0.5, 0.3]])
    e = np.array([80.0, 120.0])
    P = O.make_params(2, box, dt=0.01, step=3)
    rc, p1, e1, dp = O.fd(P, q, p, e)
    assert rc == 0
    assert np.array_equal(dp[1], -dp[0])
    assert np.abs(dp).max() > 0
    dK = _kinetic(p1) - _kinetic(p)
    assert e1[0] - e[0] == e1[1] - e[1]
    assert (e1[0] - e[0]) == pytest.approx(-0.5 * dK, rel=1e-12, abs=1e-15)


def test_no_noise_no_friction_beyond_cutoff():
    box = [3.0, 3.0, 3.0]
    q = np.array([[0.2, 1.0, 1.0], [1.25, 1.0, 1.0]])  # r = 1.05 > rc
    p = np.array([[0.7, -0.2, 0.1], [-0.4, 0.5, 0.3]])
    e = np.array([80.0, 120.0])
    rc, p1, e1, dp = O.fd(O.make_params(2, box), q, p, e)
    assert np.array_equal(p1, p) and np.array_equal(e1, e)


def _pair_geometry(q, box, rc=1.0):
    pr = _numpy_pairs(q, np.asarray(box), (1, 1, 1), rc)
    d = q[pr[:, 0]] - q[pr[:, 1]]
    d -= np.asarray(box) * np.rint(d / np.asarray(box))
    r = np.sqrt((d * d).sum(1))
    return pr, r


def test_noise_law_matches_continuous_dynamics():
    """At a frozen configuration, over many noise draws: E[dp_i] is the
    friction drift of eq. DPDE times dt, Cov[dp_i] is sum_j sigma^2 chi dt I,
    and E[d eps_i] is the internal-energy drift of eq. DPDE times dt up to
    O(dt^2) (Appendix B: E[B_ij] = d sigma^2 chi/m, E[C_ij] = 0)."""
    n = 120
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=21, eps0=100.0)
    e = e * np.random.default_rng(2).uniform(0.8, 1.2, size=n)
    dt, gamma, kT, cv = 1e-3, 4.5, 1.0, 100.0
    sigma2 = 2 * gamma * kT
    M = 3000
    dps = np.zeros((M, n, 3))
    des = np.zeros((M, n))
    for s in range(M):
        P = O.make_params(n, [L] * 3, dt=dt, step=s, seed=1234)
        rc, p1, e1, dp = O.fd(P, q, p, e)
        dps[s] = dp
        des[s] = e1 - e
    pr, r = _pair_geometry(q, [L] * 3)
    chi = (1 - r) ** 2
    invT = cv / e
    gij = 0.5 * gamma * kT * (invT[pr[:, 0]] + invT[pr[:, 1]])
    vij = p[pr[:, 0]] - p[pr[:, 1]]
    drift = np.zeros((n, 3))
    np.add.at(drift, pr[:, 0], -(gij * chi)[:, None] * vij * dt)
    np.add.at(drift, pr[:, 1], +(gij * chi)[:, None] * vij * dt)
    var = np.zeros(n)
    np.add.at(var, pr[:, 0], sigma2 * chi * dt)
    np.add.at(var, pr[:, 1], sigma2 * chi * dt)
    edrift = np.zeros(n)
    term = 0.5 * (gij * (vij * vij).sum(1) - 3 * sigma2) * chi * dt
    np.add.at(edrift, pr[:, 0], term)
    np.add.at(edrift, pr[:, 1], term)
    sel = var > 1e-4
    mean = dps.mean(0)
    z = (mean[sel] - drift[sel]) / np.sqrt(var[sel] / M)[:, None]
    assert np.abs(z).max() < 5.5 and abs(z.mean()) < 0.15
    vhat = dps.var(0)[sel]
    assert np.abs(vhat / var[sel][:, None] - 1).max() < 6 * math.sqrt(2 / M)
    ez = (des.mean(0)[sel] - edrift[sel]) / (des.std(0)[sel] / math.sqrt(M))
    assert np.abs(ez).max() < 5.5 and abs(ez.mean()) < 0.2


# ---------------------------------------------------------------------------
# Whole step: invariants and equilibrium statistics.
# ---------------------------------------------------------------------------
def test_no_conservative_force_conserves_energy_to_roundoff():
    """a = 0: VV is free flight (exact kinetic energy), SER conserves the rest."""
    n = 375
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=31)
    P = O.make_params(n, [L] * 3, a=0.0, dt=0.01)
    S = O.State(P, q, p, e)
    E0 = S.energies()[3]
    rc, rec = S.step(400, record=True)
    assert rc == 0
    assert np.abs(rec[:, 3] - E0).max() < 1e-12 * E0
    assert np.abs(rec[:, 4:7]).max() < 1e-11


def test_momentum_conserved_over_run():
    n = 375
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=32)
    S = O.State(O.make_params(n, [L] * 3), q, p, e)
    rc, rec = S.step(200, record=True)
    assert np.abs(rec[:, 4:7]).max() < 1e-11 * np.abs(p).sum()


def test_equilibrium_temperatures_agree_and_eps_is_gamma():
    """T_kin = T_int at equilibrium (Sec. 2.2) and, for constant C_v, the
    internal-energy marginal of the invariant measure e^{-beta eps + s(eps)}
    with s' = C_v/eps is Gamma(C_v+1, T): <eps> = (C_v+1) T."""
    n, cv = 375, 20.0
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=33, eps0=cv)
    S = O.State(O.make_params(n, [L] * 3, cv=cv, dt=0.005), q, p, e)
    S.step(1000)
    tk, ti, em = [], [], []
    for _ in range(60):
        rc, rec = S.step(50, record=True)
        assert rc == 0
        tk.append(rec[:, 7].mean()); ti.append(rec[:, 8].mean()); em.append(S.eps.mean())
    tk, ti, em = map(np.array, (tk, ti, em))
    se = lambda x: x.std(ddof=1) / math.sqrt(len(x))
    # weak order 1: the T_kin/T_int gap is O(dt); 5 standard errors + 1% bias
    assert abs(tk.mean() - ti.mean()) < 5 * math.hypot(se(tk), se(ti)) + 0.01 * ti.mean()
    ratio = em / ti
    assert abs(ratio.mean() - (cv + 1)) < 5 * se(ratio) + 0.02 * (cv + 1)


# ---------------------------------------------------------------------------
# Equation of state: eps(theta) = int_0^theta C_v (eq. DPDE_internalEOS),
# Newton inversion to a few ulp.
# ---------------------------------------------------------------------------
def test_nonlinear_eos_is_integral_of_heat_capacity():
    P = O.make_params(10, [5, 5, 5], eos=1)
    for th in (0.2, 0.7, 1.0, 3.0, 20.0):
        val, err = integrate.quad(lambda t: O.eos_cv(P, t)[0] if t > 0 else P.eos_c0, 0.0, th,
                                  limit=200, epsabs=1e-13, epsrel=1e-13)
        assert O.eos_energy(P, th)[0] == pytest.approx(val, rel=1e-10)


def test_nonlinear_eos_limits():
    P = O.make_params(10, [5, 5, 5], eos=1)
    n, w, c0 = 50.0, 2.0, 10.0
    # x/(e^x - 1) = 1 - x/2 + x^2/12 + O(x^4) with x = w/theta
    th = 1e4
    assert O.eos_energy(P, th)[0] == pytest.approx((n + c0) * th - n * w / 2 + n * w * w / (12 * th),
                                                   rel=1e-13)
    th = 0.02
    assert O.eos_energy(P, th)[0] == pytest.approx(c0 * th, rel=1e-12)


def test_newton_inverts_to_few_ulp():
    P = O.make_params(10, [5, 5, 5], eos=1)
    th = np.exp(np.linspace(np.log(0.05), np.log(200.0), 400))
    eps = O.eos_energy(P, th)
    got, its = O.theta_newton(P, eps)
    assert np.all(its < 60)
    assert np.abs(got / th - 1).max() < 64 * np.finfo(float).eps
    back = O.eos_energy(P, got)
    assert np.abs(back / eps - 1).max() < 16 * np.finfo(float).eps


def test_linear_eos_inversion():
    P = O.make_params(10, [5, 5, 5], eos=0, cv=100.0)
    got, its = O.theta_newton(P, np.array([100.0, 250.0, 1.0]))
    assert list(got) == [1.0, 2.5, 0.01]


# ---------------------------------------------------------------------------
# Surrogate MLP: FP64 backprop against central finite differences.
# ---------------------------------------------------------------------------
def test_mlp_backprop_matches_finite_differences():
    rng = np.random.default_rng(4)
    npar = O.mlp_nparam()
    assert npar == 1153
    w = rng.normal(0, 0.4, npar)
    x = rng.uniform(-1, 1, 64)
    t = rng.uniform(-1, 1, 64)
    loss, g = O.mlp_loss_grad(w, x, t)
    h = 1e-6
    for k in rng.choice(npar, 80, replace=False):
        wp = w.copy(); wp[k] += h
        wm = w.copy(); wm[k] -= h
        fd = (O.mlp_loss_grad(wp, x, t)[0] - O.mlp_loss_grad(wm, x, t)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


# ---------------------------------------------------------------------------
# SEM internal-energy update (Sec. 3.1.1, eq. SEM_fd; App. B).  Euler-Maruyama
# has the exact drift, so at a frozen configuration the mean over noise draws
# of d eps_i is 1/2 sum_j (gamma_ij |v_ij|^2 - d sigma^2/m) chi_ij dt with
# d = 3 noise dimensions; its fluctuating part -1/2 sigma w_ij v_ij.G_ij
# sqrt(dt) has variance 1/4 sum_j sigma^2 chi_ij |v_ij|^2 dt and covariance
# -1/2 sum_j sigma^2 chi_ij v_ij dt with dp_i (whose noise is +sigma w G_ij
# sqrt(dt)): the sign of the noise term.  The same statistics run on copies
# of the oracle with a planted mistake (a dropped 1/2, d = 1, a flipped noise
# sign, a noise term twice too large), built here on the CPU, and must fail.
# ---------------------------------------------------------------------------
_SEM_MUTATIONS = {
    "drift_half_dropped": ("double e = 0.5 * (gij * vsq - 3.0 * sigma",
                           "double e = 1.0 * (gij * vsq - 3.0 * sigma"),
    "one_noise_dimension": ("(gij * vsq - 3.0 * sigma * sigma / P->mass)",
                            "(gij * vsq - 1.0 * sigma * sigma / P->mass)"),
    "noise_sign_flipped": ("- 0.5 * sigma * w * vG * sqdt;", "+ 0.5 * sigma * w * vG * sqdt;"),
    "noise_half_dropped": ("- 0.5 * sigma * w * vG * sqdt;", "- 1.0 * sigma * w * vG * sqdt;"),
}


def _oracle_fd_from(lib):
    import ctypes as C

    import oracle.oracle as OO
    dp = C.POINTER(C.c_double)
    lib.or_fd.argtypes = [C.POINTER(O.OrParams), dp, dp, dp, dp]

    def fd(P, q, p, e):
        q = np.ascontiguousarray(q, dtype=np.float64)
        p1 = np.array(p, dtype=np.float64, copy=True)
        e1 = np.array(e, dtype=np.float64, copy=True)
        d = np.zeros_like(p1)
        rc = lib.or_fd(C.byref(P), OO._d(q), OO._d(p1), OO._d(e1), OO._d(d))
        return rc, p1, e1, d
    return fd


def _mutated_oracle(tmp_path, name):
    import ctypes as C
    import subprocess
    old, new = _SEM_MUTATIONS[name]
    import oracle.build as OB
    src = open(OB.SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"oracle_{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"liboracle_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(so), str(path), "-lm"], check=True)
    return _oracle_fd_from(C.CDLL(str(so)))


def _sem_energy_law(fd, M=2000):
    """Largest |z| of the mean, variance and dp-covariance of d eps_i under
    SEM at a frozen configuration against the values stated above."""
    n = 120
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=23, eps0=100.0)
    e = e * np.random.default_rng(3).uniform(0.8, 1.2, size=n)
    dt, gamma, kT, cv = 2e-3, 4.5, 1.0, 100.0
    sigma2 = 2 * gamma * kT
    des = np.zeros((M, n))
    dps = np.zeros((M, n, 3))
    for s in range(M):
        P = O.make_params(n, [L] * 3, dt=dt, step=s, seed=4321, scheme=1)
        rc, p1, e1, d = fd(P, q, p, e)
        assert rc == 0
        des[s] = e1 - e
        dps[s] = d
    pr, r = _pair_geometry(q, [L] * 3)
    chi = (1 - r) ** 2
    invT = cv / e
    gij = 0.5 * gamma * kT * (invT[pr[:, 0]] + invT[pr[:, 1]])
    vij = p[pr[:, 0]] - p[pr[:, 1]]
    v2 = (vij * vij).sum(1)
    mean = np.zeros(n)
    var = np.zeros(n)
    cov = np.zeros((n, 3))
    term = 0.5 * (gij * v2 - 3 * sigma2) * chi * dt
    for a, sgn in ((0, 1.0), (1, -1.0)):
        np.add.at(mean, pr[:, a], term)
        np.add.at(var, pr[:, a], 0.25 * sigma2 * chi * v2 * dt)
        np.add.at(cov, pr[:, a], -0.5 * sigma2 * dt * (chi[:, None] * sgn * vij))
    sel = var > 1e-8
    zm = (des.mean(0)[sel] - mean[sel]) / np.sqrt(var[sel] / M)
    vhat = des.var(0)[sel]
    zv = (vhat / var[sel] - 1) / math.sqrt(2 / M)
    dev = des - des.mean(0)
    chat = np.einsum("sn,snc->nc", dev, dps - dps.mean(0)) / M
    # covariance estimate error ~ sqrt(var_e var_p / M)
    vp = dps.var(0)
    zc = (chat[sel] - cov[sel]) / np.sqrt(var[sel][:, None] * vp[sel] / M + 1e-300)
    return max(np.abs(zm).max(), np.abs(zv).max(), np.abs(zc).max()), zm, zv, zc


def test_sem_internal_energy_law():
    """The oracle's SEM d eps_i: mean, variance and covariance with dp_i."""
    zmax, zm, zv, zc = _sem_energy_law(O.fd)
    assert zmax < 5.5, zmax
    assert abs(zm.mean()) < 0.2 and abs(zc.mean()) < 0.2


@pytest.mark.parametrize("name", sorted(_SEM_MUTATIONS))
def test_sem_internal_energy_law_catches_planted_mistakes(tmp_path, name):
    zmax, _, _, _ = _sem_energy_law(_mutated_oracle(tmp_path, name))
    assert zmax > 8.0, (name, zmax)
