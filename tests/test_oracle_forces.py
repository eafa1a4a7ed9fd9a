"""Pins of the oracle's synthetic chain force field and of the ratchet bias.

Expected values: textbook closed forms (harmonic bond, LJ minimum at
2^(1/6) sigma, screened Coulomb), Newton's third law (zero net force and
torque), finite differences of the energy, and the ratchet-and-pawl
properties stated with eq (FrMD): no bias while z decreases, z_m the running
minimum starting at z(X(0)), bias force = -grad of 1/2 k_R (z - z_m)^2.
"""
import numpy as np
import pytest

import oracle as O
from paper_1705_02180_amd import inputs as I


def params(**kw):
    p = dict(I._base_params())
    p.update(kw)
    return p


def test_bond_closed_form():
    p = params(lj_eps=0.0, dh_prefactor=0.0, k_bond=100.0, r_bond=3.8)
    x = np.array([[0.0, 4.3], [0.0, 0.0], [0.0, 0.0]])
    F, U = O.phys_forces(x, np.zeros(2), p)
    assert abs(U - 0.5 * 100.0 * 0.5 ** 2) < 1e-12
    assert abs(F[0, 0] - 50.0) < 1e-12 and abs(F[0, 1] + 50.0) < 1e-12


def test_lj_minimum_and_depth():
    p = params(k_bond=0.0, dh_prefactor=0.0, nb_excl=0, lj_eps=1.3, lj_sigma=4.0)
    rmin = 2 ** (1 / 6) * 4.0
    x = np.array([[0.0, rmin], [0.0, 0.0], [0.0, 0.0]])
    F, U = O.phys_forces(x, np.zeros(2), p)
    assert abs(U + 1.3) < 1e-12
    assert np.abs(F).max() < 1e-12
    x[0, 1] = 4.0                                   # U(sigma) = 0, repulsive force 24 eps / sigma
    F, U = O.phys_forces(x, np.zeros(2), p)
    assert abs(U) < 1e-12
    assert abs(F[0, 1] - 24 * 1.3 / 4.0) < 1e-12


def test_debye_hueckel_closed_form():
    p = params(k_bond=0.0, lj_eps=0.0, nb_excl=0, dh_prefactor=17.0, dh_kappa=0.1)
    r = 9.0
    x = np.array([[0.0, 0.0], [0.0, r], [0.0, 0.0]])
    q = np.array([0.5, -0.25], dtype=np.float32)
    F, U = O.phys_forces(x, q, p)
    u = 17.0 * 0.5 * -0.25 * np.exp(-0.1 * r) / r
    assert abs(U - u) < 1e-14
    # force on particle 1 along +y: -dU/dr = u (kappa + 1/r)
    assert abs(F[1, 1] - u * (0.1 + 1 / r)) < 1e-14


def test_exclusions():
    p = params(dh_prefactor=0.0, k_bond=0.0)
    x = np.array([[0.0, 3.9, 7.8, 11.7], [0.0] * 4, [0.0] * 4])
    F, U = O.phys_forces(x, np.zeros(4), p)       # only the 0-3 pair survives nb_excl = 2
    sr6 = (4.0 / 11.7) ** 6
    assert abs(U - 4 * (sr6 * sr6 - sr6)) < 1e-14


def test_newton_third_law_and_energy_gradient():
    w = I.config2(n_replicas=1)
    s = w.systems[0]
    p = w.params
    x = I.random_coil(s.n, 3)[:, :80].copy()
    q = s.charge[:80]
    F, U = O.phys_forces(x, q, p)
    scale = np.abs(F).max()
    assert np.abs(F.sum(axis=1)).max() < 1e-11 * scale * 80
    torque = np.cross(x.T, F.T).sum(axis=0)
    assert np.abs(torque).max() < 1e-10 * scale * np.abs(x).max() * 80
    h = 1e-6
    for i in (0, 13, 40, 79):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            fd = -(O.phys_forces(xp, q, p)[1] - O.phys_forces(xm, q, p)[1]) / (2 * h)
            assert abs(fd - F[c, i]) < 1e-5 * max(1.0, scale)


# ---------------------------------------------------------------------------
# ratchet-and-pawl bias, eq (FrMD)
# ---------------------------------------------------------------------------
def _rmd_system(n=30, seed=4):
    w = I.config1()
    p = dict(w.params)
    native = I.compact_native(n, seed)
    sysO = O.System(n, np.arange(n), np.ones(n), np.zeros(n), p, native_xyz=native)
    return p, sysO, native


def test_first_evaluation_sets_zm_and_applies_no_bias():
    p, s, _ = _rmd_system()
    x = I.random_coil(s.n, 5)
    cv = np.zeros(8); cv[1] = np.inf
    F, Fb, cv2 = O.total_force(p, s, x, cv)
    z = O.z_grad(x, s.cidx, s.native, grad=False)
    assert cv2[0] == z and cv2[1] == z            # z_m(0) = z(X(0))
    assert np.all(Fb == 0.0) and cv2[2] == 0.0


def test_no_bias_while_z_below_minimum():
    p, s, _ = _rmd_system()
    x = I.random_coil(s.n, 5)
    z = O.z_grad(x, s.cidx, s.native, grad=False)
    cv = np.zeros(8); cv[1] = z * 1.5                # the chain has moved below its minimum
    _, Fb, cv2 = O.total_force(p, s, x, cv)
    assert np.all(Fb == 0.0) and cv2[1] == z


def test_bias_is_minus_gradient_of_ratchet_energy():
    p, s, _ = _rmd_system()
    p["k_R"] = 0.37
    x = I.random_coil(s.n, 6)
    z, gz = O.z_grad(x, s.cidx, s.native)
    zm = 0.6 * z
    cv = np.zeros(8); cv[1] = zm
    F, Fb, cv2 = O.total_force(p, s, x, cv)
    assert abs(cv2[2] - 0.5 * 0.37 * (z - zm) ** 2) < 1e-12 * cv2[2]
    # the bias pushes z down
    assert np.sum(Fb * gz) < 0
    h = 1e-5

    def Eb(xx):
        zz = O.z_grad(xx, s.cidx, s.native, grad=False)
        return 0.5 * 0.37 * max(zz - zm, 0.0) ** 2

    for i in (0, 11, 29):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            fd = -(Eb(xp) - Eb(xm)) / (2 * h)
            assert abs(fd - Fb[c, i]) < 1e-6 * np.abs(Fb).max()


def test_running_minimum_is_nonincreasing_along_a_path():
    p, s, _ = _rmd_system(20, 2)
    x = I.straight_start(20, 1)
    cv = np.zeros(8); cv[1] = np.inf
    zms = []
    for k in range(40):
        x, _, cv, _ = O.steps(p, s, 0, x, None, cv, 5, step0=5 * k)
        zms.append(cv[1])
        assert cv[1] <= cv[0]
    assert all(b <= a for a, b in zip(zms, zms[1:]))
    assert zms[-1] < zms[0]


# ---------------------------------------------------------------------------
# nonbonded cutoff (plain truncation, like the contact cutoff after eq (Cij))
# ---------------------------------------------------------------------------
def test_nonbonded_cutoff_two_particles():
    p = params(k_bond=0.0, nb_excl=0, dh_prefactor=17.0, dh_kappa=0.1, r_cut_nb=12.0)
    q = np.array([0.5, -0.25], dtype=np.float32)
    for r, inside in ((11.999, True), (12.001, False), (30.0, False), (5.0, True)):
        x = np.array([[0.0, 0.0], [0.0, r], [0.0, 0.0]])
        F, U = O.phys_forces(x, q, p)
        F0, U0 = O.phys_forces(x, q, dict(p, r_cut_nb=0.0))
        if inside:
            np.testing.assert_array_equal(F, F0)
            assert U == U0 and U != 0.0
        else:
            assert U == 0.0 and np.abs(F).max() == 0.0


def test_nonbonded_cutoff_is_the_sum_of_pairs_inside():
    """Forces of a chain with a cutoff, rebuilt pair by pair from two-particle
    evaluations (the closed forms pinned above) over the pairs with r <= r_c."""
    w = I.config2(n_replicas=1)
    s = w.systems[0]
    p = dict(w.params, r_cut_nb=9.0)
    n = 60
    x = I.compact_native(n, 8) + np.random.default_rng(2).normal(0, 0.3, (3, n))
    q = s.charge[:n]
    F, U = O.phys_forces(x, q, p)
    Fb, Ub = O.phys_forces(x, q, dict(p, lj_eps=0.0, dh_prefactor=0.0))        # bonds alone
    pp = dict(p, k_bond=0.0, nb_excl=0, r_cut_nb=0.0)
    Fs, Us, n_in = Fb.copy(), Ub, 0
    for i in range(n):
        for j in range(i + p["nb_excl"] + 1, n):
            if np.sum((x[:, i] - x[:, j]) ** 2) > 81.0:
                continue
            n_in += 1
            f2, u2 = O.phys_forces(x[:, [i, j]], q[[i, j]], pp)
            Fs[:, i] += f2[:, 0]
            Fs[:, j] += f2[:, 1]
            Us += u2
    assert 0 < n_in < n * (n - 1) // 2 - 2 * n       # the cutoff removes pairs, and keeps some
    np.testing.assert_allclose(F, Fs, rtol=0, atol=1e-12 * np.abs(F).max())
    assert U == pytest.approx(Us, rel=1e-12)


def test_nonbonded_cutoff_newton_and_energy_gradient():
    w = I.config2(n_replicas=1)
    s = w.systems[0]
    p = dict(w.params, r_cut_nb=10.0)
    n = 70
    x = I.compact_native(n, 3) + np.random.default_rng(5).normal(0, 0.4, (3, n))
    q = s.charge[:n]
    d = np.sqrt(((x[:, :, None] - x[:, None, :]) ** 2).sum(axis=0))
    assert np.abs(d - 10.0).min() > 1e-3                  # no pair within the FD step of the cutoff
    F, U = O.phys_forces(x, q, p)
    scale = np.abs(F).max()
    assert np.abs(F.sum(axis=1)).max() < 1e-11 * scale * n
    h = 1e-6
    for i in (0, 21, 69):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            fd = -(O.phys_forces(xp, q, p)[1] - O.phys_forces(xm, q, p)[1]) / (2 * h)
            assert abs(fd - F[c, i]) < 1e-5 * max(1.0, scale)
    # a cutoff beyond every distance changes nothing
    F2, U2 = O.phys_forces(x, q, dict(p, r_cut_nb=1e6))
    F3, U3 = O.phys_forces(x, q, dict(p, r_cut_nb=0.0))
    np.testing.assert_array_equal(F2, F3)
    assert U2 == U3
