"""Pins of the oracle's counter-based noise and Langevin integrators.

Philox4x32-10 is pinned to the known-answer values published with the
Random123 library of Salmon et al. (SC'11).  The integrators are pinned to
exact stationary statistics of the discrete schemes on a harmonic dimer and
a free particle (BAOAB samples the harmonic configuration exactly; the
Euler-Maruyama variance is (kT/k)/(1 - k dt/(m gamma)) for the relative
coordinate), chosen at step sizes where the usual mistakes (wrong noise
amplitude, wrong friction factor, a missing half step) move the statistic by
many standard errors.
"""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        out = O.philox([int(v, 16) for v in case["ctr"]], [int(v, 16) for v in case["key"]])[0]
        assert [f"{v:08x}" for v in out] == case["out"]


def test_uniform_mapping_is_open_interval_and_exact_in_float32():
    assert O.uniform(0) == 2.0 ** -24
    assert O.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for w in (1, 511, 512, 0x12345678, 0xDEADBEEF):
        u = O.uniform(w)
        assert 0.0 < u < 1.0 and float(np.float32(u)) == u


def test_normals_moments_and_independence():
    m = 400_000
    z = O.normals(42, np.arange(m) % 5000, np.arange(m) // 5000, 7)
    se = 1.0 / np.sqrt(m)
    for c in range(3):
        assert abs(z[:, c].mean()) < 5 * se
        assert abs(z[:, c].var() - 1.0) < 5 * np.sqrt(2.0) * se
        k = np.mean(z[:, c] ** 4)
        assert abs(k - 3.0) < 5 * np.sqrt(96.0) * se
    cc = np.corrcoef(z.T)
    assert np.abs(cc - np.eye(3)).max() < 5 * se
    # tails: P(|z| > 3) = 0.0026998
    frac = np.mean(np.abs(z) > 3.0)
    assert abs(frac - 0.0026998) < 5 * np.sqrt(0.0027 / (3 * m))


def test_noise_depends_on_every_counter_word():
    base = O.normals(1, [3], 4, 5)
    assert not np.array_equal(base, O.normals(1, [4], 4, 5))
    assert not np.array_equal(base, O.normals(1, [3], 5, 5))
    assert not np.array_equal(base, O.normals(1, [3], 4, 6))
    assert not np.array_equal(base, O.normals(1, [3], 4, 5 + (1 << 32)))
    assert not np.array_equal(base, O.normals(2, [3], 4, 5))


# ---------------------------------------------------------------------------
# integrators on exactly solvable systems
# ---------------------------------------------------------------------------
def _dimer_params(integrator, dt, gamma, kT, k):
    return dict(integrator=integrator, bias_mode=0, dt=dt, gamma=gamma, kT=kT, k_bond=k,
                r_bond=0.0, lj_eps=0.0, lj_sigma=4.0, dh_prefactor=0.0, dh_kappa=0.1,
                nb_excl=2, min_seq_sep=0, r0_contact=7.5, r_cut_contact=0.0, k_R=0.0,
                lam=1.0, k_s=0.0, k_w=0.0, seed=99)


def _dimer_system(p, n=2):
    return O.System(n, np.zeros(0, dtype=np.int32), np.ones(n), np.zeros(n), p,
                    native_map=np.zeros(0))


def _sample(p, n_rep, n_eq, n_samp, n=2, v0=True):
    s = _dimer_system(p, n)
    per_rep = []
    vel = []
    for r in range(n_rep):
        x = np.zeros((3, n)); x[0, 1:] = 0.1
        v = np.zeros((3, n)) if v0 else None
        cv = np.zeros(8)
        x, v, cv, _ = O.steps(p, s, r, x, v, cv, n_eq)
        x, v2, cv, fr = O.steps(p, s, r, x, v, cv, n_samp, step0=n_eq, record_every=1)
        per_rep.append(fr[1:])
        vel.append(v2)
    return np.array(per_rep), vel


def test_baoab_samples_harmonic_configuration_exactly():
    # omega dt = 1.2 (sqrt(2 k/m) = 1.2 / dt): far from the small-step limit
    kT, k, dt, gamma = 1.0, 0.72, 1.0, 1.0
    p = _dimer_params(1, dt, gamma, kT, k)
    fr, _ = _sample(p, 160, 60, 400)
    d = fr[:, :, :, 0] - fr[:, :, :, 1]                # [rep][t][3]
    per_rep = (d ** 2).mean(axis=(1, 2))
    mean, se = per_rep.mean(), per_rep.std(ddof=1) / np.sqrt(len(per_rep))
    assert abs(mean - kT / k) < 4 * se
    assert se < 0.02 * kT / k


def test_baoab_free_particle_velocity_after_noise_is_maxwellian():
    p = _dimer_params(1, 0.5, 0.7, 2.0, 0.0)
    s = _dimer_system(p, 1)
    vs = []
    for r in range(3000):
        x = np.zeros((3, 1)); v = np.zeros((3, 1)); cv = np.zeros(8)
        _, v, _, _ = O.steps(p, s, r, x, v, cv, 30)
        vs.append(v[:, 0])
    vs = np.array(vs)
    # exact: the O substep is an exact Ornstein-Uhlenbeck update, so after 30
    # steps from rest <m v^2> = kT (1 - c1^(2*30))
    c1 = np.exp(-0.7 * 0.5)
    want = 2.0 * (1.0 - c1 ** 60)
    m2 = (vs ** 2).mean()
    se = (vs ** 2).std() / np.sqrt(vs.size)
    assert abs(m2 - want) < 4 * se


def test_euler_maruyama_harmonic_variance():
    kT, k, dt, mgamma = 1.0, 2.5, 0.1, 1.0      # k dt/(m gamma) = 0.25 -> factor 4/3
    p = _dimer_params(0, dt, mgamma, kT, k)
    fr, _ = _sample(p, 120, 60, 300, v0=False)
    d = fr[:, :, :, 0] - fr[:, :, :, 1]
    per_rep = (d ** 2).mean(axis=(1, 2))
    mean, se = per_rep.mean(), per_rep.std(ddof=1) / np.sqrt(len(per_rep))
    want = (kT / k) / (1.0 - k * dt / mgamma)
    assert abs(mean - want) < 4 * se
    assert abs(want - kT / k) > 10 * se             # the test can tell the scheme apart


def test_euler_maruyama_free_diffusion():
    kT, dt, mgamma = 0.8, 0.05, 2.0
    p = _dimer_params(0, dt, mgamma, kT, 0.0)
    s = _dimer_system(p, 1)
    x0 = np.zeros((3, 1))
    dx = []
    for r in range(4000):
        x, _, _, _ = O.steps(p, s, r, x0, None, np.zeros(8), 1)
        dx.append(x[:, 0])
    dx = np.array(dx)
    want = 2 * kT * dt / mgamma
    m2 = (dx ** 2).mean()
    se = (dx ** 2).std() / np.sqrt(dx.size)
    assert abs(m2 - want) < 4 * se
