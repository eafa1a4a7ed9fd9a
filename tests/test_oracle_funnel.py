"""Pins of the oracle's toy model: one particle on the two-dimensional
asymmetric funnel of eq (U) (Table 1), overdamped Langevin steps, rMD on
z = |X| and the Euclidean tube variables around a mean path.

Expected values: U and F at the origin in closed form, central differences
of U, the rotational symmetry without the gate term, free diffusion
(<dx^2> = 2 kT D n per coordinate, a statistical check on many
trajectories), the ratchet properties of eq (FrMD), the appendix limit of
the tube variables, central differences of s and w, the SCPS bias force as
minus the gradient of the ratchet energies (by differences of s and w), and
T = 0 without a bias / T = D |F_bias|^2 after one step.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1705_02180_amd import inputs as I


def test_origin_closed_form():
    p = I.funnel_params()
    U, F = O.funnel_force(p, 0.0, 0.0)
    a3 = p["xm"] ** 2 + p["ym"] ** 2 + p["s3"] ** 2
    assert U == pytest.approx(-p["A1"] / p["s1"] ** 2 + p["A2"] / p["s2"] ** 2 - p["A3"] * p["s3"] ** 2 / a3 ** 2,
                              rel=1e-15)
    # only the gate term pulls at the origin, towards the gate at (xm, ym)
    assert F[0] == pytest.approx(4 * p["A3"] * p["s3"] ** 2 * p["xm"] / a3 ** 3, rel=1e-15)
    assert F[1] == 0.0


def test_force_is_minus_gradient():
    p = I.funnel_params()
    rng = np.random.default_rng(1)
    h = 1e-6
    for x, y in rng.uniform(-6, 6, size=(25, 2)):
        _, F = O.funnel_force(p, x, y)
        gx = (O.funnel_force(p, x + h, y)[0] - O.funnel_force(p, x - h, y)[0]) / (2 * h)
        gy = (O.funnel_force(p, x, y + h)[0] - O.funnel_force(p, x, y - h)[0]) / (2 * h)
        assert F[0] == pytest.approx(-gx, abs=1e-6 * max(1.0, abs(gx)))
        assert F[1] == pytest.approx(-gy, abs=1e-6 * max(1.0, abs(gy)))


def test_radial_without_the_gate():
    p = I.funnel_params(A3=0.0)
    rng = np.random.default_rng(2)
    for x, y in rng.uniform(-5, 5, size=(10, 2)):
        _, F = O.funnel_force(p, x, y)
        assert abs(F[0] * y - F[1] * x) <= 1e-12 * max(1.0, np.hypot(*F) * np.hypot(x, y))


def test_free_diffusion_variance():
    p = I.funnel_params(A1=0.0, A2=0.0, A3=0.0, w=0.0, k_R=0.0)
    n_traj, n = 20000, 10
    xy = np.zeros((n_traj, 2))
    cv = np.zeros((n_traj, 8)); cv[:, 1] = np.inf
    xy1, cv1, _ = O.funnel_steps(p, xy, cv, n)
    want = 2 * p["kT"] * p["mob_dt"] * n
    var = xy1.var(axis=0)
    se = want * math.sqrt(2.0 / n_traj)
    assert np.all(np.abs(var - want) <= 5 * se), (var, want)
    assert np.all(np.abs(xy1.mean(axis=0)) <= 5 * math.sqrt(want / n_traj))
    assert np.all(cv1[:, 7] == 0.0)                       # no bias, T = 0


def test_rmd_ratchet_properties():
    p = I.funnel_params()
    xy = np.tile(I.FUNNEL_START, (8, 1))
    cv = np.zeros((8, 8)); cv[:, 1] = np.inf
    zprev = np.full(8, np.inf)
    for k in range(40):
        xy, cv, _ = O.funnel_steps(p, xy, cv, 1, step0=k)
        assert np.all(cv[:, 1] <= zprev) and np.all(cv[:, 1] <= cv[:, 0])   # z_m non-increasing, <= z
        zprev = cv[:, 1].copy()
    # the first evaluation sets z_m = z(X0) and applies no bias: one step equals k_R = 0
    cv0 = np.zeros((1, 8)); cv0[:, 1] = np.inf
    a, ca, _ = O.funnel_steps(p, [I.FUNNEL_START], cv0, 1)
    b, cb, _ = O.funnel_steps(dict(p, k_R=0.0), [I.FUNNEL_START], cv0, 1)
    np.testing.assert_array_equal(a, b)
    assert ca[0, 1] == 5.0 and ca[0, 7] == 0.0


def _mean_path(K=9):
    t = np.linspace(0, 1, K)
    return np.stack([1.5 * np.sin(np.pi * t), 5.0 * (1 - t)], axis=1)


@pytest.mark.parametrize("w_form", [0, 1], ids=["w_with_1_over_lambda", "w_without_1_over_lambda"])
def test_tube_appendix_limit_and_gradients(w_form):
    mp = _mean_path()
    M = len(mp) - 1
    for l in (0, 4, M):
        s, w, _, _ = O.funnel_tube(mp[l, 0], mp[l, 1], mp, 400.0, w_form=w_form)
        assert abs(s - (1 - l / M)) < 1e-12 and abs(w) < 1e-12
    h = 1e-6
    for x, y in [(0.3, 3.1), (1.2, 1.0), (-0.5, 4.4)]:
        s, w, gs, gw = O.funnel_tube(x, y, mp, 0.3, w_form=w_form)
        if w_form:
            s0, w0, gs0, gw0 = O.funnel_tube(x, y, mp, 0.3)
            assert s == s0 and w == pytest.approx(0.3 * w0, rel=1e-13)
            np.testing.assert_allclose(gw, 0.3 * gw0, rtol=1e-12)
        for c, (dx, dy) in enumerate([(h, 0), (0, h)]):
            sp, wp, _, _ = O.funnel_tube(x + dx, y + dy, mp, 0.3, w_form=w_form)
            sm, wm, _, _ = O.funnel_tube(x - dx, y - dy, mp, 0.3, w_form=w_form)
            assert gs[c] == pytest.approx((sp - sm) / (2 * h), rel=1e-6, abs=1e-9)
            assert gw[c] == pytest.approx((wp - wm) / (2 * h), rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("w_form", [0, 1], ids=["w_with_1_over_lambda", "w_without_1_over_lambda"])
def test_scps_force_is_minus_gradient_of_ratchet_energy_and_T(w_form):
    mp = _mean_path()
    p = I.funnel_params(bias_mode=1, kT=0.0, A1=0.0, A2=0.0, A3=0.0, w=0.0, w_form=w_form)   # bias alone, no noise
    x0, y0 = 0.9, 2.2
    s0, w0, _, _ = O.funnel_tube(x0, y0, mp, p["lam"], w_form=w_form)
    sm, wm = s0 - 0.2, w0 - 0.5
    cv = np.zeros((1, 8)); cv[0, 5], cv[0, 6] = sm, wm
    xy1, cv1, _ = O.funnel_steps(p, [[x0, y0]], cv, 1, mean_path=mp)
    Fb = (xy1[0] - [x0, y0]) / p["mob_dt"]

    def E(x, y):
        s, w, _, _ = O.funnel_tube(x, y, mp, p["lam"], w_form=w_form)
        return 0.5 * p["k_s"] * (s - sm) ** 2 + 0.5 * p["k_w"] * (w - wm) ** 2
    h = 1e-6
    g = [(E(x0 + h, y0) - E(x0 - h, y0)) / (2 * h), (E(x0, y0 + h) - E(x0, y0 - h)) / (2 * h)]
    np.testing.assert_allclose(Fb, -np.array(g), rtol=1e-6)
    assert cv1[0, 7] == pytest.approx(p["mob_dt"] * float(Fb @ Fb), rel=1e-9)
    assert cv1[0, 3] == s0 and cv1[0, 5] == sm
