"""Pins of the oracle's contact function and collective coordinate z.

Every expected value here comes from the paper's definitions evaluated
independently of the oracle (the literal form of eq (Cij), closed-form
special values, invariances of eq (zrMD) under rigid motion, brute force),
never from the oracle itself.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1705_02180_amd import inputs as I

R0 = 7.5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def literal_C(r, r0=R0):
    """eq (Cij) exactly as printed: (1 - (r/r0)^6) / (1 - (r/r0)^10)."""
    u = r / r0
    return (1.0 - u ** 6) / (1.0 - u ** 10)


def literal_dC_dr(r, r0=R0):
    """Quotient rule applied to the printed form of eq (Cij)."""
    u = r / r0
    num, den = 1.0 - u ** 6, 1.0 - u ** 10
    dnum, dden = -6.0 * u ** 5 / r0, -10.0 * u ** 9 / r0
    return (dnum * den - num * dden) / den ** 2


def test_contact_matches_printed_formula_away_from_r0():
    r = np.concatenate([np.linspace(0.01, 7.3, 400), np.linspace(7.7, 60.0, 400)])
    C, _ = O.contact(r ** 2, R0)
    np.testing.assert_allclose(C, literal_C(r), rtol=1e-11, atol=0)


def test_contact_special_values():
    C, dC = O.contact(np.array([0.0, R0 ** 2, (2 * R0) ** 2]), R0)
    assert C[0] == 1.0
    assert abs(C[1] - 0.6) < 1e-15                      # removable 0/0 at r0: limit 3/5
    assert abs(C[2] - 21.0 / 341.0) < 1e-15             # q = 4: (1+4+16)/(1+4+16+64+256)
    # dC/dr at r0 = -6/(5 r0) = -0.16 / A
    assert abs(dC[1] * 2 * R0 - (-6.0 / (5.0 * R0))) < 1e-14


def test_contact_tail_is_r0_over_r_to_fourth():
    r = np.array([1e3, 1e4, 1e5])
    C, _ = O.contact(r ** 2, R0)
    np.testing.assert_allclose(C * (r / R0) ** 4, 1.0, rtol=2e-4)


def test_contact_derivative_matches_printed_formula():
    r = np.concatenate([np.linspace(0.5, 7.2, 200), np.linspace(7.8, 40.0, 200)])
    _, dC_dr2 = O.contact(r ** 2, R0)
    np.testing.assert_allclose(dC_dr2 * 2 * r, literal_dC_dr(r), rtol=1e-9, atol=1e-15)


def test_contact_golden_values():
    with open(os.path.join(GOLDEN, "contact_values.json")) as f:
        g = json.load(f)
    r = np.array([e[0] for e in g["values"]])
    want = np.array([e[1] for e in g["values"]])
    C, _ = O.contact(r ** 2, g["r0"])
    np.testing.assert_allclose(C, want, rtol=0, atol=5e-12)


def test_contact_cutoff_zeroes_beyond_rc():
    C, dC = O.contact(np.array([11.9, 12.1]) ** 2, R0, 12.0)
    assert C[0] > 0.14 and C[1] == 0.0 and dC[1] == 0.0


# ---------------------------------------------------------------------------
# z and its gradient
# ---------------------------------------------------------------------------
def _small_system(n=24, seed=7):
    native = I.compact_native(n, seed)
    x = I.random_coil(n, seed + 1)
    cidx = np.arange(n, dtype=np.int32)
    return native, x, cidx


def rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


def test_z_vanishes_at_reference():
    native, _, cidx = _small_system()
    ref = O.contact_map(native, cidx)
    z, g = O.z_grad(native, cidx, ref)
    assert z == 0.0
    assert np.all(g == 0.0)


def test_z_brute_force_with_printed_formula():
    native, x, _ = _small_system(30, 11)
    cidx = np.array([0, 2, 3, 7, 8, 12, 13, 19, 22, 25, 29], dtype=np.int32)
    ref = O.contact_map(native, cidx)
    for min_sep in (0, 3, 35):
        want = 0.0
        k = 0
        for a in range(len(cidx)):
            for b in range(a + 1, len(cidx)):
                i, j = cidx[a], cidx[b]
                r_x = np.linalg.norm(x[:, i] - x[:, j])
                r_n = np.linalg.norm(native[:, i] - native[:, j])
                if abs(i - j) > min_sep:
                    want += (literal_C(r_x) - literal_C(r_n)) ** 2
                k += 1
        z = O.z_grad(x, cidx, ref, min_sep=min_sep, grad=False)
        assert abs(z - want) <= 1e-12 * max(1.0, want)
    assert O.z_grad(x, cidx, ref, min_sep=35, grad=False) == 0.0


def test_z_rigid_motion_invariance():
    native, x, cidx = _small_system()
    ref = O.contact_map(native, cidx)
    z, g = O.z_grad(x, cidx, ref)
    Q = rotation(3)
    xr = Q @ x + np.array([[13.0], [-7.5], [101.0]])
    z2, g2 = O.z_grad(xr, cidx, ref)
    assert abs(z2 - z) <= 1e-12 * z
    np.testing.assert_allclose(g2, Q @ g, rtol=0, atol=1e-10 * np.abs(g).max())


def test_grad_z_net_force_and_torque_vanish():
    native, x, cidx = _small_system()
    ref = O.contact_map(native, cidx)
    _, g = O.z_grad(x, cidx, ref)
    scale = np.abs(g).max()
    assert np.abs(g.sum(axis=1)).max() < 1e-12 * scale * x.shape[1]
    torque = np.cross(x.T, g.T).sum(axis=0)
    assert np.abs(torque).max() < 1e-11 * scale * np.abs(x).max() * x.shape[1]


def test_grad_z_two_particle_closed_form():
    x = np.array([[0.0, 6.1], [0.0, 2.0], [0.0, -1.5]])
    cidx = np.array([0, 1], dtype=np.int32)
    R = np.array([0.8])
    z, g = O.z_grad(x, cidx, R)
    d = x[:, 0] - x[:, 1]
    r = np.linalg.norm(d)
    assert abs(z - (literal_C(r) - 0.8) ** 2) < 1e-15
    want = 2 * (literal_C(r) - 0.8) * literal_dC_dr(r) * d / r
    np.testing.assert_allclose(g[:, 0], want, rtol=1e-12)
    np.testing.assert_allclose(g[:, 1], -want, rtol=1e-12)


def test_grad_z_central_differences():
    native, x, cidx = _small_system(20, 5)
    ref = O.contact_map(native, cidx)
    _, g = O.z_grad(x, cidx, ref)
    h = 1e-5
    rng = np.random.default_rng(0)
    for i in rng.choice(20, 6, replace=False):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            fd = (O.z_grad(xp, cidx, ref, grad=False) - O.z_grad(xm, cidx, ref, grad=False)) / (2 * h)
            assert abs(fd - g[c, i]) <= 1e-6 * max(1.0, np.abs(g).max())


def test_grad_z_row_restricted_differences_large_chain():
    """Moving particle i only changes row i of the map, so the difference of z
    is a sum over j of two squares; no cancellation between unrelated pairs."""
    n = 300
    native = I.compact_native(n, 9)
    x = I.random_coil(n, 10)
    cidx = np.arange(n, dtype=np.int32)
    ref_full = O.contact_map(native, cidx)
    _, g = O.z_grad(x, cidx, ref_full)
    h = 1e-4
    for i in (0, 17, 150, 299):
        others = np.array([j for j in range(n) if j != i])
        R_row = np.array([ref_full[a * n - a * (a + 1) // 2 + (b - a - 1)]
                          for a, b in ((min(i, j), max(i, j)) for j in others)])
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            rp = np.sum((xp[:, others] - xp[:, [i]]) ** 2, axis=0)
            rm = np.sum((xm[:, others] - xm[:, [i]]) ** 2, axis=0)
            Cp, _ = O.contact(rp)
            Cm, _ = O.contact(rm)
            fd = np.sum((Cp - R_row) ** 2 - (Cm - R_row) ** 2) / (2 * h)
            assert abs(fd - g[c, i]) <= 1e-6 * np.abs(g).max()
