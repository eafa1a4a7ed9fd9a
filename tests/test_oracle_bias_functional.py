"""Pins of the oracle's bias functional T[X] (rMD section and eq (T); the
protocol's variational correction ranks paths by it).

The oracle accumulates T += dt sum_i |F_bias,i|^2 / (m_i gamma) at every force
evaluation.  Expected values: T stays exactly 0 when no bias acts; after one
step T equals dt k_R^2 (z - z_m)^2 sum_i |grad_i z|^2 / (m_i gamma) built from
the separately pinned z and grad z; in SCPS mode the same with the ratchet
forces of the separately pinned tube variables; T is additive over split
calls, and it ranks a replica whose bias never fires below one whose does.
"""
import numpy as np
import pytest

import oracle as O
from paper_1705_02180_amd import inputs as I


def _chain(n=30, seed=5, params=None):
    p = dict(I.config1().params) if params is None else dict(params)
    rng = np.random.default_rng(seed)
    native = I.compact_native(n, seed)
    mass = rng.uniform(0.5, 2.0, n)                     # unequal masses: T weights 1/m_i
    s = O.System(n, np.arange(n), mass, np.zeros(n), p, native_xyz=native)
    return p, s, native


def test_no_bias_gives_zero():
    p, s, native = _chain()
    p["k_R"] = 0.0
    x = I.straight_start(s.n, 9)
    cv = np.zeros(8); cv[1] = np.inf
    _, _, cv1, _ = O.steps(p, s, 0, x, None, cv, 200)
    assert cv1[7] == 0.0
    # SCPS ratchets with zero stiffness
    rng = np.random.default_rng(1)
    stack = np.array([O.contact_map(native + rng.normal(0, 1, native.shape), s.cidx) for _ in range(4)])
    p.update(bias_mode=1, lam=5.0, k_s=0.0, k_w=0.0)
    s2 = O.System(s.n, s.cidx, s.mass, s.charge, p, native_map=s.native, stack=stack)
    cv = np.zeros(8); cv[5:7] = np.inf
    _, _, cv2, _ = O.steps(p, s2, 0, x, None, cv, 50)
    assert cv2[7] == 0.0


@pytest.mark.parametrize("integrator", [0, 1])
def test_one_step_equals_ratchet_force_norm(integrator):
    p, s, native = _chain()
    p.update(integrator=integrator, k_R=0.05, kT=0.7)
    rng = np.random.default_rng(2)
    x = native + rng.normal(0, 1.0, size=native.shape)
    z, gz = O.z_grad(x, s.cidx, s.native)
    zm = 0.6 * z
    cv = np.zeros(8); cv[1] = zm
    v = np.zeros_like(x) if integrator == 1 else None
    _, _, cv1, _ = O.steps(p, s, 0, x, v, cv, 1)
    m = s.mass.astype(np.float64)
    want = p["dt"] * (p["k_R"] * (z - zm)) ** 2 * np.sum(np.sum(gz * gz, axis=0) / (m * p["gamma"]))
    assert cv1[7] == pytest.approx(want, rel=1e-12)
    assert cv1[7] > 0


def test_one_scps_step_equals_tube_force_norm():
    p, s, native = _chain(n=24)
    p.update(bias_mode=1, lam=5.0, k_s=3.0, k_w=0.7)
    rng = np.random.default_rng(4)
    frames = np.stack([native + rng.normal(0, 1.5, size=native.shape) for _ in range(6)])
    stack = np.array([O.contact_map(f, s.cidx) for f in frames])
    s2 = O.System(s.n, s.cidx, s.mass, s.charge, p, native_map=s.native, stack=stack)
    x = frames[2] + rng.normal(0, 0.3, size=native.shape)
    sv, wv, gs, gw, _ = O.tube(x, s2.cidx, stack, s2.Z0, p["lam"])
    cv = np.zeros(8); cv[5] = sv - 0.2; cv[6] = wv - 0.05
    _, _, cv1, _ = O.steps(p, s2, 0, x, None, cv, 1)
    Fb = -p["k_s"] * 0.2 * gs - p["k_w"] * 0.05 * gw
    want = p["dt"] * np.sum(np.sum(Fb * Fb, axis=0) / (s.mass.astype(np.float64) * p["gamma"]))
    assert cv1[7] == pytest.approx(want, rel=1e-10)


def test_additive_over_split_calls_and_ranks_paths():
    p, s, native = _chain()
    p.update(k_R=0.05)
    x = I.straight_start(s.n, 7)
    cv = np.zeros(8); cv[1] = np.inf
    xa, _, cva, _ = O.steps(p, s, 3, x, None, cv, 120)
    x1, _, cv1, _ = O.steps(p, s, 3, x, None, cv, 70)
    x2, _, cv2, _ = O.steps(p, s, 3, x1, None, cv1, 50, step0=70)
    np.testing.assert_array_equal(x2, xa)
    assert cv2[7] == pytest.approx(cva[7], rel=1e-13)
    assert cva[7] > 0
    # the same start without the ratchet has T = 0 < T of the biased path
    q = dict(p, k_R=0.0)
    _, _, cvd1, _ = O.steps(q, s, 3, x, None, cv, 120)
    assert cvd1[7] == 0.0 < cva[7]


# ---------------------------------------------------------------------------
# least-biased path selection: smallest T among the successful paths
# ---------------------------------------------------------------------------
def _cv_with_T(T):
    cv = np.zeros((len(T), 8))
    cv[:, 7] = T
    return cv


@pytest.mark.parametrize("seed", range(6))
def test_least_biased_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    R = int(rng.integers(1, 40))
    T = np.round(rng.uniform(0, 3, R), 1)                  # coarse values: many ties
    succ = (rng.uniform(size=R) < 0.6).astype(np.uint8)
    succ[rng.integers(R)] = 1
    # brute force: lexicographic minimum of (T, index) over the candidates
    want = min((T[r], r) for r in range(R) if succ[r])[1]
    assert O.least_biased(_cv_with_T(T), succ) == want
    assert O.least_biased(_cv_with_T(T)) == min((T[r], r) for r in range(R))[1]


def test_least_biased_special_cases():
    T = np.array([2.0, 0.5, 0.5, 1.0])
    assert O.least_biased(_cv_with_T(T)) == 1                       # tie -> lowest index
    assert O.least_biased(_cv_with_T(T), [1, 0, 0, 1]) == 3         # the global minimum is masked out
    assert O.least_biased(_cv_with_T(T), [0, 0, 0, 0]) == -1        # no candidate
    assert O.least_biased(_cv_with_T([np.nan, 1.0]), [1, 1]) == -2  # a candidate with T = NaN
    assert O.least_biased(_cv_with_T([np.nan, 1.0]), [0, 1]) == 1   # a non-candidate's NaN is ignored
    assert O.least_biased(_cv_with_T([np.inf, 1.0])) == -2
    assert O.least_biased(_cv_with_T([7.0])) == 0


def test_least_biased_picks_the_path_the_bias_never_pushed():
    p, s, native = _chain()
    p.update(k_R=0.05)
    x = I.straight_start(s.n, 7)
    cv = np.zeros(8); cv[1] = np.inf
    cvs = [O.steps(dict(p, k_R=k), s, r, x, None, cv, 80)[2] for r, k in enumerate([0.05, 0.0, 0.02])]
    cvs = np.stack(cvs)
    assert cvs[1, 7] == 0.0 and cvs[0, 7] > 0 and cvs[2, 7] > 0
    assert O.least_biased(cvs) == 1
    assert O.least_biased(cvs, [1, 0, 1]) == int(np.argmin(cvs[[0, 2], 7])) * 2
