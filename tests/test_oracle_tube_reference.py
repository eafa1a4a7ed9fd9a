"""Pins of the oracle's path-ensemble mean map, eq (avCij), and of the
mean-field tube variables s_lambda, w_lambda with their ratchet forces.

Expected values: the appendix identity (as lambda grows, s -> 1 - l/M and
w -> 0 when X is the l-th frame of the reference path), the uniform-weight
case (identical frames give s = 1/2 exactly and w = d - log(K)/lambda),
finite differences, numpy means of independently computed maps, and the
subset/linearity properties of an arithmetic mean.
"""
import numpy as np
import pytest

import oracle as O
from paper_1705_02180_amd import inputs as I

R0 = 7.5


def _path(n=40, K=9, seed=3):
    """A short oracle trajectory (frames) from an extended start."""
    w = I.config1()
    p = dict(w.params)
    native = I.compact_native(n, seed)
    s = O.System(n, np.arange(n), np.ones(n), np.zeros(n), p, native_xyz=native)
    x = I.straight_start(n, seed + 1)
    cv = np.zeros(8); cv[1] = np.inf
    _, _, _, frames = O.steps(p, s, 0, x, None, cv, 40 * (K - 1), record_every=40)
    return native, frames, s


def test_appendix_limit_large_lambda():
    native, frames, s = _path()
    K = frames.shape[0]
    cidx = s.cidx
    stack = np.array([O.contact_map(f, cidx) for f in frames])
    Z0 = float(np.sum(O.contact_map(native, cidx) ** 2))
    M = K - 1
    for l in (0, 3, M):
        _, _, _, _, dk = O.tube(frames[l], cidx, stack, Z0, 1.0, grads=False)
        assert dk[l] == 0.0
        dmin = np.min(np.delete(dk, l))
        assert dmin > 0
        # every other frame is suppressed by at least exp(-lambda dmin)
        for lam_dmin in (2.0, 8.0, 40.0):
            lam = lam_dmin / dmin
            sv, wv, _, _, _ = O.tube(frames[l], cidx, stack, Z0, lam, grads=False)
            bound = K * np.exp(-lam_dmin)
            assert abs(sv - (1.0 - l / M)) <= bound + 1e-15
            assert 0.0 >= wv >= -bound / lam - 1e-15
        assert abs(sv - (1.0 - l / M)) < 1e-15


@pytest.mark.parametrize("w_form", [0, 1], ids=["w_with_1_over_lambda", "w_without_1_over_lambda"])
def test_identical_frames_give_uniform_weights(w_form):
    """K identical frames: p_k = 1/K, so s = 1/2 and grad s = 0 exactly, and
    log sum_k exp(-lambda d) = log K - lambda d.  With the 1/lambda of eqs
    (wX), (wXapp): w = d - log(K)/lambda and grad w = grad d; without it, as
    eq (awXa) prints w: w = lambda d - log K and grad w = lambda grad d."""
    native, frames, s = _path(30, 5, 8)
    cidx = s.cidx
    one = O.contact_map(frames[2], cidx)
    K = 7
    stack = np.tile(one, (K, 1))
    Z0 = 3.7
    lam = 13.5
    x = frames[4]
    sv, wv, gs, gw, dk = O.tube(x, cidx, stack, Z0, lam, w_form=w_form)
    d = np.sum((O.contact_map(x, cidx) - one) ** 2) / Z0
    assert np.allclose(dk, d, rtol=1e-14)
    assert abs(sv - 0.5) < 1e-14
    # grad s = 0 and grad w = (scale / Z0) grad z against the single frame
    _, gz = O.z_grad(x, cidx, one)
    assert np.abs(gs).max() < 1e-14 * max(1.0, np.abs(gw).max())
    if w_form == 0:
        assert abs(wv - (d - np.log(K) / lam)) < 1e-12
        np.testing.assert_allclose(gw, gz / Z0, rtol=1e-11, atol=1e-15)
    else:
        assert abs(wv - (lam * d - np.log(K))) < 1e-11
        np.testing.assert_allclose(gw, lam * gz / Z0, rtol=1e-11, atol=1e-14)


def _printed_contact(r, r0=R0):
    """eq (Cij) exactly as printed: (1 - (r/r0)^6) / (1 - (r/r0)^10)."""
    u = r / r0
    return (1.0 - u ** 6) / (1.0 - u ** 10)


def test_distance_norm_sums_over_the_same_pairs_at_seqsep_35():
    """The normalised distance of the SCPS section divides the sum over
    |i - j| > 35 of (C - C')^2 by the sum over the same pairs of (C0)^2.
    Brute force over a 70-bead chain with the printed form of eq (Cij):
    Z0 and every d_k of a two-frame stack at min_seq_sep = 35."""
    n, msep = 70, 35
    rng = np.random.default_rng(17)
    native = I.compact_native(n, 17)
    frames = [I.random_coil(n, 18), native + rng.normal(0, 1.0, native.shape)]
    x = native + rng.normal(0, 2.0, native.shape)
    cidx = np.arange(n, dtype=np.int32)
    p = dict(I.config1().params, min_seq_sep=msep)
    stack = np.array([O.contact_map(f, cidx) for f in frames])
    so = O.System(n, cidx, np.ones(n), np.zeros(n), p, native_xyz=native, stack=stack)

    def brute(xa, xb=None, ref=None):
        tot = 0.0
        for i in range(n):
            for j in range(i + 1, n):
                if j - i <= msep:
                    continue
                ca = _printed_contact(np.linalg.norm(xa[:, i] - xa[:, j]))
                cb = 0.0 if xb is None else _printed_contact(np.linalg.norm(xb[:, i] - xb[:, j]))
                tot += (ca - cb) ** 2
        return tot

    z0 = brute(native)
    assert so.Z0 == pytest.approx(z0, rel=1e-12)
    everything = float(np.sum(O.contact_map(native, cidx) ** 2))
    assert so.Z0 < 0.5 * everything            # most of the weight sits within 35 of the diagonal
    assert O.System(n, cidx, np.ones(n), np.zeros(n), dict(p, min_seq_sep=0), native_xyz=native).Z0 == \
        pytest.approx(everything, rel=1e-14)
    _, _, _, _, dk = O.tube(x, cidx, stack, so.Z0, 13.5, min_sep=msep, grads=False)
    for k, f in enumerate(frames):
        assert dk[k] == pytest.approx(brute(x, f) / z0, rel=1e-11)


def test_w_without_one_over_lambda_is_lambda_times_w():
    """Dropping the 1/lambda multiplies w and grad w by lambda and leaves s
    alone; the no-1/lambda form's gradients also match central differences."""
    native, frames, s = _path(24, 6, 5)
    cidx = s.cidx
    stack = np.array([O.contact_map(f, cidx) for f in frames])
    Z0 = float(np.sum(O.contact_map(native, cidx) ** 2))
    lam = 40.0
    x = 0.5 * (frames[2] + frames[3])
    s0, w0, gs0, gw0, d0 = O.tube(x, cidx, stack, Z0, lam)
    s1, w1, gs1, gw1, d1 = O.tube(x, cidx, stack, Z0, lam, w_form=1)
    assert s1 == s0 and np.array_equal(d0, d1) and np.array_equal(gs0, gs1)
    assert w1 == pytest.approx(lam * w0, rel=1e-13)
    np.testing.assert_allclose(gw1, lam * gw0, rtol=1e-12, atol=1e-15)
    h = 1e-5
    for i in (0, 9, 23):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            wp = O.tube(xp, cidx, stack, Z0, lam, grads=False, w_form=1)[1]
            wm = O.tube(xm, cidx, stack, Z0, lam, grads=False, w_form=1)[1]
            assert abs((wp - wm) / (2 * h) - gw1[c, i]) < 1e-6 * max(1e-3, np.abs(gw1).max())


def test_tube_gradients_central_differences():
    native, frames, s = _path(24, 6, 5)
    cidx = s.cidx
    stack = np.array([O.contact_map(f, cidx) for f in frames])
    Z0 = float(np.sum(O.contact_map(native, cidx) ** 2))
    lam = 40.0
    x = 0.5 * (frames[2] + frames[3])
    sv, wv, gs, gw, _ = O.tube(x, cidx, stack, Z0, lam)
    h = 1e-5
    for i in (0, 7, 23):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            sp, wp, *_ = O.tube(xp, cidx, stack, Z0, lam, grads=False)
            sm, wm, *_ = O.tube(xm, cidx, stack, Z0, lam, grads=False)
            assert abs((sp - sm) / (2 * h) - gs[c, i]) < 1e-6 * max(1e-3, np.abs(gs).max())
            assert abs((wp - wm) / (2 * h) - gw[c, i]) < 1e-6 * max(1e-3, np.abs(gw).max())


@pytest.mark.parametrize("w_form", [0, 1], ids=["w_with_1_over_lambda", "w_without_1_over_lambda"])
def test_scps_bias_force_is_minus_gradient_of_ratchet_energies(w_form):
    native, frames, s = _path(24, 6, 5)
    cidx = s.cidx
    stack = np.array([O.contact_map(f, cidx) for f in frames])
    p = dict(I.config1().params)
    p.update(bias_mode=1, lam=25.0, k_s=2.5, k_w=0.8, w_form=w_form)
    so = O.System(s.n, cidx, np.ones(s.n), np.zeros(s.n), p, native_xyz=native, stack=stack)
    x = 0.5 * (frames[2] + frames[4])
    sv, wv, *_ = O.tube(x, cidx, stack, so.Z0, 25.0, grads=False, w_form=w_form)
    sm, wm = sv - 0.05, wv - 0.01
    cv = np.zeros(8); cv[5] = sm; cv[6] = wm
    _, Fb, cv2 = O.total_force(p, so, x, cv)
    assert cv2[3] == sv and cv2[4] == wv and cv2[5] == sm and cv2[6] == wm

    def E(xx):
        a, b, *_ = O.tube(xx, cidx, stack, so.Z0, 25.0, grads=False, w_form=w_form)
        return 0.5 * 2.5 * max(a - sm, 0) ** 2 + 0.5 * 0.8 * max(b - wm, 0) ** 2

    assert abs(cv2[2] - E(x)) < 1e-12
    h = 1e-5
    for i in (1, 12, 20):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            assert abs(-(E(xp) - E(xm)) / (2 * h) - Fb[c, i]) < 1e-6 * np.abs(Fb).max()


# ---------------------------------------------------------------------------
# eq (avCij): mean contact map over successful paths
# ---------------------------------------------------------------------------
def _ensemble(n=25, n_frames=4, n_paths=6, seed=2):
    rng = np.random.default_rng(seed)
    base = I.random_coil(n, seed)
    fr = base[None, None] + rng.normal(0, 1.5, size=(n_frames, n_paths, 3, n))
    return fr


def test_reference_equals_numpy_mean_over_masked_paths():
    fr = _ensemble()
    cidx = np.array([0, 1, 4, 5, 9, 10, 16, 17, 23, 24], dtype=np.int32)
    succ = np.array([1, 0, 1, 1, 0, 1], dtype=np.uint8)
    out, ns = O.update_reference(25, cidx, fr, succ)
    assert ns == 4
    for k in range(fr.shape[0]):
        maps = [O.contact_map(fr[k, q], cidx) for q in range(fr.shape[1]) if succ[q]]
        np.testing.assert_allclose(out[k], np.mean(maps, axis=0), rtol=1e-14)


def test_reference_of_identical_paths_is_their_map():
    fr = _ensemble(n_paths=1)
    fr = np.repeat(fr, 5, axis=1)
    cidx = np.arange(25, dtype=np.int32)
    out, ns = O.update_reference(25, cidx, fr, np.ones(5, dtype=np.uint8))
    for k in range(fr.shape[0]):
        np.testing.assert_allclose(out[k], O.contact_map(fr[k, 0], cidx), rtol=1e-14)


def test_reference_is_linear_in_the_path_set():
    fr = _ensemble()
    cidx = np.arange(25, dtype=np.int32)
    a = np.array([1, 1, 0, 0, 0, 0], dtype=np.uint8)
    b = np.array([0, 0, 1, 1, 1, 1], dtype=np.uint8)
    ra, _ = O.update_reference(25, cidx, fr, a)
    rb, _ = O.update_reference(25, cidx, fr, b)
    rab, _ = O.update_reference(25, cidx, fr, a | b)
    np.testing.assert_allclose(rab, (2 * ra + 4 * rb) / 6, rtol=1e-13)


def test_reference_with_no_success_reports_zero():
    fr = _ensemble()
    out, ns = O.update_reference(25, np.arange(25), fr, np.zeros(6, dtype=np.uint8))
    assert ns == 0 and np.all(out == 0.0)


# ---------------------------------------------------------------------------
# global progress coordinate sigma, eq (sigma)
# ---------------------------------------------------------------------------
def _stacks_sharing_frame(l, n=36, K=7, seed=5):
    """Three reference paths (three initial conditions) whose frame l is the
    same configuration and whose other frames differ."""
    native, frames, s = _path(n, K, seed)
    rng = np.random.default_rng(seed)
    cidx = s.cidx
    stacks = []
    for k in range(3):
        fr = frames + rng.normal(0, 0.8, frames.shape)
        fr[l] = frames[l]
        stacks.append(np.array([O.contact_map(f, cidx) for f in fr]))
    Z0 = float(np.sum(O.contact_map(native, cidx) ** 2))
    return frames, cidx, stacks, Z0


@pytest.mark.parametrize("l", [0, 2, 6])
def test_sigma_reaches_l_over_M_at_a_shared_frame(l):
    """Appendix limit for every stack at once: at the frame all paths share,
    s^k -> 1 - l/M for large lambda, so sigma -> l/M."""
    frames, cidx, stacks, Z0 = _stacks_sharing_frame(l)
    M = len(frames) - 1
    dmin = min(np.min(np.delete(O.tube(frames[l], cidx, st, Z0, 1.0, grads=False)[4], l)) for st in stacks)
    lam = 60.0 / dmin
    sg = O.sigma(frames[l], cidx, stacks, [Z0] * 3, lam)
    assert abs(sg - l / M) <= len(frames) * np.exp(-60.0) + 1e-14


def test_sigma_range_order_and_duplicates():
    frames, cidx, stacks, Z0 = _stacks_sharing_frame(3)
    rng = np.random.default_rng(9)
    for _ in range(5):
        x = frames[rng.integers(len(frames))] + rng.normal(0, 1.0, frames[0].shape)
        sg = O.sigma(x, cidx, stacks, [Z0] * 3, 13.5)
        assert 0.0 <= sg <= 1.0
        assert O.sigma(x, cidx, stacks[::-1], [Z0] * 3, 13.5) == pytest.approx(sg, rel=1e-14)
        # a stack counted twice weighs twice; one stack alone gives 1 - s
        one = 1.0 - O.tube(x, cidx, stacks[1], Z0, 13.5, grads=False)[0]
        assert O.sigma(x, cidx, [stacks[1]] * 2, [Z0] * 2, 13.5) == pytest.approx(one, rel=1e-14)
        two = O.sigma(x, cidx, stacks[:2], [Z0] * 2, 13.5)
        assert O.sigma(x, cidx, [stacks[0], stacks[1], stacks[1], stacks[0]], [Z0] * 4, 13.5) == pytest.approx(two,
                                                                                                             rel=1e-14)
