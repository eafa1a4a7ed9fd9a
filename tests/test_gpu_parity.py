"""GPU parity: the HIP library, called through its C ABI, against the FP64
CPU oracle on the same seeded inputs.

Tolerances (pair arithmetic in float32, sums in float64):
  z:      |z_gpu - z_ref| <= 1e-5 * max(z_ref, 1e-3 * Z0)
  forces: max_i |F_gpu,i - F_ref,i| <= 1e-5 * max_i |F_ref,i| per replica
          (normwise: a per-component relative error is meaningless near 0)
Forces are read back from one BAOAB step at kT = 0 from rest, where the new
velocity is exactly c1 dt F / m (float32 storage adds at most 6e-8).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1705_02180_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1705_02180_amd import scps
    return scps


def dev(a, dtype="f32"):
    import torch
    t = {"f32": torch.float32, "f64": torch.float64}[dtype]
    return torch.as_tensor(np.ascontiguousarray(a), dtype=t, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def context(S, w, params=None, exec_mode=0, replica_system=None, replica_base=0):
    ctx = S.Context.from_workload(w, exec_mode=exec_mode, params=params, replica_system=replica_system,
                                  replica_base=replica_base)
    for s, sy in enumerate(w.systems):
        ctx.set_reference_map(s, native_xyz=sy.native)
    return ctx


def normwise(a, b):
    """max_i |a_i - b_i| / max_i |b_i| over particles (3-vectors)."""
    d = np.linalg.norm((a - b).reshape(3, -1), axis=0).max()
    return d / max(np.linalg.norm(b.reshape(3, -1), axis=0).max(), 1e-300)


def single_system_workload(n, contact_idx, params, n_rep, seed=11, charges=True):
    rng = np.random.default_rng(seed)
    sy = I.System(n=n, contact_idx=np.asarray(contact_idx, dtype=np.int32),
                  mass=np.full(n, 12.011 * I.AMU, dtype=np.float32),
                  charge=(rng.normal(0, 0.3, n) if charges else np.zeros(n)).astype(np.float32),
                  native=I.compact_native(n, seed), start=I.persistent_start(n, seed + 1))
    return I.Workload(f"chain{n}", dict(params), [sy], np.zeros(n_rep, dtype=np.int32), 1)


def states(sy, n_rep, seed):
    """Different conformations per replica: random coils, a perturbed native, the start."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_rep):
        if r % 3 == 0:
            x = I.random_coil(sy.n, seed + 100 + r)
        elif r % 3 == 1:
            x = sy.native + rng.normal(0, 0.4, size=sy.native.shape)
        else:
            x = sy.start + rng.normal(0, 0.2, size=sy.start.shape)
        out.append(x.astype(np.float32))
    return np.stack(out)


# ---------------------------------------------------------------------------
# z and grad z
# ---------------------------------------------------------------------------
EVAL_CASES = [
    ("fip35_shaped_560", 560, "heavy", {}),
    ("ragged_100_all", 100, "all", {}),
    ("ragged_257_every3", 257, "every3", {}),
    ("seqsep35_300", 300, "all", {"min_seq_sep": 35}),
    ("cutoff12_200", 200, "all", {"r_cut_contact": 12.0}),
    ("tiny_2", 2, "all", {}),
    ("no_contacts_70", 70, "none", {}),
]


def _cidx(n, kind):
    if kind == "all":
        return np.arange(n)
    if kind == "heavy":
        return np.nonzero(np.arange(n) % 16 < 8)[0]
    if kind == "every3":
        return np.arange(0, n, 3)
    return np.zeros(0, dtype=np.int32)


@pytest.mark.parametrize("name,n,kind,over", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
def test_eval_z_and_grad_matches_oracle(S, name, n, kind, over):
    import torch
    p = dict(I._base_params())
    p.update(over)
    w = single_system_workload(n, _cidx(n, kind), p, 4)
    ctx = context(S, w)
    sy = w.systems[0]
    X = states(sy, 4, 5) if n > 2 else np.array([[[0.0, 6.0], [0.0, 1.0], [0.0, 2.0]]] * 4, dtype=np.float32)
    x = dev(X.ravel())
    z = torch.zeros(4, dtype=torch.float64, device="cuda")
    g = torch.zeros(3 * 4 * n, dtype=torch.float32, device="cuda")
    ctx.eval_z_and_grad(x, z, g)
    z_only = torch.zeros_like(z)
    ctx.eval_z_and_grad(x, z_only)
    torch.cuda.synchronize()
    zg, gg, zo = host(z), host(g).reshape(4, 3, n), host(z_only)
    osys = O.System.from_inputs(sy, p)
    for r in range(4):
        zr, gr = O.z_grad(X[r].astype(np.float64), osys.cidx, osys.native, p["r0_contact"],
                          p["r_cut_contact"], p["min_seq_sep"])
        bound = TOL * max(zr, 1e-3 * osys.Z0, 1e-300)
        assert abs(zg[r] - zr) <= bound, (r, zg[r], zr)
        assert abs(zo[r] - zr) <= bound
        if np.abs(gr).max() > 0:
            assert normwise(gg[r], gr) <= TOL, (r, normwise(gg[r], gr))
        else:
            assert np.all(gg[r] == 0)


def test_eval_grad_coef_scales_the_gradient(S):
    import torch
    p = dict(I._base_params())
    w = single_system_workload(130, np.arange(130), p, 3)
    ctx = context(S, w)
    X = states(w.systems[0], 3, 9)
    x = dev(X.ravel())
    z = torch.zeros(3, dtype=torch.float64, device="cuda")
    g1 = torch.zeros(3 * 3 * 130, dtype=torch.float32, device="cuda")
    g2 = torch.zeros_like(g1)
    ctx.eval_z_and_grad(x, z, g1)
    ctx.eval_z_and_grad(x, z, g2, dev([2.0, -0.5, 0.0], "f64"))
    a, b = host(g1).reshape(3, -1), host(g2).reshape(3, -1)
    np.testing.assert_allclose(b[0], 2.0 * a[0], rtol=1e-6, atol=0)
    np.testing.assert_allclose(b[1], -0.5 * a[1], rtol=1e-6, atol=0)
    assert np.all(b[2] == 0)


# ---------------------------------------------------------------------------
# forces of one step (rMD), both execution paths
# ---------------------------------------------------------------------------
def _force_readback_params(base, **kw):
    p = dict(base)
    p.update(integrator=1, kT=0.0, gamma=1e-3, dt=0.002)
    p.update(kw)
    return p


def _gpu_forces_one_step(S, w, p, X, cv0, exec_mode):
    import torch
    R = w.n_replicas
    ctx = context(S, w, params=p, exec_mode=exec_mode)
    x = dev(np.concatenate([np.ravel(a) for a in X]))        # replicas may have different lengths
    v = torch.zeros_like(x)
    cv = dev(cv0, "f64")
    ctx.step_replicas(x, v, cv, 1, step0=3)
    ctx.sync()
    c1 = math.exp(-p["gamma"] * p["dt"])
    V = host(v)
    out = []
    off = 0
    for r in range(R):
        sy = w.systems[w.replica_system[r]]
        n = sy.n
        m = sy.mass.astype(np.float64)
        out.append(V[3 * off:3 * (off + n)].reshape(3, n).astype(np.float64) * m / (c1 * p["dt"]))
        off += n
    return out, host(cv)


@pytest.mark.parametrize("exec_mode", [0, 1], ids=["persistent", "per_step"])
@pytest.mark.parametrize("case", ["fip35_shaped", "bias_only", "ragged_all"])
def test_step_forces_match_oracle(S, exec_mode, case):
    if case == "fip35_shaped":
        w = I.config2(n_replicas=6, n_steps=1)
        p = _force_readback_params(w.params, k_R=2e-3)
    elif case == "bias_only":
        w = I.config2(n_replicas=6, n_steps=1)
        p = _force_readback_params(w.params, k_R=0.5, k_bond=0.0, lj_eps=0.0, dh_prefactor=0.0)
    else:
        base = dict(I._base_params())
        w = single_system_workload(333, np.arange(333), base, 5)
        p = _force_readback_params(base, k_R=1e-2)
    sy = w.systems[0]
    R = w.n_replicas
    X = states(sy, R, 21)
    osys = O.System.from_inputs(sy, p)
    cv0 = np.zeros((R, 8))
    cv0[:, 1] = np.inf
    zs = [O.z_grad(X[r].astype(np.float64), osys.cidx, osys.native, grad=False) for r in range(R)]
    for r in range(1, R):         # replica 0 starts its running minimum; the others are biased
        cv0[r, 1] = 0.7 * zs[r] if r % 2 else 1.3 * zs[r]
    Fg, cvg = _gpu_forces_one_step(S, w, p, X, cv0, exec_mode)
    for r in range(R):
        F, Fb, cvr = O.total_force(p, osys, X[r].astype(np.float64), cv0[r])
        err = normwise(Fg[r], F)
        assert err <= TOL, (r, err)
        assert abs(cvg[r, 0] - cvr[0]) <= TOL * max(cvr[0], 1e-3 * osys.Z0)
        assert abs(cvg[r, 1] - cvr[1]) <= TOL * max(cvr[1], 1e-3 * osys.Z0)
        assert abs(cvg[r, 2] - cvr[2]) <= 1e-4 * max(cvr[2], 1e-12) + 1e-12
        # bias functional after the step (the oracle's own one-step accumulation)
        _, _, cvs, _ = O.steps(p, osys, r, X[r].astype(np.float64), np.zeros(X[r].shape), cv0[r], 1, step0=3)
        assert abs(cvg[r, 7] - cvs[7]) <= TOL * cvs[7] + 1e-300, (r, cvg[r, 7], cvs[7])
        assert (cvs[7] > 0) == (r % 2 == 1)                  # only the replicas below their z_m are biased


# ---------------------------------------------------------------------------
# noise: the counter layout and the normals
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("exec_mode", [0, 1], ids=["persistent", "per_step"])
def test_noise_matches_oracle_philox(S, exec_mode):
    import torch
    n, R = 150, 5
    p = dict(I._base_params())
    # free overdamped particles with unit noise amplitude: x1 = x0 + xi
    p.update(integrator=0, dt=1.0, gamma=1.0, kT=0.5, k_bond=0.0, lj_eps=0.0, dh_prefactor=0.0, k_R=0.0,
             seed=0x1234_5678_9ABC)
    w = single_system_workload(n, np.arange(0, n, 2), p, R, charges=False)
    w.systems[0].mass[:] = 1.0
    ctx = context(S, w, params=p, exec_mode=exec_mode, replica_base=7)
    x = torch.zeros(3 * n * R, dtype=torch.float32, device="cuda")
    cv = dev(np.tile([0, np.inf, 0, 0, 0, np.inf, np.inf, 0], (R, 1)), "f64")
    step = (1 << 32) + 5
    ctx.step_replicas(x, None, cv, 1, step0=step)
    got = host(x).reshape(R, 3, n)
    for r in range(R):
        want = O.normals(p["seed"], np.arange(n), 7 + r, step).T
        # same Philox words and uniforms; Box-Muller in float32 on the GPU
        # (a few ulp of |xi| <= ~5.5) against float64 in the oracle
        np.testing.assert_allclose(got[r], want, rtol=1e-6, atol=1e-6)


# ---------------------------------------------------------------------------
# one full noisy step and short trajectories
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("exec_mode", [0, 1], ids=["persistent", "per_step"])
def test_one_noisy_baoab_step_matches_oracle(S, exec_mode):
    import torch
    w = I.config2(n_replicas=4, n_steps=1)
    p = dict(w.params)
    sy = w.systems[0]
    X = states(sy, 4, 3)
    V = np.stack([w.initial_v(5)[3 * sy.n * r:3 * sy.n * (r + 1)].reshape(3, sy.n) for r in range(4)])
    ctx = context(S, w, exec_mode=exec_mode)
    x, v = dev(X.ravel()), dev(V.ravel())
    cv = dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(x, v, cv, 1, step0=11)
    Xg, Vg = host(x).reshape(4, 3, -1), host(v).reshape(4, 3, -1)
    osys = O.System.from_inputs(sy, p)
    for r in range(4):
        xo, vo, cvo, _ = O.steps(p, osys, r, X[r].astype(np.float64), V[r].astype(np.float64),
                                 w.initial_cvstate()[r], 1, step0=11)
        disp = np.abs(xo - X[r]).max()
        assert np.abs(Xg[r] - xo).max() <= TOL * disp + 2.0 ** -24 * np.abs(xo).max()
        assert np.abs(Vg[r] - vo).max() <= TOL * np.abs(vo).max()


def test_short_trajectory_pathwise_config1(S):
    import torch
    w = I.config1(n_replicas=16, n_steps=10)
    p = dict(w.params)
    ctx = context(S, w)
    x = dev(w.initial_x())
    cv = dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(x, None, cv, 10)
    ctx.sync()
    osys = O.System.from_inputs(w.systems[0], p)
    X0 = w.initial_x().reshape(16, 3, 20).astype(np.float64)
    Xg = host(x).reshape(16, 3, 20)
    CVg = host(cv)
    for r in range(16):
        xo, _, cvo, _ = O.steps(p, osys, r, X0[r], None, w.initial_cvstate()[r], 10)
        disp = np.abs(xo - X0[r]).max()
        assert np.abs(Xg[r] - xo).max() <= 1e-4 * disp, (r, np.abs(Xg[r] - xo).max() / disp)
        assert abs(CVg[r, 1] - cvo[1]) <= 1e-4 * cvo[1]
        # bias functional T = dt sum |F_bias|^2 / (m gamma): a bias-force error below
        # tol * max|F| bounds |sqrt(T_gpu) - sqrt(T)| by tol * max|F| sqrt(dt steps sum 1/(m gamma))
        F0 = O.total_force(p, osys, X0[r], w.initial_cvstate()[r])[0]
        fmax = np.linalg.norm(F0, axis=0).max()
        m = osys.mass.astype(np.float64)
        tol_t = 1e-4 * fmax * np.sqrt(p["dt"] * 10 * np.sum(1.0 / (m * p["gamma"])))
        assert cvo[7] > 0 and abs(np.sqrt(CVg[r, 7]) - np.sqrt(cvo[7])) <= tol_t


def test_persistent_and_per_step_paths_agree(S):
    import torch
    w = I.config2(n_replicas=8, n_steps=20)
    res = []
    for mode in (0, 1):
        ctx = context(S, w, exec_mode=mode)
        x, v = dev(w.initial_x()), dev(w.initial_v(1))
        cv = dev(w.initial_cvstate(), "f64")
        ctx.step_replicas(x, v, cv, 20, step0=100)
        ctx.sync()
        res.append((host(x), host(v), host(cv)))
    x0 = w.initial_x()
    disp = np.abs(res[0][0] - x0).max()
    assert np.abs(res[0][0] - res[1][0]).max() <= 1e-4 * disp
    np.testing.assert_allclose(res[0][2][:, :2], res[1][2][:, :2], rtol=1e-5)


def test_batched_equals_one_replica_contexts(S):
    import torch
    w = I.config2(n_replicas=4, n_steps=6)
    xb, vb = dev(w.initial_x()), dev(w.initial_v(2))
    cvb = dev(w.initial_cvstate(), "f64")
    ctx = context(S, w)
    ctx.step_replicas(xb, vb, cvb, 6)
    n3 = 3 * w.systems[0].n
    X0, V0 = w.initial_x(), w.initial_v(2)
    for r in range(4):
        c1 = context(S, w, replica_system=[0], replica_base=r)
        x1, v1 = dev(X0[r * n3:(r + 1) * n3]), dev(V0[r * n3:(r + 1) * n3])
        cv1 = dev(w.initial_cvstate()[r:r + 1], "f64")
        c1.step_replicas(x1, v1, cv1, 6)
        disp = np.abs(host(xb)[r * n3:(r + 1) * n3] - X0[r * n3:(r + 1) * n3]).max()
        assert np.abs(host(x1) - host(xb)[r * n3:(r + 1) * n3]).max() <= 1e-4 * disp


def test_split_calls_equal_one_call(S):
    w = I.config1(n_replicas=4, n_steps=8)
    ctx = context(S, w)
    xa, cva = dev(w.initial_x()), dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(xa, None, cva, 8, step0=40)
    xb, cvb = dev(w.initial_x()), dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(xb, None, cvb, 3, step0=40)
    ctx.step_replicas(xb, None, cvb, 5, step0=43)
    # float64 atomics from different wavefronts commute only up to rounding
    disp = np.abs(host(xa) - w.initial_x()).max()
    assert np.abs(host(xa) - host(xb)).max() <= 1e-5 * disp
    np.testing.assert_allclose(host(cva)[:, :3], host(cvb)[:, :3], rtol=1e-6)


def test_frames_are_recorded(S):
    import torch
    w = I.config1(n_replicas=3, n_steps=10)
    for mode in (0, 1):
        ctx = context(S, w, exec_mode=mode)
        x, cv = dev(w.initial_x()), dev(w.initial_cvstate(), "f64")
        fr = torch.full((10 // 4 + 1, 3 * 60), -1.0, dtype=torch.float32, device="cuda")
        ctx.step_replicas(x, None, cv, 10, record_every=4, frames=fr)
        x2, cv2 = dev(w.initial_x()), dev(w.initial_cvstate(), "f64")
        ctx.step_replicas(x2, None, cv2, 8)
        F = host(fr)
        np.testing.assert_array_equal(F[0], w.initial_x())
        disp = np.abs(host(x2) - w.initial_x()).max()
        assert np.abs(F[2] - host(x2)).max() <= 1e-5 * disp
        assert np.abs(F[1] - w.initial_x()).max() > 0


def test_nonfinite_replica_is_reported(S):
    import torch
    w = I.config1(n_replicas=3, n_steps=2)
    ctx = context(S, w)
    X = w.initial_x()
    X[60 + 5] = np.nan
    x, cv = dev(X), dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(x, None, cv, 2)
    with pytest.raises(S.ScpsError) as e:
        ctx.sync()
    assert e.value.status == -6 and "[1]" in str(e.value)


# ---------------------------------------------------------------------------
# eq (avCij) and the SCPS bias
# ---------------------------------------------------------------------------
def _ensemble_frames(sy, n_frames, n_paths, seed):
    rng = np.random.default_rng(seed)
    out = np.empty((n_frames, n_paths, 3, sy.n), dtype=np.float32)
    for k in range(n_frames):
        lam = k / max(n_frames - 1, 1)
        base = (1 - lam) * sy.start + lam * sy.native
        for q in range(n_paths):
            out[k, q] = base + rng.normal(0, 0.8, size=base.shape)
    return out


def test_update_reference_matches_oracle(S):
    base = dict(I._base_params())
    w = single_system_workload(200, np.arange(0, 200, 2), base, 2)
    sy = w.systems[0]
    ctx = context(S, w)
    fr = _ensemble_frames(sy, 6, 5, 4)
    succ = np.array([1, 0, 1, 1, 1], dtype=np.uint8)
    maps = ctx.update_reference_from_paths(0, dev(fr.ravel()), 5, 6, succ, want_maps=True)
    want, ns = O.update_reference(sy.n, sy.contact_idx, fr.astype(np.float64), succ)
    assert ns == 4
    np.testing.assert_allclose(maps, want, rtol=1e-12, atol=1e-15)
    with pytest.raises(S.ScpsError) as e:
        ctx.update_reference_from_paths(0, dev(fr.ravel()), 5, 6, np.zeros(5, dtype=np.uint8))
    assert e.value.status == -7


SCPS_CASES = [
    # id, chain sizes, contact sets, frames K, replicas, bias only, parameters
    ("all_180_K9", [180], ["all"], 9, 4, False, {}),
    ("every3_300_K9", [300], ["every3"], 9, 4, False, {}),
    ("bias_only_180_K9", [180], ["all"], 9, 4, True, {}),
    ("all_130_K51_R40", [130], ["all"], 51, 40, False, {}),
    ("bias_only_150_K33_seqsep5", [150], ["all"], 33, 6, True, {"min_seq_sep": 5}),
    ("bias_only_160_K17_cutoff12", [160], ["all"], 17, 4, True, {"r_cut_contact": 12.0}),
    ("two_systems_K20", [150, 200], ["all", "every3"], 20, 6, False, {}),
    ("smallest_stack_K2", [100], ["all"], 2, 3, False, {}),
    ("K53_partial_frame_pairs", [120], ["all"], 53, 4, False, {}),
    ("K64_bias_only", [120], ["all"], 64, 5, True, {}),
    ("K65_one_frame_past_a_block", [100], ["every3"], 65, 3, False, {}),
    ("K72_protocol_frames", [140], ["all"], 72, 5, False, {}),
    ("K128_largest_stack_R36", [110], ["all"], 128, 36, False, {}),
    ("two_systems_K48_K100", [130, 150], ["all", "every3"], [48, 100], 4, True, {}),
    ("seqsep35_200_K21", [200], ["all"], 21, 5, False, {"min_seq_sep": 35}),
    ("one_block_60_K5", [60], ["all"], 5, 3, False, {}),
]
SCPS_FORMS = [(0, 0), (2, 0), (0, 1), (3, 0)]


@pytest.mark.parametrize("exec_mode,w_form", SCPS_FORMS,
                         ids=["fused", "two_pass", "fused_w_without_1_over_lambda", "fused_nonbonded_beside"])
@pytest.mark.parametrize("name,sizes,kinds,K,R,bias_only,extra", SCPS_CASES, ids=[c[0] for c in SCPS_CASES])
def test_scps_step_forces_match_oracle(S, name, sizes, kinds, K, R, bias_only, extra, exec_mode, w_form):
    """One SCPS step (distances to all K frames, tube variables and ratchets,
    bias + physics) against the oracle, with the frame stack built on the GPU
    from recorded paths and, separately, uploaded from the oracle's FP64 maps.
    K > 64 takes the distance pass in two frame blocks and the bias pass in
    two MFMA chains; R > 32 several replica groups; two systems two stacks
    (of different sizes when K is a list).  Both forms of the bias: the
    effective references formed inside the bias pass (fused) and written to
    device memory first (two_pass); and both forms of w (with the 1/lambda of
    eq (wX), and without it as eq (awXa) prints it)."""
    import torch
    base = dict(I._base_params())
    p = _force_readback_params(base, bias_mode=1, lam=13.5, k_s=50.0, k_w=5.0, w_form=w_form, **extra)
    Ks = list(K) if isinstance(K, list) else [K] * len(sizes)
    if bias_only:
        p.update(k_bond=0.0, lj_eps=0.0, dh_prefactor=0.0)
    n_paths = 4
    systems, stacks, frames = [], [], []
    for s_id, (n, kind) in enumerate(zip(sizes, kinds)):
        rng = np.random.default_rng(11 + s_id)
        sy = I.System(n=n, contact_idx=np.asarray(_cidx(n, kind), dtype=np.int32),
                      mass=np.full(n, 12.011 * I.AMU, dtype=np.float32),
                      charge=rng.normal(0, 0.3, n).astype(np.float32),
                      native=I.compact_native(n, 11 + s_id), start=I.persistent_start(n, 12 + s_id))
        fr = _ensemble_frames(sy, Ks[s_id], n_paths, 8 + s_id)
        st, ns = O.update_reference(sy.n, sy.contact_idx, fr.astype(np.float64), np.ones(n_paths, dtype=np.uint8),
                                    p["r0_contact"], p["r_cut_contact"])
        assert ns == n_paths
        systems.append(sy)
        stacks.append(st)
        frames.append(fr)
    rsys = np.arange(R, dtype=np.int32) % len(sizes)
    w = I.Workload(name, dict(p), systems, rsys, 1)
    osys = [O.System(sy.n, sy.contact_idx, sy.mass, sy.charge, p, native_xyz=sy.native, stack=st)
            for sy, st in zip(systems, stacks)]
    X, cv0 = [], np.zeros((R, 8))
    cv0[:, 5:7] = np.inf
    for r in range(R):
        fr = frames[rsys[r]]
        X.append(fr[(3 + 2 * r) % Ks[rsys[r]], r % n_paths].astype(np.float32))
        if r >= 1:
            sv, wv, *_ = O.tube(X[r].astype(np.float64), osys[rsys[r]].cidx, stacks[rsys[r]], osys[rsys[r]].Z0,
                                p["lam"], p["r0_contact"], p["r_cut_contact"], p["min_seq_sep"], grads=False,
                                w_form=w_form)
            cv0[r, 5] = sv - 0.05 * (1 + r % 3)
            cv0[r, 6] = wv - 0.01 * (1 + r % 3)
    want = [O.total_force(p, osys[rsys[r]], X[r].astype(np.float64), cv0[r]) for r in range(R)]
    xflat = np.concatenate([x.ravel() for x in X])
    c1 = math.exp(-p["gamma"] * p["dt"])
    for how in ("update", "upload"):
        ctx = context(S, w, params=p, exec_mode=exec_mode)
        for s_id, sy in enumerate(systems):
            if how == "update":
                maps = ctx.update_reference_from_paths(s_id, dev(frames[s_id].ravel()), n_paths, Ks[s_id],
                                                       np.ones(n_paths, dtype=np.uint8), want_maps=True)
                np.testing.assert_allclose(maps, stacks[s_id], rtol=1e-12, atol=1e-15)
            else:
                ctx.set_reference_map(s_id, maps=stacks[s_id])
        x = dev(xflat)
        v = torch.zeros_like(x)
        cv = dev(cv0, "f64")
        ctx.step_replicas(x, v, cv, 1)
        ctx.sync()
        V = host(v)
        CV = host(cv)
        off = 0
        for r in range(R):
            sy = systems[rsys[r]]
            n = sy.n
            Vr = V[3 * off:3 * (off + n)].reshape(3, n).astype(np.float64) * sy.mass.astype(np.float64) / (c1 * p["dt"])
            off += n
            F, Fb, cvr = want[r]
            if np.abs(F).max() > 0:
                assert normwise(Vr, F) <= TOL, (how, r, normwise(Vr, F))
            else:
                assert np.all(Vr == 0)
            if bias_only:
                assert r == 0 or np.abs(Fb).max() > 0          # the ratchets are active
            np.testing.assert_allclose(CV[r, 3:7], cvr[3:7], rtol=0, atol=1e-5, err_msg=f"{how} replica {r}")
            # bias functional T = dt sum_i |F_bias,i|^2 / (m_i gamma): a bias-force error within the
            # normwise bound TOL max_i |F_i| moves sqrt(T) by at most TOL max_i |F_i| sqrt(dt sum_i 1/(m_i gamma))
            _, _, cvs, _ = O.steps(p, osys[rsys[r]], r, X[r].astype(np.float64), np.zeros(X[r].shape), cv0[r], 1)
            fmax = np.linalg.norm(F, axis=0).max()
            tol_t = TOL * fmax * np.sqrt(p["dt"] * np.sum(1.0 / (sy.mass.astype(np.float64) * p["gamma"])))
            assert abs(np.sqrt(CV[r, 7]) - np.sqrt(cvs[7])) <= tol_t + 1e-300, (how, r, CV[r, 7], cvs[7])
        ctx.close()


@pytest.mark.parametrize("other_mode", [2, 3], ids=["two_pass", "nonbonded_beside"])
def test_scps_forms_agree_over_steps(S, other_mode):
    """The forms of the SCPS step (effective references formed inside the
    bias pass, written to device memory first, or formed inside the bias pass
    with the nonbonded pass on a second stream beside the distance pass) step
    the same replicas alike over ten noisy BAOAB steps: they differ only in
    the float32 summation order of the force partials.  300 beads with every third in
    the contact set (tiles without contacts, blocks straddling the contact
    set), 36 replicas (two replica groups), 17 frames."""
    import torch
    base = dict(I._base_params(), bias_mode=1, lam=13.5, k_s=50.0, k_w=5.0)
    n, R, K, n_paths = 300, 36, 17, 4
    rng = np.random.default_rng(21)
    sy = I.System(n=n, contact_idx=np.asarray(_cidx(n, "every3"), dtype=np.int32),
                  mass=np.full(n, 12.011 * I.AMU, dtype=np.float32),
                  charge=rng.normal(0, 0.3, n).astype(np.float32),
                  native=I.compact_native(n, 21), start=I.persistent_start(n, 22))
    w = I.Workload("chain300_scps", dict(base), [sy], np.zeros(R, dtype=np.int32), 1)
    fr = _ensemble_frames(sy, K, n_paths, 23)               # the recorded paths behind the stack
    x0 = _clean_starts(sy, R, 24).ravel()                   # no overlapping beads: the runs stay finite
    cv0 = np.zeros((R, 8))
    cv0[:, 5:7] = np.inf
    out = []
    for mode in (0, other_mode):
        ctx = context(S, w, params=base, exec_mode=mode)
        ctx.update_reference_from_paths(0, dev(fr.ravel()), n_paths, K, np.ones(n_paths, dtype=np.uint8))
        x, v, cv = dev(x0), dev(np.zeros_like(x0)), dev(cv0, "f64")
        ctx.step_replicas(x, v, cv, 10, step0=7)
        ctx.sync()
        out.append((host(x), host(v), host(cv)))
        ctx.close()
    (xa, va, cva), (xb, vb, cvb) = out
    assert np.isfinite(xa).all() and np.isfinite(xb).all()
    disp = np.abs(xa - x0).max()
    assert disp > 0
    assert np.abs(xa - xb).max() <= 1e-4 * disp, (np.abs(xa - xb).max(), disp)
    assert np.abs(va - vb).max() <= 1e-4 * np.abs(va).max()
    np.testing.assert_allclose(cva[:, 3:7], cvb[:, 3:7], rtol=0, atol=1e-6)
    assert (cva[:, 7] > 0).any()                     # the tube ratchets acted
    np.testing.assert_allclose(cva[:, 7], cvb[:, 7], rtol=1e-4, atol=1e-12 * cva[:, 7].max())


@pytest.mark.parametrize("exec_mode", [0, 3], ids=["one_stream", "nonbonded_beside"])
def test_scps_step_on_a_caller_stream(S, exec_mode):
    """Stepping an SCPS context on a non-default torch stream gives what the
    default stream gives (up to the float32 summation order of the force
    partials), and the caller's next work on that stream sees the updated
    state -- also with the nonbonded pass on the context's second stream,
    forked from and joined back to the caller's stream."""
    import torch
    base = dict(I._base_params(), bias_mode=1, lam=13.5, k_s=50.0, k_w=5.0)
    n, R, K, n_paths = 150, 6, 9, 3
    w = single_system_workload(n, np.arange(n), base, R, seed=31)
    sy = w.systems[0]
    fr = _ensemble_frames(sy, K, n_paths, 32)
    x0 = _clean_starts(sy, R, 33).ravel()
    cv0 = np.zeros((R, 8))
    cv0[:, 5:7] = np.inf
    out = []
    for use_side in (False, True):
        side = torch.cuda.Stream() if use_side else torch.cuda.current_stream()
        with torch.cuda.stream(side):
            ctx = context(S, w, params=base, exec_mode=exec_mode)
            ctx.update_reference_from_paths(0, dev(fr.ravel()), n_paths, K, np.ones(n_paths, dtype=np.uint8))
            x, v, cv = dev(x0), dev(np.zeros_like(x0)), dev(cv0, "f64")
            ctx.step_replicas(x, v, cv, 8, step0=11)
            moved = (x - dev(x0)).abs().max()          # queued on the same stream, after the steps
        side.synchronize()
        out.append((host(x), host(v), host(cv), float(moved)))
        ctx.close()
    (xa, va, cva, ma), (xb, vb, cvb, mb) = out
    disp = np.abs(xa - x0).max()
    assert disp > 0 and abs(ma - disp) <= 1e-6 * disp and abs(mb - np.abs(xb - x0).max()) <= 1e-6 * disp
    assert np.abs(xa - xb).max() <= 1e-4 * disp, (np.abs(xa - xb).max(), disp)
    assert np.abs(va - vb).max() <= 1e-4 * np.abs(va).max()
    np.testing.assert_allclose(cva[:, 3:7], cvb[:, 3:7], rtol=0, atol=1e-6)


# ---------------------------------------------------------------------------
# autograd wrapper
# ---------------------------------------------------------------------------
def test_zbias_autograd_matches_oracle_gradient(S):
    import torch
    base = dict(I._base_params())
    base["k_R"] = 3e-3
    w = single_system_workload(400, np.arange(400), base, 3)
    sy = w.systems[0]
    ctx = context(S, w)
    X = states(sy, 3, 13)
    osys = O.System.from_inputs(sy, base)
    zr = [O.z_grad(X[r].astype(np.float64), osys.cidx, osys.native) for r in range(3)]
    zm = np.array([0.8 * zr[0][0], 1.2 * zr[1][0], 0.5 * zr[2][0]])
    x = dev(X.ravel()).requires_grad_(True)
    z, Eb = S.zbias(x, dev(zm, "f64"), ctx)
    (z.sum() + Eb.sum()).backward()
    G = host(x.grad).reshape(3, 3, -1)
    for r in range(3):
        d = zr[r][0] - zm[r]
        th = 1.0 if d >= 0 else 0.0
        assert abs(host(Eb)[r] - 0.5 * base["k_R"] * d * d * th) <= 1e-4 * max(0.5 * base["k_R"] * d * d, 1e-12)
        want = (1.0 + base["k_R"] * d * th) * zr[r][1]
        assert normwise(G[r], want) <= TOL
    # central differences of the oracle's z (float64, h = 1e-4 A) on 8 particles
    rng = np.random.default_rng(0)
    for r in range(3):
        xr = X[r].astype(np.float64)
        for i in rng.choice(sy.n, 8, replace=False):
            for c in range(3):
                xp = xr.copy(); xp[c, i] += 1e-4
                xm = xr.copy(); xm[c, i] -= 1e-4
                fd = (O.z_grad(xp, osys.cidx, osys.native, grad=False) -
                      O.z_grad(xm, osys.cidx, osys.native, grad=False)) / 2e-4
                d = zr[r][0] - zm[r]
                want = (1.0 + base["k_R"] * d * (d >= 0)) * fd
                assert abs(G[r, c, i] - want) <= 2e-4 * np.abs(G[r]).max()


def test_zbias_partial_gradients_and_no_grad_forward(S):
    """The kept dz/dx serves any output weights: E_b alone, z alone, and a
    forward without a gradient gives the same z."""
    import torch
    base = dict(I._base_params(), k_R=3e-3)
    w = single_system_workload(260, np.arange(260), base, 4)
    sy = w.systems[0]
    ctx = context(S, w)
    X = states(sy, 4, 17)
    osys = O.System.from_inputs(sy, base)
    zr = [O.z_grad(X[r].astype(np.float64), osys.cidx, osys.native) for r in range(4)]
    zm = np.array([0.8, 1.3, 0.6, 0.95]) * np.array([z[0] for z in zr])
    for weights in ((1.0, 0.0), (0.0, 1.0), (2.5, -0.7)):
        x = dev(X.ravel()).requires_grad_(True)
        z, Eb = S.zbias(x, dev(zm, "f64"), ctx)
        (weights[0] * z.sum() + weights[1] * Eb.sum()).backward()
        G = host(x.grad).reshape(4, 3, -1)
        for r in range(4):
            d = zr[r][0] - zm[r]
            want = (weights[0] + weights[1] * base["k_R"] * d * (d >= 0)) * zr[r][1]
            if np.abs(want).max() == 0:
                assert np.all(G[r] == 0)
            else:
                assert normwise(G[r], want) <= TOL, (weights, r)
    with torch.no_grad():
        z2, _ = S.zbias(dev(X.ravel()), dev(zm, "f64"), ctx)
    np.testing.assert_allclose(host(z2), host(z), rtol=1e-8)      # z-only and z + gradient passes: float32 partial order
    # the scaling entry point alone, in place, on seeded values
    rng = np.random.default_rng(6)
    g = rng.normal(size=3 * 4 * sy.n).astype(np.float32)
    coef = rng.normal(size=4)
    t = dev(g)
    ctx.scale_by_replica(t, dev(coef, "f64"), t)
    want = (coef[:, None] * g.reshape(4, -1).astype(np.float64)).astype(np.float32).ravel()
    np.testing.assert_array_equal(host(t), want)
    ctx.close()


def test_fused_zbias_calls_match_the_separate_calls(S):
    """scps_eval_zbias against scps_eval_z_and_grad + scps_ratchet_energy (z
    and E_b bit for bit, dz/dx up to the order of the float64 atomic sums)
    and scps_zbias_backward against scps_ratchet_energy's coef +
    scps_scale_by_replica (bit for bit) with contiguous, broadcast (stride 0)
    and strided incoming gradients, one of them absent; a forward without
    dz/dx gives the same z and E_b; argument errors come from the library."""
    import ctypes as C
    import torch
    base = dict(I._base_params(), k_R=4e-3)
    w = single_system_workload(330, np.arange(330), base, 5)
    sy = w.systems[0]
    ctx = context(S, w)
    R = 5
    X = states(sy, R, 23)
    x = dev(X.ravel())
    z0 = torch.empty(R, dtype=torch.float64, device="cuda")
    ctx.eval_z_and_grad(x, z0)
    zm = z0 * torch.tensor([0.8, 1.2, 1.0, 0.5, 1.01], dtype=torch.float64, device="cuda")
    z_a, eb_a = torch.empty_like(z0), torch.empty_like(z0)
    dz_a = torch.empty_like(x)
    ctx.eval_z_and_grad(x, z_a, dz_a)
    ctx.ratchet_energy(z_a, zm, eb_a)
    z_b, eb_b = torch.empty_like(z0), torch.empty_like(z0)
    dz_b = torch.empty_like(x)
    ctx.eval_zbias(x, zm, z_b, eb_b, dz_b)
    assert torch.equal(z_a, z_b) and torch.equal(eb_a, eb_b)
    assert (host(eb_b) > 0).any() and (host(eb_b) == 0).any()        # replicas on both sides of z_m
    np.testing.assert_allclose(host(dz_b), host(dz_a), rtol=1e-6, atol=1e-7 * np.abs(host(dz_a)).max())
    z_c, eb_c = torch.empty_like(z0), torch.empty_like(z0)
    ctx.eval_zbias(x, zm, z_c, eb_c, None)
    np.testing.assert_allclose(host(z_c), host(z_b), rtol=1e-8)
    np.testing.assert_allclose(host(eb_c), host(eb_b), rtol=1e-6, atol=1e-12)
    rng = np.random.default_rng(24)
    gz_full = dev(rng.normal(size=2 * R), "f64")
    cases = [(dev(rng.normal(size=R), "f64"), dev(rng.normal(size=R), "f64")),
             (torch.full((1,), 1.5, dtype=torch.float64, device="cuda").expand(R), None),
             (None, torch.full((1,), -0.7, dtype=torch.float64, device="cuda").expand(R)),
             (gz_full[::2], gz_full[1::2])]
    for gz, gE in cases:
        coef = torch.empty_like(z0)
        ctx.ratchet_energy(z_b, zm, None, None if gz is None else gz.contiguous(),
                           None if gE is None else gE.contiguous(), coef)
        want = torch.empty_like(x)
        ctx.scale_by_replica(dz_b, coef, want)
        got = torch.empty_like(x)
        ctx.zbias_backward(z_b, zm, gz, gE, dz_b, got)
        assert torch.equal(got, want)
    lib, h = S._lib, ctx._ctx()
    p = lambda t: C.c_void_p(t.data_ptr())
    assert lib.scps_zbias_backward(h, p(z_b), p(zm), p(z_b), C.c_int64(-1), None, C.c_int64(0), p(dz_b),
                                   p(got)) == -1
    assert lib.scps_zbias_backward(h, p(z_b), None, None, C.c_int64(0), None, C.c_int64(0), p(dz_b), p(got)) == -1
    assert lib.scps_eval_zbias(h, p(x), None, p(z_c), p(eb_c), None) == -1
    ctx.close()


def test_zbias_on_uneven_systems_matches_oracle(S):
    """The autograd wrapper over replicas of two chains of different lengths
    (one with every third particle in the contact set), interleaved: z, E_b
    and the gradient of z + 2 E_b per replica against the oracle (the fused
    forward and backward index each replica's own particles and order)."""
    import torch
    base = dict(I._base_params(), k_R=5e-3)
    rng = np.random.default_rng(41)
    systems = []
    for n, kind, seed in ((150, "all", 42), (333, "every3", 43)):
        systems.append(I.System(n=n, contact_idx=np.asarray(_cidx(n, kind), dtype=np.int32),
                                mass=np.full(n, 12.011 * I.AMU, dtype=np.float32),
                                charge=rng.normal(0, 0.3, n).astype(np.float32), native=I.compact_native(n, seed),
                                start=I.persistent_start(n, seed + 1)))
    rsys = np.array([1, 0, 1, 0, 1], dtype=np.int32)
    R = len(rsys)
    w = I.Workload("two_chains_zbias", dict(base), systems, rsys, 1)
    ctx = context(S, w)
    X = [_clean_starts(systems[s], 1, 50 + r)[0] for r, s in enumerate(rsys)]
    osys = [O.System.from_inputs(sy, base) for sy in systems]
    zr = [O.z_grad(X[r].astype(np.float64), osys[s].cidx, osys[s].native) for r, s in enumerate(rsys)]
    zm = np.array([0.7, 1.3, 0.9, 1.1, 0.5]) * np.array([z[0] for z in zr])
    x = dev(np.concatenate([xr.ravel() for xr in X])).requires_grad_(True)
    z, Eb = S.zbias(x, dev(zm, "f64"), ctx)
    (z.sum() + 2.0 * Eb.sum()).backward()
    G, zg, Ebg = host(x.grad), host(z), host(Eb)
    off = 0
    for r, s in enumerate(rsys):
        n = systems[s].n
        d = zr[r][0] - zm[r]
        th = 1.0 if d >= 0 else 0.0
        assert abs(zg[r] - zr[r][0]) <= 1e-5 * zr[r][0]
        assert abs(Ebg[r] - 0.5 * base["k_R"] * d * d * th) <= 1e-4 * max(0.5 * base["k_R"] * d * d, 1e-12)
        want = (1.0 + 2.0 * base["k_R"] * d * th) * zr[r][1]
        assert normwise(G[3 * off:3 * (off + n)].reshape(3, n), want) <= TOL, r
        off += n
    assert off * 3 == G.size
    ctx.close()


# ---------------------------------------------------------------------------
# the benchmark configuration at full size, sampled replicas
# ---------------------------------------------------------------------------
def test_full_config2_sampled(S):
    import torch
    w = I.config2()                       # 256 replicas x 560 particles
    p = _force_readback_params(w.params, k_R=2e-3)
    sy = w.systems[0]
    R = w.n_replicas
    rng = np.random.default_rng(17)
    X = np.stack([sy.start + rng.normal(0, 0.5, size=sy.start.shape) for _ in range(R)]).astype(np.float32)
    osys = O.System.from_inputs(sy, p)
    cv0 = np.zeros((R, 8))
    cv0[:, 1] = np.inf
    sample = [0, 1, 77, 128, 200, 255]
    for r in sample[1:]:
        cv0[r, 1] = 0.9 * O.z_grad(X[r].astype(np.float64), osys.cidx, osys.native, grad=False)
    Fg, cvg = _gpu_forces_one_step(S, w, p, X, cv0, 0)
    for r in sample:
        F, _, cvr = O.total_force(p, osys, X[r].astype(np.float64), cv0[r])
        assert normwise(Fg[r], F) <= TOL, (r, normwise(Fg[r], F))
        assert abs(cvg[r, 0] - cvr[0]) <= TOL * max(cvr[0], 1e-3 * osys.Z0)


# ---------------------------------------------------------------------------
# degenerate calls and limits
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("exec_mode", [0, 1], ids=["persistent", "per_step"])
def test_zero_steps_leave_state_unchanged(S, exec_mode):
    w = I.config2(n_replicas=3, n_steps=1)
    ctx = context(S, w, exec_mode=exec_mode)
    x0, v0, cv0 = w.initial_x(), w.initial_v(2), w.initial_cvstate()
    cv0[:, 7] = 1.25
    x, v, cv = dev(x0), dev(v0), dev(cv0, "f64")
    ctx.step_replicas(x, v, cv, 0, step0=5)
    ctx.sync()
    np.testing.assert_array_equal(host(x), x0)
    np.testing.assert_array_equal(host(v), v0)
    np.testing.assert_array_equal(host(cv), cv0)


@pytest.mark.parametrize("exec_mode", [0, 1], ids=["persistent", "per_step"])
@pytest.mark.parametrize("cut", [0.0, 12.0], ids=["no_cutoff", "cutoffs_lists"])
def test_two_particle_chain_matches_oracle(S, exec_mode, cut):
    base = dict(I._base_params(), r_cut_contact=cut, r_cut_nb=cut)
    p = _force_readback_params(base, k_R=0.3)
    w = single_system_workload(2, np.arange(2), p, 2)
    sy = w.systems[0]
    X = np.stack([sy.native + 0.7, sy.native * 1.6]).astype(np.float32)
    osys = O.System.from_inputs(sy, p)
    cv0 = np.zeros((2, 8))
    cv0[:, 1] = np.inf
    cv0[1, 1] = 0.5 * O.z_grad(X[1].astype(np.float64), osys.cidx, osys.native, grad=False)
    Fg, cvg = _gpu_forces_one_step(S, w, p, X, cv0, exec_mode)
    for r in range(2):
        F, _, cvr = O.total_force(p, osys, X[r].astype(np.float64), cv0[r])
        assert normwise(Fg[r], F) <= TOL, (r, normwise(Fg[r], F))
        assert abs(cvg[r, 0] - cvr[0]) <= TOL * max(cvr[0], 1e-3 * osys.Z0)


def test_frame_stack_limit_is_enforced(S):
    """Stacks hold 2 .. 128 frames; 129 are rejected with SHAPE by both ways of
    setting a stack, and the context stays usable."""
    base = dict(I._base_params(), bias_mode=1)
    w = single_system_workload(70, np.arange(70), base, 2)
    sy = w.systems[0]
    ctx = context(S, w, params=base)
    fr = _ensemble_frames(sy, 129, 1, 3)
    with pytest.raises(S.ScpsError) as e:
        ctx.update_reference_from_paths(0, dev(fr.ravel()), 1, 129, np.ones(1, dtype=np.uint8))
    assert e.value.status == -2
    P = 70 * 69 // 2
    with pytest.raises(S.ScpsError) as e:
        ctx.set_reference_map(0, maps=np.full((129, P), 0.5))
    assert e.value.status == -2
    import torch
    x = dev(np.stack([sy.start, sy.start]).astype(np.float32).ravel())
    with pytest.raises(S.ScpsError) as e:        # SCPS stepping needs a stack of >= 2 frames
        ctx.step_replicas(x, torch.zeros_like(x), dev(w.initial_cvstate(), "f64"), 1)
    assert e.value.status == -5
    ctx.set_reference_map(0, maps=np.full((128, P), 0.5))       # the largest stack is accepted
    ctx.step_replicas(x, torch.zeros_like(x), dev(w.initial_cvstate(), "f64"), 1)
    ctx.sync()


def test_autotune_picks_a_valid_launch_and_keeps_results(S):
    w = I.config2(n_replicas=8, n_steps=20)
    x0, v0, cv0 = w.initial_x(), w.initial_v(1), w.initial_cvstate()
    tuned = context(S, w)
    x, v, cv = dev(x0), dev(v0), dev(cv0, "f64")
    path, threads = tuned.autotune(x, v, cv, 5)
    assert (path == 0 and threads in (256, 512, 1024)) or (path == 1 and threads == 0)
    np.testing.assert_array_equal(host(x), x0)           # the state it timed on is untouched
    np.testing.assert_array_equal(host(cv), cv0)
    plain = context(S, w)
    res = []
    for ctx in (tuned, plain):
        x, v, cv = dev(x0), dev(v0), dev(cv0, "f64")
        ctx.step_replicas(x, v, cv, 20, step0=100)
        ctx.sync()
        res.append((host(x), host(cv)))
    disp = np.abs(res[1][0] - x0).max()
    assert np.abs(res[0][0] - res[1][0]).max() <= 1e-4 * disp
    np.testing.assert_allclose(res[0][1][:, :2], res[1][1][:, :2], rtol=1e-5)
    # an SCPS context has only the per-step path
    base = dict(I._base_params(), bias_mode=1)
    ws = single_system_workload(90, np.arange(90), base, 2)
    sc = context(S, ws, params=base)
    sc.update_reference_from_paths(0, dev(_ensemble_frames(ws.systems[0], 4, 2, 5).ravel()), 2, 4,
                                   np.ones(2, dtype=np.uint8))
    xs = dev(np.stack([ws.systems[0].start] * 2).astype(np.float32).ravel())
    import torch
    path_s, overlap_s = sc.autotune(xs, torch.zeros_like(xs), dev(ws.initial_cvstate(), "f64"), 2)
    assert path_s == 1 and overlap_s in (0, 1)       # per step; nonbonded pass after or beside
    # 20-bead chains: the packed kernel (3 replicas per wavefront, 1, 2, 4 or 8 wavefronts per
    # workgroup) and one wavefront per replica are also candidates, and results keep matching
    w1 = I.config1(n_replicas=64, n_steps=1)
    t1, p1 = context(S, w1), context(S, w1)
    x1 = dev(w1.initial_x())
    path, threads = t1.autotune(x1, None, dev(w1.initial_cvstate(), "f64"), 50)
    print(f"  20-bead chains: autotune picked path {path}, {threads} threads", flush=True)
    assert ((path == 0 and threads in (64, 256, 512, 1024)) or (path == 1 and threads == 0)
            or (path == 2 and threads in (3, 6, 12, 24)))
    out = []
    for ctx in (t1, p1):
        xa, cva = dev(w1.initial_x()), dev(w1.initial_cvstate(), "f64")
        ctx.step_replicas(xa, None, cva, 30)
        ctx.sync()
        out.append(host(xa))
    assert np.abs(out[0] - out[1]).max() <= 1e-4 * np.abs(out[1] - w1.initial_x()).max()


# ---------------------------------------------------------------------------
# least-biased path selection (smallest bias functional T among successful paths)
# ---------------------------------------------------------------------------
def test_least_biased_path_matches_oracle(S):
    w = I.config1(n_replicas=1000, n_steps=1)
    ctx = context(S, w)
    R = w.n_replicas
    for seed in range(5):
        rng = np.random.default_rng(700 + seed)
        cv = rng.normal(size=(R, 8))
        cv[:, 7] = np.round(rng.uniform(0, 4, R), 2)      # many exact ties
        succ = None if seed == 0 else (rng.uniform(size=R) < [0.5, 0.05, 0.9, 0.002][seed - 1]).astype(np.uint8)
        if succ is not None and not succ.any():
            succ[rng.integers(R)] = 1
        want = O.least_biased(cv, succ)
        got, t = ctx.least_biased_path(dev(cv, "f64"), succ)
        print(f"  seed {seed}: candidates {R if succ is None else int(succ.sum())}, index {got}", flush=True)
        assert got == want and t == cv[want, 7]
    # every value equal: the lowest candidate id
    cv = np.zeros((R, 8)); cv[:, 7] = 1.25
    succ = np.zeros(R, dtype=np.uint8); succ[[17, 400, 999]] = 1
    assert ctx.least_biased_path(dev(cv, "f64"), succ) == (17, 1.25)
    # errors: no candidate; a candidate with a non-finite T (a non-candidate's is ignored)
    with pytest.raises(S.ScpsError) as e:
        ctx.least_biased_path(dev(cv, "f64"), np.zeros(R, dtype=np.uint8))
    assert e.value.status == -7
    cv[5, 7] = np.nan
    with pytest.raises(S.ScpsError) as e:
        ctx.least_biased_path(dev(cv, "f64"))
    assert e.value.status == -1
    succ = np.ones(R, dtype=np.uint8); succ[5] = 0
    assert ctx.least_biased_path(dev(cv, "f64"), succ) == (0, 1.25)
    ctx.close()


def test_least_biased_after_stepping_matches_oracle(S):
    w = I.config1(n_replicas=16, n_steps=20)
    p = dict(w.params)
    ctx = context(S, w)
    x = dev(w.initial_x())
    cv = dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(x, None, cv, 20)
    ctx.sync()
    osys = O.System.from_inputs(w.systems[0], p)
    X0 = w.initial_x().reshape(16, 3, 20).astype(np.float64)
    cvo = np.stack([O.steps(p, osys, r, X0[r], None, w.initial_cvstate()[r], 20)[2] for r in range(16)])
    CVg = host(cv)
    succ = np.array([r % 4 != 1 for r in range(16)], dtype=np.uint8)
    got, t = ctx.least_biased_path(cv, succ)
    want = O.least_biased(cvo, succ)
    assert t == CVg[got, 7] and succ[got]
    T = np.where(succ > 0, cvo[:, 7], np.inf)
    order = np.argsort(T)
    print(f"  T oracle {T[order[:3]]}, GPU pick {got} (T {t:.6e}), oracle pick {want}", flush=True)
    if T[order[1]] - T[order[0]] > 1e-3 * T[order[0]]:   # a clear winner: both sides pick it
        assert got == want
    else:                                                # near tie: the pick is one of the tied paths
        assert T[got] <= T[order[0]] * (1 + 1e-3)
    ctx.close()


# ---------------------------------------------------------------------------
# cutoff variant: contact and nonbonded cutoffs; neighbour lists on the per-step path
# ---------------------------------------------------------------------------
CUT_CASES = [
    # name, n, exec_mode, r_cut_contact, r_cut_nb
    ("both12_persistent", 333, 0, 12.0, 12.0),
    ("both12_lists", 333, 1, 12.0, 12.0),
    ("both12_all_tiles", 333, 2, 12.0, 12.0),
    ("nb_only10_per_step", 257, 1, 0.0, 10.0),
    ("nb_only10_persistent", 257, 0, 0.0, 10.0),
    ("cut9_nb10_lists_1500", 1500, 1, 9.0, 10.0),
    ("cut12_nb9_lists_ragged_1100", 1100, 1, 12.0, 9.0),
]


@pytest.mark.parametrize("name,n,exec_mode,rc,rnb", CUT_CASES, ids=[c[0] for c in CUT_CASES])
def test_cutoff_forces_match_oracle(S, name, n, exec_mode, rc, rnb):
    base = dict(I._base_params(), r_cut_contact=rc, r_cut_nb=rnb)
    R = 5
    w = single_system_workload(n, np.arange(n), base, R)
    p = _force_readback_params(base, k_R=1e-2)
    sy = w.systems[0]
    X = states(sy, R, 41)
    osys = O.System.from_inputs(sy, p)
    cv0 = np.zeros((R, 8))
    cv0[:, 1] = np.inf
    for r in range(1, R):
        cv0[r, 1] = 0.8 * O.z_grad(X[r].astype(np.float64), osys.cidx, osys.native, r_cut=rc, grad=False)
    Fg, cvg = _gpu_forces_one_step(S, w, p, X, cv0, exec_mode)
    for r in range(R):
        F, Fb, cvr = O.total_force(p, osys, X[r].astype(np.float64), cv0[r])
        err = normwise(Fg[r], F)
        print(f"  {name} replica {r}: force err {err:.2e}, z {cvg[r, 0]:.6f} (oracle {cvr[0]:.6f})", flush=True)
        assert err <= TOL, (r, err)
        assert abs(cvg[r, 0] - cvr[0]) <= TOL * max(cvr[0], 1e-3 * osys.Z0)
        assert abs(cvg[r, 1] - cvr[1]) <= TOL * max(cvr[1], 1e-3 * osys.Z0)


def _list_vs_tiles(S, n, R, base, X0, n_steps, calls=1):
    import torch
    w = single_system_workload(n, np.arange(n), base, R)
    res = []
    for mode in (1, 2):
        ctx = context(S, w, params=base, exec_mode=mode)
        x = dev(X0.ravel())
        v = torch.zeros_like(x)
        cv = dev(w.initial_cvstate(), "f64")
        for c in range(calls):
            ctx.step_replicas(x, v, cv, n_steps // calls, step0=5 + c * (n_steps // calls))
        ctx.sync()
        res.append((host(x).reshape(R, 3, n), host(cv)))
        ctx.close()
    return res


def _clean_starts(sy, R, seed):
    """Random coils and the jittered extended start: no overlapping beads (a
    perturbed native can put two beads 1.7 A apart and blow a run up)."""
    rng = np.random.default_rng(seed)
    return np.stack([I.random_coil(sy.n, 300 + seed + r) if r % 2 == 0
                     else sy.start + rng.normal(0, 0.05, sy.start.shape) for r in range(R)]).astype(np.float32)


def test_list_steps_equal_all_tile_steps(S):
    """The lists hold every pair within the cutoffs, so a noisy trajectory
    agrees with the all-tiles path up to the order of the float32 sums."""
    n, R = 1400, 4
    base = dict(I._base_params(), r_cut_contact=10.0, r_cut_nb=10.0, k_R=5e-3)
    sy = single_system_workload(n, np.arange(n), base, R).systems[0]
    X0 = _clean_starts(sy, R, 7)
    res = _list_vs_tiles(S, n, R, base, X0, 30)
    disp = np.abs(res[1][0] - X0).max()
    d = np.abs(res[0][0] - res[1][0]).max()
    print(f"  lists vs all tiles after 30 steps: max |dx| {d:.2e} (displacement {disp:.2e})", flush=True)
    assert d <= 1e-4 * disp + 1e-4
    np.testing.assert_allclose(res[0][1][:, :2], res[1][1][:, :2], rtol=1e-7)
    # E_b = k_R (z - z_m)^2 / 2 takes a small difference of two large z values
    np.testing.assert_allclose(res[0][1][:, 2], res[1][1][:, 2], rtol=1e-4, atol=1e-7)
    np.testing.assert_allclose(res[0][1][:, 7], res[1][1][:, 7], rtol=1e-4)


def test_lists_are_rebuilt_as_particles_move(S):
    """A hot run (kT x 6) moves particles by several list skins within a call
    and between calls: the list path still follows the all-tiles path."""
    n, R = 900, 4
    base = dict(I._base_params(), r_cut_contact=9.0, r_cut_nb=9.0, k_R=5e-3)
    base["kT"] *= 6.0
    sy = single_system_workload(n, np.arange(n), base, R).systems[0]
    X0 = _clean_starts(sy, R, 11)
    res = _list_vs_tiles(S, n, R, base, X0, 150, calls=3)
    disp = np.abs(res[1][0] - X0).max()
    d = np.abs(res[0][0] - res[1][0]).max()
    print(f"  hot run, 150 steps in 3 calls: max displacement {disp:.2f} A, lists vs all tiles {d:.2e}", flush=True)
    assert disp > 2.0                                        # a rebuild at every 0.75 A: several were needed
    assert d <= 1e-3 * disp
    np.testing.assert_allclose(res[0][1][:, :2], res[1][1][:, :2], rtol=1e-4)


def test_list_overflow_is_reported(S):
    """600 beads inside a 4 A ball (no pair forces): every list would need 599
    entries, more than the capacity; the step reports it instead of dropping pairs."""
    import torch
    n = 600
    base = dict(I._base_params(), r_cut_contact=12.0, r_cut_nb=12.0, lj_eps=0.0, dh_prefactor=0.0, k_bond=0.0)
    w = single_system_workload(n, np.arange(n), base, 1)
    ctx = context(S, w, params=base, exec_mode=1)
    rng = np.random.default_rng(3)
    u = rng.normal(size=(3, n))
    X = (4.0 * u / np.linalg.norm(u, axis=0) * rng.uniform(0, 1, n) ** (1 / 3)).astype(np.float32)
    x = dev(X.ravel())
    with pytest.raises(S.ScpsError) as e:
        ctx.step_replicas(x, torch.zeros_like(x), dev(w.initial_cvstate(), "f64"), 1)
        ctx.sync()
    assert e.value.status == -6 and "neighbours" in str(e.value)


def test_lists_follow_positions_changed_between_calls(S):
    """The caller replaces every position between two calls on one context:
    the displacement test rebuilds the lists, and the second call matches a
    fresh all-tiles context started from the new positions."""
    import torch
    n, R = 800, 3
    base = dict(I._base_params(), r_cut_contact=10.0, r_cut_nb=10.0, k_R=5e-3)
    w = single_system_workload(n, np.arange(n), base, R)
    sy = w.systems[0]
    XA, XB = _clean_starts(sy, R, 21), _clean_starts(sy, R, 22)[::-1].copy()
    ctx = context(S, w, params=base, exec_mode=1)
    x = dev(XA.ravel())
    v = torch.zeros_like(x)
    cv = dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(x, v, cv, 10)
    x.copy_(dev(XB.ravel()))
    v.zero_()
    cv.copy_(dev(w.initial_cvstate(), "f64"))
    ctx.step_replicas(x, v, cv, 10, step0=40)
    ctx.sync()
    ref = context(S, w, params=base, exec_mode=2)
    x2, v2, cv2 = dev(XB.ravel()), torch.zeros_like(x), dev(w.initial_cvstate(), "f64")
    ref.step_replicas(x2, v2, cv2, 10, step0=40)
    ref.sync()
    disp = np.abs(host(x2) - XB.ravel()).max()
    d = np.abs(host(x) - host(x2)).max()
    print(f"  new positions between calls: lists vs all tiles {d:.2e} (displacement {disp:.2e})", flush=True)
    assert d <= 1e-4 * disp + 1e-4
    np.testing.assert_allclose(host(cv)[:, :2], host(cv2)[:, :2], rtol=1e-7)
    ctx.close()
    ref.close()


# ---------------------------------------------------------------------------
# tube variables against any stack, and the global coordinate sigma(X)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode,w_form", [(0, 0), (1, 0), (1, 1)],
                         ids=["rmd_context", "scps_context", "scps_context_w_without_1_over_lambda"])
def test_eval_tube_and_sigma_match_oracle(S, mode, w_form):
    """Three initial conditions of one chain (three systems, each with the
    stack of its own paths); every replica is measured against every stack,
    and sigma is the mean of 1 - s over them."""
    import torch
    n, K, n_paths, R = 170, 11, 3, 7
    base = dict(I._base_params(), bias_mode=mode, lam=13.5, k_s=2.5, k_w=2.5e-4, w_form=w_form)
    rng = np.random.default_rng(4)
    proto = I.System(n=n, contact_idx=np.arange(n, dtype=np.int32), mass=np.full(n, 12.011 * I.AMU, np.float32),
                     charge=rng.normal(0, 0.3, n).astype(np.float32), native=I.compact_native(n, 4),
                     start=I.persistent_start(n, 5))
    systems, stacks, frames = [], [], []
    for k in range(3):
        sy = I.System(n=n, contact_idx=proto.contact_idx, mass=proto.mass, charge=proto.charge,
                      native=proto.native, start=I.persistent_start(n, 40 + k))
        fr = _ensemble_frames(sy, K, n_paths, 60 + k)
        st, _ = O.update_reference(n, sy.contact_idx, fr.astype(np.float64), np.ones(n_paths, np.uint8), 7.5, 0.0)
        systems.append(sy)
        stacks.append(st)
        frames.append(fr)
    rsys = np.arange(R, dtype=np.int32) % 3
    w = I.Workload("three_ics", dict(base), systems, rsys, 1)
    ctx = context(S, w, params=base)
    for k in range(3):
        ctx.set_reference_map(k, maps=stacks[k])
    X = np.stack([frames[(r + 1) % 3][(2 * r) % K, r % n_paths] + rng.normal(0, 0.3, (3, n))
                  for r in range(R)]).astype(np.float32)
    x = dev(X.ravel())
    Z0 = O.System.from_inputs(proto, base).Z0
    for b in range(3):
        s = torch.zeros(R, dtype=torch.float64, device="cuda")
        wv = torch.zeros_like(s)
        ctx.eval_tube(b, x, s, wv)
        ctx.sync()
        for r in range(R):
            so, wo, *_ = O.tube(X[r].astype(np.float64), proto.contact_idx, stacks[b], Z0, 13.5, grads=False,
                                w_form=w_form)
            print(f"  stack {b} replica {r}: s {host(s)[r]:.6f} (oracle {so:.6f}), w {host(wv)[r]:.6f} "
                  f"(oracle {wo:.6f})", flush=True)
            assert abs(host(s)[r] - so) <= 1e-5 and abs(host(wv)[r] - wo) <= 1e-5 * max(1.0, abs(wo))
    for sel in ([0, 1, 2], [2], [1, 1, 0]):
        sg = torch.zeros(R, dtype=torch.float64, device="cuda")
        ctx.eval_sigma(sel, x, sg)
        ctx.sync()
        want = [O.sigma(X[r].astype(np.float64), proto.contact_idx, [stacks[b] for b in sel], [Z0] * len(sel), 13.5)
                for r in range(R)]
        np.testing.assert_allclose(host(sg), want, rtol=0, atol=1e-5)
    ctx.close()


def test_eval_tube_rejects_other_chains_and_missing_stacks(S):
    import torch
    base = dict(I._base_params(), lam=13.5)
    sys_a = single_system_workload(120, np.arange(120), base, 1).systems[0]
    sys_b = single_system_workload(121, np.arange(121), base, 1).systems[0]
    w = I.Workload("mixed", dict(base), [sys_a, sys_b], np.array([0, 1], dtype=np.int32), 1)
    ctx = context(S, w, params=base)
    fr = _ensemble_frames(sys_a, 4, 2, 3)
    ctx.update_reference_from_paths(0, dev(fr.ravel()), 2, 4, np.ones(2, dtype=np.uint8))
    x = dev(np.concatenate([sys_a.start.ravel(), sys_b.start.ravel()]).astype(np.float32))
    s = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(S.ScpsError) as e:
        ctx.eval_tube(0, x, s)                   # replica 1 runs a 121-particle chain
    assert e.value.status == -2
    with pytest.raises(S.ScpsError) as e:
        ctx.eval_tube(1, x, s)                   # system 1 has no frame stack
    assert e.value.status == -5
    ctx.close()


# ---------------------------------------------------------------------------
# convergence measure between iterations
# ---------------------------------------------------------------------------
def test_path_distance_matches_oracle(S):
    import torch
    grid = dict(x0=0.0, y0=0.0, cell=0.8, nx=20, ny=20)
    for seed in range(4):
        rng = np.random.default_rng(90 + seed)
        a = rng.normal(8.0, 2.5, size=(20000, 2)).astype(np.float32)
        b = rng.normal(8.0 + 0.3 * seed, 2.0 + 0.4 * seed, size=(15000 + 1000 * seed, 2)).astype(np.float32)
        a[:50] = 0.8 * rng.integers(0, 20, size=(50, 2))        # points on cell edges
        want = O.path_distance(a, b, **grid)
        got = S.path_distance(dev(a), dev(b), **grid)
        print(f"  seed {seed}: D {got:.12f} (oracle {want:.12f})", flush=True)
        assert got == pytest.approx(want, rel=1e-14, abs=1e-15)
    assert S.path_distance(dev(a), dev(a), **grid) == 0.0
    with pytest.raises(S.ScpsError) as e:                      # no point inside the grid
        S.path_distance(dev(a), dev(np.full((3, 2), -5.0, np.float32)), **grid)
    assert e.value.status == -1


def test_lists_with_uneven_systems_and_partial_contact_sets(S):
    """Lists over replicas of two chains of different lengths (ragged blocks),
    one with every third particle in the contact set and min_seq_sep 4: one
    step against the oracle, and 20 noisy steps against the all-tiles path."""
    import torch
    base = dict(I._base_params(), r_cut_contact=11.0, r_cut_nb=9.5, min_seq_sep=4)
    rng = np.random.default_rng(8)
    systems = []
    for n, kind, seed in ((301, "all", 21), (1100, "every3", 22)):
        systems.append(I.System(n=n, contact_idx=np.asarray(_cidx(n, kind), dtype=np.int32),
                                mass=np.full(n, 12.011 * I.AMU, dtype=np.float32),
                                charge=rng.normal(0, 0.3, n).astype(np.float32), native=I.compact_native(n, seed),
                                start=I.persistent_start(n, seed + 1)))
    rsys = np.array([0, 1, 1, 0, 1], dtype=np.int32)
    R = len(rsys)
    X = [_clean_starts(systems[s], 1, 30 + r)[0] for r, s in enumerate(rsys)]
    p = _force_readback_params(base, k_R=1e-2)
    w = I.Workload("two_chains_cut", dict(p), systems, rsys, 1)
    osys = [O.System.from_inputs(sy, p) for sy in systems]
    cv0 = np.zeros((R, 8))
    cv0[:, 1] = np.inf
    for r in range(1, R):
        o = osys[rsys[r]]
        cv0[r, 1] = 0.8 * O.z_grad(X[r].astype(np.float64), o.cidx, o.native, r_cut=11.0, min_sep=4, grad=False)
    Fg, cvg = _gpu_forces_one_step(S, w, p, X, cv0, 1)
    for r in range(R):
        F, _, cvr = O.total_force(p, osys[rsys[r]], X[r].astype(np.float64), cv0[r])
        err = normwise(Fg[r], F)
        print(f"  replica {r} (N = {systems[rsys[r]].n}): force err {err:.2e}", flush=True)
        assert err <= TOL, (r, err)
        assert abs(cvg[r, 0] - cvr[0]) <= TOL * max(cvr[0], 1e-3 * osys[rsys[r]].Z0)
    # noisy steps: lists against all tiles
    wn = I.Workload("two_chains_cut", dict(base, k_R=5e-3), systems, rsys, 1)
    xflat = np.concatenate([x.ravel() for x in X])
    res = []
    for mode in (1, 2):
        ctx = context(S, wn, params=dict(base, k_R=5e-3), exec_mode=mode)
        x = dev(xflat)
        v = torch.zeros_like(x)
        cv = dev(wn.initial_cvstate(), "f64")
        ctx.step_replicas(x, v, cv, 20)
        ctx.sync()
        res.append((host(x), host(cv)))
        ctx.close()
    disp = np.abs(res[1][0] - xflat).max()
    d = np.abs(res[0][0] - res[1][0]).max()
    print(f"  20 steps: lists vs all tiles {d:.2e} (displacement {disp:.2e})", flush=True)
    assert d <= 1e-4 * disp + 1e-4
    np.testing.assert_allclose(res[0][1][:, :2], res[1][1][:, :2], rtol=1e-7)


# ---------------------------------------------------------------------------
# equipartition at the bath temperature (no bias)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("exec_mode", [0, 1], ids=["persistent", "per_step"])
def test_equipartition_at_bath_temperature(S, exec_mode):
    """k_R = 0: after 3000 BAOAB steps (6 ps from the extended start, several
    friction times) the mean of m v^2 per degree of freedom over 256 x 560
    particles, sampled every 50 steps for 1000 more, equals kT within 1 %
    (one snapshot's statistical error is ~0.2 %; BAOAB's kinetic-temperature
    error at dt = 2 fs stays well below that over all modes)."""
    import torch
    w = I.config2(n_replicas=256, n_steps=1)
    p = dict(w.params, k_R=0.0)
    ctx = context(S, w, params=p, exec_mode=exec_mode)
    x = dev(w.initial_x())
    v = dev(w.initial_v(3))
    cv = dev(w.initial_cvstate(), "f64")
    ctx.step_replicas(x, v, cv, 3000)
    m = np.tile(w.systems[0].mass.astype(np.float64), 3 * 256)   # [R][3][n] layout, mass per particle
    ratios = []
    for k in range(20):
        ctx.step_replicas(x, v, cv, 50, step0=3000 + 50 * k)
        ctx.sync()
        ratios.append(np.mean(m * host(v).astype(np.float64) ** 2) / p["kT"])
    r = float(np.mean(ratios))
    print(f"  <m v^2> / kT = {r:.4f} (snapshots {np.min(ratios):.4f} .. {np.max(ratios):.4f})", flush=True)
    assert abs(r - 1.0) < 0.01
    ctx.close()
