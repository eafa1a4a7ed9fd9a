"""The packed persistent kernel: chains of at most 64 particles, floor(64 / n)
replicas per wavefront (one for 33 .. 64), 1 .. 8 wavefronts per workgroup,
all steps of a call in one launch.  Forces, z and the bias functional of one
step against the FP64 oracle (chains of 2 .. 64 particles,
ragged replica counts, two systems of different lengths in one wavefront,
sequence separation and cutoffs), the Philox noise stream, short noisy
trajectories and recorded frames against the one-replica-per-workgroup
kernel and the per-step path, and the launch-configuration calls."""
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


def normwise(a, b):
    d = np.linalg.norm((a - b).reshape(3, -1), axis=0).max()
    return d / max(np.linalg.norm(b.reshape(3, -1), axis=0).max(), 1e-300)


def _system(n, contact, seed):
    rng = np.random.default_rng(seed)
    cidx = {"all": np.arange(n), "half": np.arange(0, n, 2), "tail": np.arange(n // 3, n)}[contact]
    return I.System(n=n, contact_idx=np.asarray(cidx, dtype=np.int32),
                    mass=rng.uniform(1.0, 16.0, n).astype(np.float32) * np.float32(I.AMU),
                    charge=rng.normal(0, 0.3, n).astype(np.float32),
                    native=I.compact_native(n, seed), start=I.persistent_start(n, seed + 1))


def _coil_or_native(sy, r, seed):
    rng = np.random.default_rng(seed + r)
    if r % 2 == 0:
        return I.random_coil(sy.n, seed + 50 + r).astype(np.float32)
    return (sy.native + rng.normal(0, 0.4, sy.native.shape)).astype(np.float32)


def _context(S, w, params, launch=None, exec_mode=0):
    ctx = S.Context.from_workload(w, params=params, exec_mode=exec_mode)
    for s, sy in enumerate(w.systems):
        ctx.set_reference_map(s, native_xyz=sy.native)
    if launch is not None:
        ctx.set_launch(*launch)
    return ctx


# name, chain lengths, contact set, replicas, replica -> system pattern, parameter overrides
CASES = [
    ("two_particles", [2], "all", 5, None, {}),
    ("chain7_nine_per_wave", [7], "all", 12, None, {}),
    ("chain20_three_per_wave", [20], "all", 16, None, {}),
    ("chain32_two_per_wave_half_contacts", [32], "half", 11, None, {}),
    ("lengths_13_and_20_in_one_wave", [13, 20], "all", 10, [0, 1, 1, 0, 1, 0, 0, 1, 1, 0], {}),
    ("seqsep_and_cutoffs", [24], "tail", 7, None,
     {"min_seq_sep": 3, "r_cut_contact": 9.0, "r_cut_nb": 10.0}),
    ("bias_only", [20], "all", 6, None, {"k_bond": 0.0, "lj_eps": 0.0, "dh_prefactor": 0.0, "k_R": 0.5}),
    ("chain48_one_per_wave", [48], "half", 5, None, {}),
    ("chain64_full_wave_with_33", [64, 33], "all", 9, [0, 1, 0, 1, 1, 0, 0, 1, 0], {}),
]


@pytest.mark.parametrize("waves", [1, 8], ids=["1_wave", "8_waves"])
@pytest.mark.parametrize("name,sizes,contact,R,rsys,extra", CASES, ids=[c[0] for c in CASES])
def test_packed_step_forces_match_oracle(S, name, sizes, contact, R, rsys, extra, waves):
    """One BAOAB step from rest at kT = 0 reads back the total force (v =
    c1 dt F / m): normwise within 1e-5 of the oracle for every replica, with
    z, z_m, E_b and the bias functional T; half the replicas start below
    their running minimum (biased), one starts it."""
    import torch
    base = dict(I._base_params(), integrator=1, kT=0.0, gamma=1e-3, dt=0.002, k_R=2e-2)
    base.update(extra)
    systems = [_system(n, contact, 40 + 7 * i) for i, n in enumerate(sizes)]
    rs = np.asarray(rsys if rsys is not None else [0] * R, dtype=np.int32)
    w = I.Workload(name, dict(base), systems, rs, 1)
    X = [_coil_or_native(systems[rs[r]], r, 90) for r in range(R)]
    osys = [O.System.from_inputs(sy, base) for sy in systems]
    cv0 = np.zeros((R, 8))
    cv0[:, 1] = np.inf
    for r in range(1, R):
        o = osys[rs[r]]
        z = O.z_grad(X[r].astype(np.float64), o.cidx, o.native, grad=False)
        cv0[r, 1] = 0.7 * z if r % 2 else 1.3 * z
    ctx = _context(S, w, base, launch=(2, waves))
    x = dev(np.concatenate([a.ravel() for a in X]))
    v = torch.zeros_like(x)
    cv = dev(cv0, "f64")
    ctx.step_replicas(x, v, cv, 1, step0=3)
    ctx.sync()
    ctx.close()
    V, CV = host(v), host(cv)
    c1 = math.exp(-base["gamma"] * base["dt"])
    off = 0
    for r in range(R):
        sy, o = systems[rs[r]], osys[rs[r]]
        n = sy.n
        Fg = V[3 * off:3 * (off + n)].reshape(3, n).astype(np.float64) * sy.mass.astype(np.float64) / (c1 * base["dt"])
        off += n
        F, _, cvr = O.total_force(base, o, X[r].astype(np.float64), cv0[r])
        assert normwise(Fg, F) <= TOL, (r, normwise(Fg, F))
        zs = max(cvr[0], 1e-3 * max(o.Z0, 1e-300))
        assert abs(CV[r, 0] - cvr[0]) <= TOL * zs + 1e-12, (r, CV[r, 0], cvr[0])
        assert abs(CV[r, 1] - cvr[1]) <= TOL * max(cvr[1], 1e-3 * max(o.Z0, 1e-300)) + 1e-12
        assert abs(CV[r, 2] - cvr[2]) <= 1e-4 * max(cvr[2], 1e-12) + 1e-12
        # bias functional T = dt sum_i |F_bias,i|^2 / (m_i gamma): sqrt(T) is a weighted
        # norm of the bias force, so a force error below TOL max|F| moves it by at most
        # TOL max|F| sqrt(dt sum_i 1 / (m_i gamma)) (near the native map the bias force is
        # a cancelling C - R far below the chain forces, so T has no relative bound)
        _, _, cvs, _ = O.steps(base, o, r, X[r].astype(np.float64), np.zeros(X[r].shape), cv0[r], 1, step0=3)
        fmax = np.linalg.norm(F, axis=0).max()
        tol_t = TOL * fmax * math.sqrt(base["dt"] * np.sum(1.0 / (sy.mass.astype(np.float64) * base["gamma"])))
        assert abs(math.sqrt(CV[r, 7]) - math.sqrt(cvs[7])) <= tol_t, (r, CV[r, 7], cvs[7])
        if r % 2 == 0:                    # at or above the running minimum: no bias at all
            assert cvs[7] == 0.0 and CV[r, 7] == 0.0


def test_packed_noise_matches_oracle_philox(S):
    """Free overdamped particles with unit noise amplitude (x1 = x0 + xi):
    every particle of every replica draws the oracle's Philox normals for
    (chain index, replica_base + r, step), here with a 64-bit step."""
    import torch
    n, R = 30, 7
    p = dict(I._base_params(), integrator=0, dt=1.0, gamma=1.0, kT=0.5, k_bond=0.0, lj_eps=0.0,
             dh_prefactor=0.0, k_R=0.0, seed=0x1234_5678_9ABC)
    sy = _system(n, "half", 3)
    sy.mass[:] = 1.0
    w = I.Workload("noise", dict(p), [sy], np.zeros(R, dtype=np.int32), 1)
    ctx = S.Context.from_workload(w, params=p, replica_base=7)
    ctx.set_reference_map(0, native_xyz=sy.native)
    ctx.set_launch(2, 4)
    x = torch.zeros(3 * n * R, dtype=torch.float32, device="cuda")
    cv = dev(np.tile([0, np.inf, 0, 0, 0, np.inf, np.inf, 0], (R, 1)), "f64")
    step = (1 << 32) + 5
    ctx.step_replicas(x, None, cv, 1, step0=step)
    got = host(x).reshape(R, 3, n)
    ctx.close()
    for r in range(R):
        want = O.normals(p["seed"], np.arange(n), 7 + r, step).T
        np.testing.assert_allclose(got[r], want, rtol=1e-6, atol=1e-6)


def _run(S, w, p, launch, exec_mode, x0, v0, n_steps, record_every=0):
    import torch
    ctx = _context(S, w, p, launch=launch, exec_mode=exec_mode)
    x = dev(x0)
    v = dev(v0) if v0 is not None else None
    cv = dev(w.initial_cvstate(), "f64")
    frames = None
    if record_every:
        frames = torch.zeros((n_steps // record_every + 1) * x0.size, dtype=torch.float32, device="cuda")
    ctx.step_replicas(x, v, cv, n_steps, step0=17, record_every=record_every, frames=frames)
    ctx.sync()
    ctx.close()
    return host(x), (host(v) if v is not None else None), host(cv), (host(frames) if record_every else None)


@pytest.mark.parametrize("integrator", [0, 1], ids=["overdamped", "baoab"])
def test_packed_trajectories_agree_with_other_launches(S, integrator):
    """37 replicas of the 20-bead chain (a ragged last workgroup), 20 noisy
    steps with frames every 5: the packed kernel (1, 2, 4, 8 wavefronts per
    workgroup), the persistent kernel with one wavefront per replica and the
    per-step path agree up to the float32 summation order of the forces,
    and frame 0 is the start exactly."""
    R = 37
    w = I.config1(n_replicas=R, n_steps=20)
    p = dict(w.params)
    v0 = None
    if integrator == 1:
        p.update(integrator=1, dt=0.002, gamma=1.0, kT=2.494, k_bond=100.0)
        v0 = w.initial_v(5)
    x0 = w.initial_x()
    ref = _run(S, w, p, (0, 64), 0, x0, v0, 20, 5)
    disp = np.abs(ref[0] - x0).max()
    assert disp > 0
    others = [((2, k), 0) for k in (1, 2, 4, 8)] + [(None, 1)]
    for launch, mode in others:
        got = _run(S, w, p, launch, mode, x0, v0, 20, 5)
        assert np.abs(got[0] - ref[0]).max() <= 1e-4 * disp, (launch, np.abs(got[0] - ref[0]).max(), disp)
        np.testing.assert_allclose(got[2][:, :2], ref[2][:, :2], rtol=1e-4, atol=1e-12)
        # E_b = k_R (z - z_m)^2 / 2: compare z - z_m, a difference of two z-sized numbers
        dz_got, dz_ref = (np.sqrt(2.0 * c[:, 2] / p["k_R"]) for c in (got[2], ref[2]))
        assert np.abs(dz_got - dz_ref).max() <= 1e-4 * ref[2][:, 0].max()
        assert np.array_equal(got[3][:x0.size], x0)
        assert np.abs(got[3] - ref[3]).max() <= 1e-4 * disp
        if integrator == 1:
            assert np.abs(got[1] - ref[1]).max() <= 1e-4 * np.abs(ref[1]).max()


def test_packed_is_the_default_for_short_chains_and_autotune_keeps_results(S):
    """An untuned context runs 20-particle chains packed; the
    autotuner's choice (any of the packed, persistent and per-step
    configurations) gives the same trajectory up to summation order, and
    the caller's state is untouched by the trial runs."""
    R = 48
    w = I.config1(n_replicas=R, n_steps=10)
    p = dict(w.params)
    x0 = w.initial_x()
    untuned = _run(S, w, p, None, 0, x0, None, 10)
    packed = _run(S, w, p, (2, 4), 0, x0, None, 10)
    assert np.array_equal(untuned[0], packed[0]) and np.array_equal(untuned[2], packed[2])
    ctx = _context(S, w, p)
    x, cv = dev(x0), dev(w.initial_cvstate(), "f64")
    path, param = ctx.autotune(x, None, cv, 5)
    print(f"  autotune on 48 x 20 beads: path {path}, parameter {param}", flush=True)
    assert path in (0, 1, 2)
    if path == 2:
        assert param in (3, 6, 12, 24)             # 3 replicas per wavefront x 1, 2, 4, 8 wavefronts
    assert np.array_equal(host(x), x0)
    ctx.step_replicas(x, None, cv, 10, step0=17)
    ctx.sync()
    ctx.close()
    disp = np.abs(untuned[0] - x0).max()
    assert np.abs(host(x) - untuned[0]).max() <= 1e-4 * disp


def test_untuned_launch_defaults(S):
    """get_launch reports what step_replicas takes: untuned, chains of at most
    48 particles run packed (four wavefronts per workgroup, floor(64/n)
    replicas each), 49 .. 64 from 2048 replicas up; longer chains, or smaller
    batches, take the persistent kernel, with 256 threads per replica below
    512 replicas of a chain of at most 128 particles; set_launch, other exec
    modes and SCPS contexts are reported as they run.  A 40-particle untuned
    run is the packed launch bit for bit."""
    base = dict(I._base_params())
    for n, R, want in ((20, 48, (2, 12)), (33, 16, (2, 4)), (48, 5, (2, 4)), (49, 16, (0, 256)),
                       (64, 600, (0, 64)), (64, 2048, (2, 4)), (65, 16, (0, 256)), (128, 511, (0, 256)),
                       (128, 512, (0, 64))):
        w = I.Workload("d", dict(base), [_system(n, "all", 3)], np.zeros(R, dtype=np.int32), 1)
        ctx = _context(S, w, base)
        assert ctx.get_launch() == want, (n, R)
        if n == 20:
            for launch, got in (((0, 512), (0, 512)), ((1, 0), (1, 0)), ((2, 1), (2, 3))):
                ctx.set_launch(*launch)
                assert ctx.get_launch() == got, launch
        ctx.close()
    wl = I.config2(n_replicas=2, n_steps=1)                   # 560 particles: 45 tiles, 1024 threads
    ctx = _context(S, wl, dict(wl.params))
    assert ctx.get_launch() == (0, 1024)
    ctx.close()
    w = I.Workload("d", dict(base), [_system(20, "all", 3)], np.zeros(4, dtype=np.int32), 1)
    ctx = _context(S, w, base, exec_mode=1)
    assert ctx.get_launch() == (1, 0)
    ctx.close()
    w = I.Workload("d", dict(base), [_system(40, "all", 4)], np.zeros(8, dtype=np.int32), 1)
    x0 = w.initial_x()
    untuned = _run(S, w, base, None, 0, x0, np.zeros_like(x0), 10)
    packed = _run(S, w, base, (2, 4), 0, x0, np.zeros_like(x0), 10)
    assert np.array_equal(untuned[0], packed[0]) and np.array_equal(untuned[2], packed[2])


def test_set_launch_validation(S):
    """set_launch accepts the configurations that fit and rejects the rest."""
    w = I.config1(n_replicas=4, n_steps=1)
    ctx = _context(S, w, dict(w.params))
    for path, param in ((2, 1), (2, 8), (0, 64), (0, 256), (1, 0)):
        ctx.set_launch(path, param)
    for path, param, status in ((2, 0, -1), (2, 9, -1), (0, 100, -1), (3, 0, -1)):
        with pytest.raises(S.ScpsError) as e:
            ctx.set_launch(path, param)
        assert e.value.status == status, (path, param)
    ctx.close()
    wl = I.config2(n_replicas=2, n_steps=1)                  # 560 particles: no packed launch
    ctx = _context(S, wl, dict(wl.params))
    with pytest.raises(S.ScpsError) as e:
        ctx.set_launch(2, 4)
    assert e.value.status == -2
    ctx.close()
    base = dict(I._base_params())
    for n, ok in ((64, True), (65, False)):                  # one replica per wavefront at most 64 lanes
        wn = I.Workload("edge", dict(base), [_system(n, "all", 5)], np.zeros(2, dtype=np.int32), 1)
        ctx = _context(S, wn, base)
        if ok:
            ctx.set_launch(2, 8)
        else:
            with pytest.raises(S.ScpsError) as e:
                ctx.set_launch(2, 1)
            assert e.value.status == -2
        ctx.close()
    ctx = _context(S, w, dict(w.params), exec_mode=1)       # a fixed exec mode
    with pytest.raises(S.ScpsError) as e:
        ctx.set_launch(2, 4)
    assert e.value.status == -5
    ctx.close()
