"""Captured step blocks on the per-step path: whole blocks of graph_steps
steps replay one HIP graph of their kernel launches (the update reads the
block's first step from device memory).  The replays draw the same noise as
the steps launched one by one (bit for bit on free particles), step SCPS and
rMD replicas as the launch-by-launch path does (up to the order of the
float64 atomic sums, as two launch-by-launch runs differ) over several calls
in a row with recorded frames and other GPU work between them, are captured
again for a new cvstate buffer, and the block length is validated."""
import numpy as np
import pytest

from paper_1705_02180_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def _system(n, cidx, seed):
    rng = np.random.default_rng(seed)
    return I.System(n=n, contact_idx=np.asarray(cidx, dtype=np.int32), mass=np.full(n, 12.011 * I.AMU, np.float32),
                    charge=rng.normal(0, 0.3, n).astype(np.float32), native=I.compact_native(n, seed),
                    start=I.persistent_start(n, seed + 1))


def _context(S, w, params, exec_mode, graph_steps):
    ctx = S.Context.from_workload(w, params=params, exec_mode=exec_mode)
    for s, sy in enumerate(w.systems):
        ctx.set_reference_map(s, native_xyz=sy.native)
    ctx.set_graph_steps(graph_steps)
    return ctx


def _starts(sy, R, seed):
    rng = np.random.default_rng(seed)
    return np.stack([I.random_coil(sy.n, 400 + seed + r) if r % 2 == 0
                     else sy.start + rng.normal(0, 0.05, sy.start.shape) for r in range(R)]).astype(np.float32)


def test_replayed_noise_is_the_launched_noise(S):
    """Free particles (no force terms): every step adds the noise of its
    step index alone, so blocks replayed from the graph and steps launched
    one by one must agree bit for bit, across two calls (40 steps: two
    blocks and an 8-step tail; then 37 more from a step past 2^32)."""
    n, R = 150, 5
    p = dict(I._base_params(), integrator=0, dt=1.0, gamma=1.0, kT=0.5, k_bond=0.0, lj_eps=0.0,
             dh_prefactor=0.0, k_R=0.0, seed=0x5EED_0F_6A)
    sy = _system(n, np.arange(0, n, 2), 3)
    sy.mass[:] = 1.0
    w = I.Workload("free", dict(p), [sy], np.zeros(R, dtype=np.int32), 1)
    out = []
    for gs in (0, 16):
        ctx = _context(S, w, p, 1, gs)
        x = dev(np.zeros(3 * n * R, np.float32))
        cv = dev(np.tile([0, np.inf, 0, 0, 0, np.inf, np.inf, 0], (R, 1)), "f64")
        step = (1 << 32) - 20
        ctx.step_replicas(x, None, cv, 40, step0=step)
        ctx.step_replicas(x, None, cv, 37, step0=step + 40)
        ctx.sync()
        out.append(host(x))
        ctx.close()
    assert np.abs(out[0]).max() > 0
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("exec_mode", [0, 3], ids=["sequential", "overlapped"])
def test_scps_blocks_match_launch_by_launch(S, exec_mode):
    """SCPS replicas under the tube ratchets (150 beads, every second in the
    contact set, 6 replicas, 9 frames): 48 steps recording a frame every 20
    (a replayed block and 4 launched steps before each recorded frame),
    other GPU work and a host synchronisation, 37 more steps (two blocks and
    a tail), then 16 steps on a copy of cvstate (a new capture).  Positions, velocities, recorded frames, s, w, their
    minima and T agree with the launch-by-launch run, with the nonbonded pass
    after the bias pass and beside the distance pass on the context's second
    stream (captured as two branches of the graph)."""
    import torch
    base = dict(I._base_params(), bias_mode=1, lam=13.5, k_s=50.0, k_w=5.0)
    n, R, K, n_paths = 150, 6, 9, 2
    sy = _system(n, np.arange(0, n, 2), 31)
    w = I.Workload("scps150", dict(base), [sy], np.zeros(R, dtype=np.int32), 1)
    rng = np.random.default_rng(32)
    fr = np.empty((K, n_paths, 3, n), dtype=np.float32)
    for k in range(K):
        t = k / (K - 1)
        for q in range(n_paths):
            fr[k, q] = (1 - t) * sy.start + t * sy.native + rng.normal(0, 0.8, (3, n))
    x0 = _starts(sy, R, 33).ravel()
    cv0 = np.zeros((R, 8))
    cv0[:, 5:7] = np.inf
    out = []
    for gs in (0, 16):
        ctx = _context(S, w, base, exec_mode, gs)
        ctx.update_reference_from_paths(0, dev(fr.ravel()), n_paths, K, np.ones(n_paths, dtype=np.uint8))
        x, v, cv = dev(x0), dev(np.zeros_like(x0)), dev(cv0, "f64")
        frames = torch.zeros(3 * x0.size, dtype=torch.float32, device="cuda")
        ctx.step_replicas(x, v, cv, 48, step0=5, record_every=20, frames=frames)
        junk = (x * 2.0 + 1.0).sum()                      # other work on the stream between the calls
        ctx.sync()
        assert torch.isfinite(junk)
        ctx.step_replicas(x, v, cv, 37, step0=53)
        cv2 = cv.clone()
        ctx.step_replicas(x, v, cv2, 16, step0=90)
        ctx.sync()
        out.append((host(x), host(v), host(cv2), host(frames)))
        ctx.close()
    (xa, va, cva, fa), (xb, vb, cvb, fb) = out
    assert np.isfinite(xa).all() and np.isfinite(xb).all()
    disp = np.abs(xa - x0).max()
    assert disp > 0
    assert np.abs(xa - xb).max() <= 1e-4 * disp, (np.abs(xa - xb).max(), disp)
    assert np.abs(va - vb).max() <= 1e-4 * np.abs(va).max()
    assert np.array_equal(fa[:x0.size], x0) and np.array_equal(fb[:x0.size], x0)
    assert np.abs(fa - fb).max() <= 1e-4 * disp
    np.testing.assert_allclose(cva[:, 3:7], cvb[:, 3:7], rtol=0, atol=1e-6)
    assert (cva[:, 7] > 0).any()                          # the tube ratchets acted
    np.testing.assert_allclose(cva[:, 7], cvb[:, 7], rtol=1e-4, atol=1e-12 * cva[:, 7].max())


def test_rmd_per_step_blocks_match_launch_by_launch(S):
    """rMD on the per-step path (exec mode 1, 200 beads, 4 replicas, ratchet
    on z): 40 noisy BAOAB steps in blocks of 8 (five replays) against the
    launch-by-launch run."""
    p = dict(I._base_params(), k_R=5e-3)
    n, R = 200, 4
    sy = _system(n, np.arange(n), 41)
    w = I.Workload("rmd200", dict(p), [sy], np.zeros(R, dtype=np.int32), 1)
    x0 = _starts(sy, R, 42).ravel()
    cv0 = np.tile([0, np.inf, 0, 0, 0, np.inf, np.inf, 0], (R, 1))
    out = []
    for gs in (0, 8):
        ctx = _context(S, w, p, 1, gs)
        x, v, cv = dev(x0), dev(np.zeros_like(x0)), dev(cv0, "f64")
        ctx.step_replicas(x, v, cv, 40, step0=11)
        ctx.sync()
        out.append((host(x), host(cv)))
        ctx.close()
    (xa, cva), (xb, cvb) = out
    disp = np.abs(xa - x0).max()
    assert disp > 0
    assert np.abs(xa - xb).max() <= 1e-4 * disp
    np.testing.assert_allclose(cva[:, :3], cvb[:, :3], rtol=1e-6, atol=1e-12)


def test_graph_steps_validation(S):
    """0 .. SCPS_MAX_GRAPH_STEPS (256) steps per graph; anything else is an
    argument error."""
    p = dict(I._base_params())
    w = I.Workload("v", dict(p), [_system(64, np.arange(64), 5)], np.zeros(2, dtype=np.int32), 1)
    ctx = _context(S, w, p, 1, 16)
    for ok in (0, 1, 256):
        ctx.set_graph_steps(ok)
    for bad in (-1, 257):
        with pytest.raises(S.ScpsError) as e:
            ctx.set_graph_steps(bad)
        assert e.value.status == -1
    ctx.close()
