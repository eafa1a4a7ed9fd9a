"""Throughput of batched rMD / SCPS stepping on one MI355X.

Default workload (the headline line, --workload scps6000): one self-consistent
path-sampling iteration of the serpin-sized chain -- 32 replicas of a
6000-particle chain (17,997,000 contact pairs, LJ + Debye-Hueckel), BAOAB at
dt = 2 fs, T = 300 K, under the SCPS tube-variable ratchets on a stack of 51
frame maps.  One benchmark step = 200 Langevin steps of every replica (one
frame interval) with its frame recorded; 50 steps make the 10^4-step
iteration, and the timed region ends with the iteration's eq (avCij) over the
recorded frames.  Before timing, a parity check at the same configuration
(forces, s and w of two replicas against the FP64 oracle).  Inputs are seeded
and synthetic and resident in HBM before timing.

Other workloads (--workload), each printed as its own JSON line:
  chain560      256 replicas of a 560-particle chain (35 groups of 16,
                contacts over the 280 heavy particles), ratchet on z, blocks
                of 100 steps in one persistent launch
  chain20       16384 replicas of the 20-bead chain (several per wavefront,
                blocks of 1000 steps), the 16-replica batch beside it
  uneven512     512 chains, N ~ U{200..3000}, each with its own native map,
                100-step blocks replayed from one captured HIP graph
  scps560       the SCPS iteration of the headline on the 560-particle
                (Fip35-sized) chain of chain560: 32 replicas, 51 frames
  autograd3000  z and E_b forward + backward for 64 chains of 3000 particles
  cutoff6000    the 6000-particle chain under rMD with contact and nonbonded
                cutoffs of 12 A from compact states: neighbour lists against
                the all-tiles path
  funnel        the toy model: 262,144 trajectories on the asymmetric funnel,
                rMD from (0, 5), the mean path of the successful ones, then
                the tube-ratchet iteration (the timed line)

Printed: replica-steps/s (value), contact-pair evals/s, the plain
one-replica-per-call form, the roofline of the dominant kernel (algorithmic
bytes or flops per launch / its launch duration from HIP events on its
stream), HBM traffic from committed counter summaries, and the FP64 CPU oracle
timed on this host on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "replica-steps/s & contact-pair evals/s, batched vs plain, 1 MI355X, 1e-5 rel"
# Algorithmic FP32 flops (an FMA counts 2; rcp, rsqrt, exp count 1):
FLOPS_CONTACT = 43      # contact pair: geometry 8, C(q) 10, C'(q) 11, (C-R)^2 3, both gradient sides 11
FLOPS_CONTACT_Z = 21    # contact pair, z only: geometry 8, C(q) 10, (C-R)^2 3
FLOPS_NONBONDED = 40    # LJ 12-6 + Debye-Hueckel pair incl. geometry 8 and both force sides
FLOPS_GEOMETRY = 8      # shared by the two terms when a pair is both (a fused pair counts 75)
FLOPS_MAP = 18          # one C(q) for the ensemble mean (float64)


def flops_scps_contact(K):
    """SCPS step per contact pair: pass 1 (geometry, C, K squared differences)
    18 + 3K; pass 2 (a contact-gradient pair with the effective reference
    sum_k c_k R_k) 43 + 2K."""
    return 18 + 3 * K + 43 + 2 * K


FLOPS_FUNNEL = 60       # toy model step: force of eq (U) ~40, rMD bias ~10, update and noise transform ~10
FLOPS_FUNNEL_FRAME = 32  # per mean-path frame and step, float64: the largest exponent (distance 5, scale and
                         # max 2), then the weight (distance 5, shift 2, exp 1), its sums (3) and the four
                         # gradient sums (14)

PEAK_FP32 = 157.3e12    # MI355X vector FP32, 256 CUs x 2.4 GHz (packed two-wide FMAs)
PEAK_FP32_UNPACKED = 78.6e12   # the same with one FMA per lane and cycle: packed FP32 is compiled out here
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12       # MI355X HBM3E, bytes/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="scps6000",
                    choices=["chain560", "chain20", "uneven512", "autograd3000", "scps6000", "scps560", "cutoff6000",
                             "funnel"])
    ap.add_argument("--steps", type=int, default=None,
                    help="timed benchmark steps (default: 50 for scps6000, one 10^4-step iteration; else 20)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed benchmark steps (default 2 / 3)")
    ap.add_argument("--block", type=int, default=None,
                    help="Langevin steps per benchmark step (default: 200 for scps6000, a frame interval; else 100)")
    ap.add_argument("--replicas", type=int, default=0, help="0: the workload's own count")
    ap.add_argument("--graph-steps", type=int, default=None,
                    help="steps per replayed HIP graph on the per-step path (scps_set_graph_steps; "
                         "uneven512 default: the block, 100; other workloads: the library's default, 0)")
    ap.add_argument("--plain-replicas", type=int, default=8)
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the parity check before timing (short profiler runs only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (to scale HBM byte counters)")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = SCPS_ITER_STEPS // 200 if a.workload in ("scps6000", "scps560") else 20
    if a.warmup is None:
        a.warmup = 2 if a.workload in ("scps6000", "scps560") else 3
    if a.block is None:
        a.block = {"scps6000": 200, "scps560": 200, "chain20": 1000}.get(a.workload, 100)
    return a


# sources of the persistent rMD kernel: its counter summary is valid for these
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1705_02180_amd", "csrc", f)
                  for f in ("scps_kernels.hip", "scps_device.h", "scps_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rmd_persistent_traffic.json")


def source_sha256():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, or None when
    it is missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_sha256():
        return None
    return t.get("bytes_per_launch")


SCPS_KERNEL_SOURCES = [os.path.join(ROOT, "paper_1705_02180_amd", "csrc", f)
                       for f in ("scps_maps.hip", "scps_device.h", "scps_internal.h")]
SCPS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_scps_traffic_chain6000x32.json")


def measured_scps_traffic():
    """HBM bytes per launch of the SCPS step's two passes ({"distance": B,
    "bias": B}) from the committed counter summary, or None when it is
    missing or was taken on different kernel sources."""
    import hashlib
    try:
        with open(SCPS_TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for path in SCPS_KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    if t.get("source_sha256") != h.hexdigest():
        return None
    return t.get("bytes_per_launch")


def copy_calibration():
    import torch
    n = 64 * 1024 * 1024                     # 64 Mi float32 = 256 MiB read + 256 MiB written
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)


def pair_counts(sy, params):
    """(contact pairs, nonbonded pairs, pairs that are both) of one chain."""
    n, ci = sy.n, sy.contact_idx
    nc = len(ci)
    ex, msep = params["nb_excl"], params["min_seq_sep"]
    nb = n * (n - 1) // 2 - sum(n - d for d in range(1, ex + 1) if d < n)
    if nc == n and msep <= ex:
        # every particle is a contact: all nonbonded pairs are also contacts
        con = n * (n - 1) // 2 - sum(n - d for d in range(1, msep + 1) if d < n)
        return con, nb, nb
    import numpy as np
    d = ci[None, :] - ci[:, None]
    con = int(np.count_nonzero(d > msep))
    both = int(np.count_nonzero(d > max(msep, ex)))
    return con, nb, both


def step_flops(con, nb, both):
    return FLOPS_CONTACT * con + FLOPS_NONBONDED * nb - FLOPS_GEOMETRY * both


def timed_calls(torch, fn, n_calls):
    """Run fn() n_calls times on torch's current stream (the one the library
    launches on); returns (wall seconds, per-call milliseconds from HIP events)."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_calls + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(n_calls):
        fn(k)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [ev[k].elapsed_time(ev[k + 1]) for k in range(n_calls)]


def median(v):
    s = sorted(v)
    m = len(s) // 2
    return s[m] if len(s) % 2 else 0.5 * (s[m - 1] + s[m])


def base_line(args, value, unit, wall, n_calls, config, dtype="f32"):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": n_calls,
            "warmup": args.warmup, "ms_per_step": 1e3 * wall / n_calls, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def roofline(flops_per_call, per_call_ms, kernel, traffic=None, peak=PEAK_FP32):
    avg_s = sum(per_call_ms) / len(per_call_ms) / 1e3
    achieved = flops_per_call / avg_s
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "kernel": kernel, "avg_launch_ms": 1e3 * avg_s,
            "median_launch_ms": median(per_call_ms)}


def unpacked_view(line):
    """The FP32 roofline line against the unpacked FMA peak (78.6 TFLOP/s): the
    kernels are built without packed FP32, so one FMA per lane and cycle is
    their arithmetic ceiling.  Reported beside `roofline`, which keeps the
    published 157.3 TFLOP/s."""
    v = dict(line)
    v["peak"] = PEAK_FP32_UNPACKED / 1e12
    v["frac"] = line["achieved"] * 1e12 / PEAK_FP32_UNPACKED
    v["note"] = "FP32 with packed two-wide FMAs compiled out: one FMA per lane and cycle"
    return v


def roofline_hbm(bytes_per_call, per_call_ms, kernel, traffic=None):
    avg_s = sum(per_call_ms) / len(per_call_ms) / 1e3
    achieved = bytes_per_call / avg_s
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": achieved / PEAK_HBM, "traffic": traffic, "kernel": kernel, "avg_launch_ms": 1e3 * avg_s,
            "median_launch_ms": median(per_call_ms)}


def host_threads():
    return len(os.sched_getaffinity(0))


# ---------------------------------------------------------------------------
# 256 x 560: the headline workload
# ---------------------------------------------------------------------------
def run_plain(scps, torch, w, n_rep, n_steps):
    """One replica per context and per launch sequence (a few kernels per step)."""
    sy = w.systems[0]
    n3 = 3 * sy.n
    X0, V0 = w.initial_x(), w.initial_v(7)
    ctxs, bufs = [], []
    for r in range(n_rep):
        c = scps.Context.from_workload(w, exec_mode=1, replica_system=[0], replica_base=r)
        c.set_reference_map(0, native_xyz=sy.native)
        x = torch.as_tensor(X0[r * n3:(r + 1) * n3], device="cuda")
        v = torch.as_tensor(V0[r * n3:(r + 1) * n3], device="cuda")
        cv = torch.as_tensor(w.initial_cvstate()[r:r + 1], device="cuda")
        ctxs.append(c)
        bufs.append((x, v, cv))
    for c, (x, v, cv) in zip(ctxs, bufs):          # warm-up
        c.step_replicas(x, v, cv, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m in range(n_steps):
        for c, (x, v, cv) in zip(ctxs, bufs):
            c.step_replicas(x, v, cv, 1, step0=1 + m)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    return n_rep * n_steps / dt


def cpu_baseline_steps(w, n_steps, replicas=None, what=""):
    """The FP64 oracle (OpenMP over replicas) on replicas x n_steps, from the
    workload's start states."""
    import numpy as np
    import oracle as O
    rs = np.asarray(w.replica_system if replicas is None else w.replica_system[replicas], dtype=np.int32)
    used_sys = sorted(set(rs.tolist()))
    remap = {s: k for k, s in enumerate(used_sys)}
    systems = [O.System.from_inputs(w.systems[s], w.params) for s in used_sys]
    rs_local = np.array([remap[s] for s in rs.tolist()], dtype=np.int32)
    ids = np.arange(w.n_replicas) if replicas is None else np.asarray(replicas)
    own = w.notes.get("replica_starts")
    x = np.concatenate([(own[r] if own is not None else w.systems[w.replica_system[r]].start).ravel()
                        for r in ids.tolist()]).astype(np.float64)
    v = np.zeros_like(x) if w.params["integrator"] == 1 else None
    cv = np.zeros((len(rs), 8))
    cv[:, 1] = cv[:, 5] = cv[:, 6] = np.inf
    t0 = time.perf_counter()
    _, _, _, used = O.run_batch(w.params, systems, rs_local, x, v, cv, n_steps, 0, host_threads())
    dt = time.perf_counter() - t0
    return {"value": len(rs) * n_steps / dt, "unit": "replica-steps/s", "cores": int(used), "kind": "oracle",
            "sample": f"{len(rs)} replicas x {n_steps} Langevin steps{what}, FP64, OpenMP over replicas "
                      f"({dt:.1f} s)"}


def bench_chain560(args, torch, I, scps):
    R = args.replicas or 256
    w = I.config2(n_replicas=R)
    sy = w.systems[0]
    con, nb, both = pair_counts(sy, w.params)
    ctx = scps.Context.from_workload(w)
    ctx.set_reference_map(0, native_xyz=sy.native)
    x = torch.as_tensor(w.initial_x(), device="cuda")
    v = torch.as_tensor(w.initial_v(7), device="cuda")
    cv = torch.as_tensor(w.initial_cvstate(), device="cuda")
    step = [0]
    path, threads = ctx.autotune(x, v, cv, args.block)      # on copies of the state, before timing

    def call(_):
        ctx.step_replicas(x, v, cv, args.block, step0=step[0])
        step[0] += args.block

    for _ in range(args.warmup):
        call(0)
    ctx.sync()
    wall, per_ms = timed_calls(torch, call, args.steps)
    ctx.sync()
    value = R * args.block * args.steps / wall
    out = base_line(args, value, "replica-steps/s", wall, args.steps, {
        "workload": f"chain560_fip35_shaped: {R} replicas x 560 particles, {con} contact pairs + "
                    f"{nb} LJ/Debye-Hueckel pairs ({both} both), BAOAB dt=2 fs, {args.block} Langevin "
                    f"steps per benchmark step",
        "replicas": R, "particles": sy.n, "block": args.block,
        "launch": "persistent, %d threads per replica" % threads if path == 0 else "per-step"})
    out["contact_pair_evals_per_s"] = value * con
    out["nonbonded_pair_evals_per_s"] = value * nb
    out["roofline"] = roofline(R * args.block * step_flops(con, nb, both), per_ms, "k_rmd_persistent",
                               measured_traffic())
    out["roofline_fp32_unpacked"] = unpacked_view(out["roofline"])
    if not args.no_plain:
        plain = run_plain(scps, torch, w, args.plain_replicas, args.plain_steps)
        out["plain"] = {"value": plain, "unit": "replica-steps/s",
                        "form": f"one replica per context, one launch sequence per Langevin step "
                                f"({args.plain_replicas} replicas x {args.plain_steps} steps)"}
        out["speedup_vs_plain"] = value / plain
    ctx.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_steps(w, args.cpu_steps, what=" of the same workload")
    return out


# ---------------------------------------------------------------------------
# the 20-bead chain, many replicas per wavefront
# ---------------------------------------------------------------------------
def bench_chain20(args, torch, I, scps):
    """The 20-bead overdamped chain (LJ, contacts against a compact native
    map) batched: 16384 replicas by default, floor(64 / 20) = 3 per
    wavefront on the packed kernel unless the autotuner finds better; the
    16-replica batch of the CPU-sized configuration is timed beside it."""
    R = args.replicas or 16384
    w = I.config1(n_replicas=R)
    sy = w.systems[0]
    con, nb, both = pair_counts(sy, w.params)

    def make(wl):
        c = scps.Context.from_workload(wl)
        c.set_reference_map(0, native_xyz=sy.native)
        return (c, torch.as_tensor(wl.initial_x(), device="cuda"),
                torch.as_tensor(wl.initial_cvstate(), device="cuda"))

    ctx, x, cv = make(w)
    path, param = ctx.autotune(x, None, cv, args.block // 10)  # on copies of the state, before timing
    step = [0]

    def call(_):
        ctx.step_replicas(x, None, cv, args.block, step0=step[0])
        step[0] += args.block

    for _ in range(args.warmup):
        call(0)
    ctx.sync()
    wall, per_ms = timed_calls(torch, call, args.steps)
    ctx.sync()
    value = R * args.block * args.steps / wall
    launch = {0: f"persistent, {param} threads per replica", 1: "per-step",
              2: f"packed, {param} replicas per workgroup ({64 // sy.n} per wavefront)"}[path]
    out = base_line(args, value, "replica-steps/s", wall, args.steps, {
        "workload": f"chain20_config1: {R} replicas x 20 beads, {con} contact pairs + {nb} LJ pairs, "
                    f"overdamped dt=0.01, {args.block} Langevin steps per benchmark step",
        "replicas": R, "particles": sy.n, "block": args.block, "launch": launch + " (autotuned)"})
    out["contact_pair_evals_per_s"] = value * con
    out["nonbonded_pair_evals_per_s"] = value * nb
    kname = {0: "k_rmd_persistent", 1: "k_pairs", 2: "k_rmd_packed"}[path]
    out["roofline"] = roofline(R * args.block * step_flops(con, nb, both), per_ms, kname, None)
    out["roofline"]["note"] = ("flop counts each pair once, as the packed kernel evaluates it (the j side's "
                               "partials travel between lanes)")
    out["roofline_fp32_unpacked"] = unpacked_view(out["roofline"])
    ctx.close()
    # the CPU-sized configuration as stated: 16 replicas
    w16 = I.config1(n_replicas=16)
    c16, x16, cv16 = make(w16)
    c16.step_replicas(x16, None, cv16, 10)
    c16.sync()
    t0 = time.perf_counter()
    c16.step_replicas(x16, None, cv16, 1000, step0=10)
    c16.sync()
    out["config1_16_replicas"] = {"value": 16 * 1000 / (time.perf_counter() - t0), "unit": "replica-steps/s",
                                  "launch": "default (packed, 4 wavefronts per workgroup)"}
    c16.close()
    if not args.no_plain:
        plain = run_plain(scps, torch, w, args.plain_replicas, args.plain_steps)
        out["plain"] = {"value": plain, "unit": "replica-steps/s",
                        "form": f"one replica per context, one launch sequence per Langevin step "
                                f"({args.plain_replicas} replicas x {args.plain_steps} steps)"}
        out["speedup_vs_plain"] = value / plain
    if not args.no_cpu:
        # about 20 s of oracle work: the 20-bead chain costs ~0.1 ms per replica-step on one core
        out["cpu_baseline"] = cpu_baseline_steps(w, max(args.cpu_steps, 30000), replicas=list(range(min(R, 2048))),
                                                 what=" of the same workload")
    return out


# ---------------------------------------------------------------------------
# 512 uneven chains
# ---------------------------------------------------------------------------
def bench_uneven512(args, torch, I, scps):
    import numpy as np
    R = args.replicas or 512
    w = I.config3(n_replicas=R)
    counts = [pair_counts(s, w.params) for s in w.systems]
    con = sum(c[0] for c in counts)
    flops = sum(step_flops(*c) for c in counts)
    ctx = scps.Context.from_workload(w)
    for s, sy in enumerate(w.systems):
        ctx.set_reference_map(s, native_xyz=sy.native)
    x = torch.as_tensor(w.initial_x(), device="cuda")
    v = torch.as_tensor(w.initial_v(7), device="cuda")
    cv = torch.as_tensor(w.initial_cvstate(), device="cuda")
    step = [0]
    ctx.autotune(x, v, cv, 5)                                # on copies of the state, before timing
    # the per-step path's blocks replayed from one captured HIP graph each
    gsteps = min(args.block, 256) if args.graph_steps is None else args.graph_steps
    ctx.set_graph_steps(gsteps)

    def call(_):
        ctx.step_replicas(x, v, cv, args.block, step0=step[0])
        step[0] += args.block

    for _ in range(args.warmup):
        call(0)
    ctx.sync()
    wall, per_ms = timed_calls(torch, call, args.steps)
    ctx.sync()
    value = R * args.block * args.steps / wall
    sizes = w.replica_sizes()
    out = base_line(args, value, "replica-steps/s", wall, args.steps, {
        "workload": f"uneven_chains: {R} chains, N ~ U{{200..3000}} (sum {int(sizes.sum())}, max "
                    f"{int(sizes.max())}), own native map each, all particles in the contact set "
                    f"({con} contact pairs per batched step), LJ + Debye-Hueckel, BAOAB dt=2 fs, "
                    f"{args.block} Langevin steps per benchmark step",
        "replicas": R, "particles_total": int(sizes.sum()), "block": args.block,
        "graph_steps": gsteps})
    out["contact_pair_evals_per_s"] = value / R * con
    out["roofline"] = roofline(args.block * flops, per_ms, "scps_step_replicas (all kernels of a block)")
    out["roofline_fp32_unpacked"] = unpacked_view(out["roofline"])
    # every chain has its own float32 reference map, read once per step: the
    # map stream is about as binding as the arithmetic here
    out["roofline_hbm"] = roofline_hbm(args.block * con * 4, per_ms, "each chain's reference map read once per step")
    ctx.close()
    if not args.no_cpu:
        rng = np.random.default_rng(5)
        sample = np.sort(rng.choice(R, size=min(R, 64), replace=False))
        out["cpu_baseline"] = cpu_baseline_steps(w, max(1, args.cpu_steps // 8), replicas=sample,
                                                 what=" (a random 64 of the chains)")
    return out


# ---------------------------------------------------------------------------
# 64 x 3000: autograd forward + backward
# ---------------------------------------------------------------------------
def bench_autograd3000(args, torch, I, scps):
    import numpy as np
    R = args.replicas or 64
    w = I.config4(n_chains=R)
    n = w.systems[0].n
    P = n * (n - 1) // 2
    ctx = scps.Context.from_workload(w)
    for s, sy in enumerate(w.systems):
        ctx.set_reference_map(s, native_xyz=sy.native)
    X = np.concatenate([I.random_coil(n, 9000 + s).astype(np.float32).ravel() for s in range(R)])
    x = torch.as_tensor(X, device="cuda").requires_grad_(True)
    z0 = torch.empty(R, dtype=torch.float64, device="cuda")
    ctx.eval_z_and_grad(x.detach(), z0)
    zm = 0.9 * z0

    def call(_):
        x.grad = None
        z, eb = scps.zbias(x, zm, ctx)
        (z.sum() + eb.sum()).backward()

    for _ in range(args.warmup):
        call(0)
    torch.cuda.synchronize()
    wall, per_ms = timed_calls(torch, call, args.steps)
    value = R * args.steps / wall
    out = base_line(args, value, "chain fwd+bwd/s", wall, args.steps, {
        "workload": f"autograd_chains: {R} chains x {n} particles, {P} contact pairs each, z and E_b "
                    f"forward + backward (one pair pass for z and dz/dx in the forward; the backward scales "
                    f"the kept dz/dx per chain)",
        "chains": R, "particles": n})
    out["contact_pair_evals_per_s"] = value * P
    # each chain has its own float32 reference map, streamed once per forward + backward:
    # that stream, not the arithmetic, is the bound
    out["roofline"] = roofline_hbm(R * P * 4, per_ms, "forward + backward: each chain's reference map read once")
    out["roofline_alu"] = roofline(R * P * FLOPS_CONTACT, per_ms, "the same calls against the FP32 peak")
    ctx.close()
    if not args.no_cpu:
        import oracle as O
        m = R
        t0 = time.perf_counter()
        for s in range(m):
            osys = O.System.from_inputs(w.systems[s], w.params)
            xs = X[3 * n * s:3 * n * (s + 1)].reshape(3, n).astype(np.float64)
            O.z_grad(xs, osys.cidx, osys.native, grad=True)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m / dt, "unit": "chain fwd+bwd/s", "cores": 1, "kind": "oracle",
                               "sample": f"{m} chains, z and grad z, FP64, one thread ({dt:.1f} s)"}
    return out


# ---------------------------------------------------------------------------
# 32 x 6000, 51 frames: one SCPS iteration (the headline workload)
# ---------------------------------------------------------------------------
SCPS_FRAMES = 51          # a frame every 200 steps over a 10^4-step iteration
PASS_TIMING_PERIOD = 8    # scps_time_passes: events around the passes of every 8th step
SCPS_ITER_STEPS = 10000


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _pmap(fn, items, threads):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max(1, threads)) as ex:      # the oracle's ctypes calls release the GIL
        return list(ex.map(fn, items))


def oracle_stack(sy, frames, params, threads):
    """eq (avCij) of one path's frames [K][1][3][n] by the oracle, the frames
    split over threads; float64 [K][P]."""
    import numpy as np
    import oracle as O
    K = frames.shape[0]
    P = len(sy.contact_idx) * (len(sy.contact_idx) - 1) // 2
    out = np.empty((K, P))
    chunks = [list(range(k, min(K, k + 4))) for k in range(0, K, 4)]

    def one(ch):
        st, _ = O.update_reference(sy.n, sy.contact_idx, frames[ch].astype(np.float64), np.ones(1, dtype=np.uint8),
                                   params["r0_contact"], params["r_cut_contact"])
        out[ch] = st
    _pmap(one, chunks, threads)
    return out


def scps6000_parity(torch, scps, w, threads):
    """Parity check at the timed configuration before timing: the same chain,
    replica count, stack size and launch path, with the stack of one path's
    51 frames computed by both sides; forces read back from one BAOAB step
    from rest at kT = 0 (v = c1 dt F / m) on two sampled replicas with active
    tube ratchets, against the oracle's total force (1e-5 normwise), and s, w
    (1e-5).  Returns (summary, the oracle's stack, its frames)."""
    import math
    import numpy as np
    import oracle as O
    sy = w.systems[0]
    n, R, K = sy.n, w.n_replicas, SCPS_FRAMES
    p = dict(w.params, bias_mode=1, kT=0.0, gamma=1e-3)
    rng = np.random.default_rng(31)
    frames = np.empty((K, 1, 3, n), dtype=np.float32)
    for k in range(K):
        lam = k / (K - 1)
        frames[k, 0] = (1 - lam) * sy.start + lam * sy.native + rng.normal(0, 0.5, size=(3, n))
    t0 = time.perf_counter()
    stack = oracle_stack(sy, frames, p, threads)
    osys = O.System(n, sy.contact_idx, sy.mass, sy.charge, p, native_xyz=sy.native, stack=stack)
    X = np.stack([(frames[(7 + 3 * r) % K, 0] + rng.normal(0, 0.3, size=(3, n))) for r in range(R)]).astype(np.float32)
    sample = [13, R - 1]
    cv0 = np.zeros((R, 8))
    cv0[:, 5:7] = np.inf
    for r in sample:
        sv, wv, *_ = O.tube(X[r].astype(np.float64), osys.cidx, stack, osys.Z0, p["lam"], grads=False)
        cv0[r, 5], cv0[r, 6] = sv - 0.05, wv - 0.01
    ctx = scps.Context.from_workload(w, params=p)
    ctx.set_reference_map(0, native_xyz=sy.native)
    ctx.update_reference_from_paths(0, torch.as_tensor(frames.ravel(), device="cuda"), 1, K,
                                    np.ones(1, dtype=np.uint8))
    x = torch.as_tensor(X.ravel(), device="cuda")
    v = torch.zeros_like(x)
    cv = torch.as_tensor(cv0, device="cuda")
    ctx.step_replicas(x, v, cv, 1)
    ctx.sync()
    ctx.close()
    c1 = math.exp(-p["gamma"] * p["dt"])
    V = v.cpu().numpy().reshape(R, 3, n).astype(np.float64) * sy.mass.astype(np.float64) / (c1 * p["dt"])
    CV = cv.cpu().numpy()
    want = _pmap(lambda r: O.total_force(p, osys, X[r].astype(np.float64), cv0[r]), sample, threads)
    errs, ds, dw = [], [], []
    for r, (F, Fb, cvo) in zip(sample, want):
        d = np.linalg.norm(V[r] - F, axis=0).max() / np.linalg.norm(F, axis=0).max()
        errs.append(float(d))
        ds.append(float(abs(CV[r, 3] - cvo[3])))
        dw.append(float(abs(CV[r, 4] - cvo[4])))
    ok = max(errs) <= 1e-5 and max(ds) <= 1e-5 and max(dw) <= 1e-5
    summary = {"replicas": sample, "force_err_normwise": errs, "s_err": ds, "w_err": dw, "tol": 1e-5,
               "passed": bool(ok), "oracle_s": round(time.perf_counter() - t0, 1),
               "check": f"{R} x {n}, {K}-frame stack of one path (both sides compute it), forces of one BAOAB "
                        f"step from rest at kT = 0 on replicas {sample} (tube ratchets active), s and w"}
    print(f"parity at the timed configuration: {summary}", file=sys.stderr, flush=True)
    return summary, stack, frames


def bench_scps6000(args, torch, I, scps, fip=False):
    import numpy as np
    R = args.replicas or 32
    # the serpin-sized chain of the headline, or (fip) the 560-particle Fip35-sized chain under SCPS
    w = I.config2(n_replicas=R) if fip else I.config5(n_replicas=R)
    sy = w.systems[0]
    n = sy.n
    con, nb, both = pair_counts(sy, w.params)
    K = SCPS_FRAMES
    blk = args.block
    threads = min(host_threads(), 16)
    parity, ostack = None, None
    if not args.no_parity:
        parity, ostack, _ = scps6000_parity(torch, scps, w, threads)
    # the stack the timed iteration starts from: the ensemble mean of a short
    # rMD run's recorded frames (iteration 0, abbreviated here)
    rmd = scps.Context.from_workload(w)
    rmd.set_reference_map(0, native_xyz=sy.native)
    x = torch.as_tensor(w.initial_x(), device="cuda")
    v = torch.as_tensor(w.initial_v(7), device="cuda")
    cv = torch.as_tensor(w.initial_cvstate(), device="cuda")
    frames0 = torch.empty(K * 3 * R * n, dtype=torch.float32, device="cuda")
    rmd.step_replicas(x, v, cv, 2 * (K - 1), record_every=2, frames=frames0)
    rmd.sync()
    rmd.close()
    p = dict(w.params, bias_mode=1)
    ctx = scps.Context.from_workload(w, params=p)
    ctx.set_reference_map(0, native_xyz=sy.native)
    succ = np.ones(R, dtype=np.uint8)
    ctx.update_reference_from_paths(0, frames0, R, K, succ)
    cvs = torch.as_tensor(w.initial_cvstate(), device="cuda")
    x0, v0 = x.clone(), v.clone()
    n3 = 3 * R * n
    nrec = min(args.steps + 1, 128)                  # frames of the iteration for eq (avCij)
    frames = torch.empty((args.steps + 1) * n3, dtype=torch.float32, device="cuda")
    step = [0]

    def block_call(b):
        # one frame interval for every replica: its start and end configurations are recorded
        ctx.step_replicas(x, v, cvs, blk, step0=step[0], record_every=blk, frames=frames[b * n3:(b + 2) * n3])
        step[0] += blk

    _, overlap = ctx.autotune(x, v, cvs, 10)                # on copies of the state, before timing
    # the passes are timed on every PASS_TIMING_PERIOD-th step of the timed
    # region (a timed step's kernels cannot overlap across its events); with
    # --graph-steps the timed steps replay captured graphs instead and the
    # passes are timed in a launch-by-launch segment after the timed region
    gsteps = args.graph_steps or 0
    ctx.set_graph_steps(gsteps)
    for _ in range(args.warmup):
        block_call(0)
    ctx.sync()
    if not gsteps:
        ctx.time_passes(PASS_TIMING_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(args.steps):
        block_call(b)
    # the iteration ends with eq (avCij) over its recorded frames (blocks until done)
    torch.cuda.synchronize()                             # (only to split the time between the two parts)
    t_upd = time.perf_counter()
    ctx.update_reference_from_paths(0, frames[(args.steps + 1 - nrec) * n3:], R, nrec, succ)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    if gsteps:
        ctx.time_passes(PASS_TIMING_PERIOD)
        for b in range(2):
            block_call(b)
        ctx.sync()
    pass_ms, timed = ctx.pass_times()
    ctx.time_passes(False)
    ctx.sync()
    value = R * blk * args.steps / wall
    out = base_line(args, value, "replica-steps/s", wall, args.steps, {
        "workload": f"{w.name} SCPS iteration: {R} replicas x {n} particles, SCPS bias on a stack "
                    f"of {K} frame maps x {con} contact pairs, LJ + Debye-Hueckel, BAOAB dt=2 fs; one benchmark "
                    f"step = {blk} Langevin steps of every replica with its frame recorded; the timed region "
                    f"ends with eq (avCij) over the {nrec} recorded frames (once per iteration)",
        "replicas": R, "particles": n, "frames": K, "block": blk,
        "iteration_steps": blk * args.steps,
        "launch": "per step: distance pass, ratchets, bias pass, update; nonbonded pass " +
                  ("beside the distance pass on a second stream" if overlap else "after the bias pass") +
                  " (autotuned)" + (f"; blocks of {gsteps} steps replayed from a captured HIP graph" if gsteps else ""),
        "graph_steps": gsteps})
    out["contact_pair_evals_per_s"] = value * con
    out["eq_avCij_ms"] = 1e3 * (t1 - t_upd)
    out["parity"] = parity
    # the two passes of a step each stream the float32 frame stack once per
    # group of up to 32 replicas: the bound of the step
    groups = (R + 31) // 32
    stack_bytes = groups * K * con * 4
    per = {k: pass_ms[k] / max(timed, 1) for k in ("distance", "bias")}
    dom = max(per, key=per.get)
    names = {"distance": "k_scps_dist (distances to every frame)",
             "bias": "k_scps_bias (effective references and bias forces)"}
    traffic = None if fip else measured_scps_traffic()   # the counter record is the serpin-sized chain's
    out["roofline"] = roofline_hbm(stack_bytes, [per[dom]] * 1, names[dom],
                                   traffic.get(dom) if traffic else None)
    out["roofline"]["launches_timed"] = timed
    out["roofline"]["pass_timing"] = (
        f"HIP events around each pass on every {PASS_TIMING_PERIOD}th step of the timed region" if not gsteps else
        f"HIP events around each pass on every {PASS_TIMING_PERIOD}th of {2 * blk} launch-by-launch steps after "
        f"the timed region (the timed steps replay graphs)")
    other = "bias" if dom == "distance" else "distance"
    out["roofline_other_pass"] = roofline_hbm(stack_bytes, [per[other]], names[other],
                                              traffic.get(other) if traffic else None)
    step_ms = 1e3 * (t_upd - t0) / (args.steps * blk)
    per_step = flops_scps_contact(K) * con + FLOPS_NONBONDED * nb - FLOPS_GEOMETRY * both
    out["step_ms"] = step_ms
    out["roofline_alu"] = roofline(R * per_step, [step_ms], "the whole SCPS step against the FP32 peak "
                                                           "(MFMA contraction flops included)")
    out["roofline_step_hbm"] = roofline_hbm(2 * stack_bytes, [step_ms], "the whole SCPS step: stack read twice")
    ctx.close()
    if args.no_plain:
        out["cpu_baseline"] = scps6000_cpu(w, p, ostack, threads) if not args.no_cpu else None
        return out
    # the plain form: one replica per context and per call, a host loop over replicas
    plain = scps.Context.from_workload(w, params=p, replica_system=[0])
    plain.set_reference_map(0, native_xyz=sy.native)
    plain.update_reference_from_paths(0, frames0, R, K, succ)          # the same stack as the batched run
    reps = list(range(min(R, args.plain_replicas)))
    st = [(x0[3 * n * r:3 * n * (r + 1)].clone(), v0[3 * n * r:3 * n * (r + 1)].clone(),
           torch.as_tensor(w.initial_cvstate()[:1], device="cuda")) for r in reps]
    for xr, vr, cr in st:
        plain.step_replicas(xr, vr, cr, 1)
    plain.sync()
    n_plain = 2
    tp = time.perf_counter()
    for m in range(n_plain):
        for xr, vr, cr in st:
            plain.step_replicas(xr, vr, cr, 1, step0=1 + m)
    plain.sync()
    rate_plain = len(reps) * n_plain / (time.perf_counter() - tp)
    plain.close()
    out["plain"] = {"value": rate_plain, "unit": "replica-steps/s",
                    "form": f"one replica per context and call, host loop ({len(reps)} replicas x {n_plain} steps)"}
    out["speedup_vs_plain"] = value / rate_plain
    if not args.no_cpu:
        out["cpu_baseline"] = scps6000_cpu(w, p, ostack, threads)
    return out


def scps6000_cpu(w, p, stack, threads):
    """The oracle on the same chain and stack size: SCPS steps of one replica
    on one thread, and of `threads` replicas side by side, as many steps as
    make each sample last about 10 s (one for the serpin-sized chain)."""
    import numpy as np
    import oracle as O
    sy = w.systems[0]
    if stack is None:          # no parity check ran: a stack of shifted native maps (the cost is the same)
        nat = O.contact_map(sy.native, sy.contact_idx)
        stack = np.repeat(nat[None], SCPS_FRAMES, axis=0)
        stack *= np.linspace(0.9, 1.0, SCPS_FRAMES)[:, None]
    osys = O.System(sy.n, sy.contact_idx, sy.mass, sy.charge, p, native_xyz=sy.native, stack=stack)
    res = {}
    for m in (1, threads):
        k = 1
        while True:
            xs = np.concatenate([sy.start.ravel()] * m).astype(np.float64)
            vs = np.zeros_like(xs)
            cv0 = np.zeros((m, 8))
            cv0[:, 1] = cv0[:, 5] = cv0[:, 6] = np.inf
            t0 = time.perf_counter()
            _, _, _, used = O.run_batch(p, [osys], np.zeros(m, dtype=np.int32), xs, vs, cv0, k, 0, m)
            dt = time.perf_counter() - t0
            if dt >= 5.0 or k >= 4096:
                break
            k = min(4096, max(2 * k, int(k * 10.0 / max(dt, 1e-3)) + 1))
        res[m] = (m * k / dt, int(used), dt, k)
    v_all, used, dt, k_all = res[threads]
    v_one, _, dt1, k_one = res[1]
    return {"value": v_all, "unit": "replica-steps/s", "cores": used, "kind": "oracle",
            "single_thread_value": v_one, "cpu_model": cpu_model(),
            "sample": f"{threads} replicas x {k_all} SCPS step(s) of the same chain and stack size, FP64, OpenMP "
                      f"over replicas ({dt:.1f} s); single thread: 1 replica x {k_one} step(s) ({dt1:.1f} s)"}


# ---------------------------------------------------------------------------
# 32 x 6000 with 12 A cutoffs: the linear-scaling variant
# ---------------------------------------------------------------------------
def pairs_within(x, r_cut, nb_excl, min_sep):
    """(contact, nonbonded, both) pairs of one all-contact chain closer than
    r_cut, at coordinates x [3][n] (float64)."""
    import numpy as np
    from scipy.spatial import cKDTree
    pr = cKDTree(np.ascontiguousarray(x.T)).query_pairs(r_cut, output_type="ndarray")
    sep = np.abs(pr[:, 0] - pr[:, 1])
    con = int(np.count_nonzero(sep > min_sep))
    nb = int(np.count_nonzero(sep > nb_excl))
    both = int(np.count_nonzero(sep > max(min_sep, nb_excl)))
    return con, nb, both


def bench_cutoff6000(args, torch, I, scps):
    import numpy as np
    R = args.replicas or 32
    w = I.config6(n_replicas=R)
    sy = w.systems[0]
    p = w.params
    X0 = w.initial_x().reshape(R, 3, sy.n).astype(np.float64)
    within = [pairs_within(X0[r], p["r_cut_contact"], p["nb_excl"], p["min_seq_sep"]) for r in range(R)]
    con = sum(c[0] for c in within) / R
    flops = sum(step_flops(*c) for c in within)             # per batched step, pairs inside the cutoff
    all_con, all_nb, all_both = pair_counts(sy, p)
    rates = {}
    for mode, label in ((1, "lists"), (2, "all_tiles")):
        ctx = scps.Context.from_workload(w, exec_mode=mode)
        ctx.set_reference_map(0, native_xyz=sy.native)
        x = torch.as_tensor(w.initial_x(), device="cuda")
        v = torch.as_tensor(w.initial_v(7), device="cuda")
        cv = torch.as_tensor(w.initial_cvstate(), device="cuda")
        step = [0]

        def call(_):
            ctx.step_replicas(x, v, cv, args.block, step0=step[0])
            step[0] += args.block

        for _ in range(args.warmup):
            call(0)
        ctx.sync()
        n_calls = args.steps if mode == 1 else max(2, args.steps // 10)
        wall, per_ms = timed_calls(torch, call, n_calls)
        ctx.sync()
        ctx.close()
        rates[label] = (R * args.block * n_calls / wall, wall, n_calls, per_ms)
    value, wall, n_calls, per_ms = rates["lists"]
    out = base_line(args, value, "replica-steps/s", wall, n_calls, {
        "workload": f"chain6000_cutoff: {R} replicas x {sy.n} particles, rMD, contact and LJ/Debye-Hueckel "
                    f"cutoffs {p['r_cut_contact']:g} A, compact starts (native + 0.05 A jitter), "
                    f"{con:.0f} contact pairs inside the cutoff per replica (of {all_con}), BAOAB dt=2 fs, "
                    f"{args.block} Langevin steps per benchmark step",
        "replicas": R, "particles": sy.n, "block": args.block, "launch": "per-step, neighbour lists"})
    out["pairs_within_cutoff_per_s"] = value * con
    out["roofline"] = roofline(args.block * flops, per_ms,
                               "scps_step_replicas (list upkeep + list pass + update, pairs inside the cutoff)")
    out["all_tiles"] = {"value": rates["all_tiles"][0], "unit": "replica-steps/s",
                        "form": "the same library and state on the per-step path over every tile pair",
                        "steps": rates["all_tiles"][2]}
    out["speedup_vs_all_tiles"] = value / rates["all_tiles"][0]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_steps(w, max(1, args.cpu_steps // 3), replicas=np.arange(min(R, 16)),
                                                 what=" of the same workload (all pairs, the plain loop)")
    return out


# ---------------------------------------------------------------------------
# the toy model: trajectories on the asymmetric funnel
# ---------------------------------------------------------------------------
def bench_funnel(args, torch, I, scps):
    import numpy as np
    n = args.replicas or 262144          # 4 wavefronts per SIMD; one thread per trajectory
    p = I.funnel_params()
    n_rmd, rec = 2000, 40
    K = n_rmd // rec + 1

    def fresh():
        cv = np.zeros((n, 8))
        cv[:, 1] = cv[:, 5] = cv[:, 6] = np.inf
        return (torch.as_tensor(np.tile(I.FUNNEL_START, (n, 1)), dtype=torch.float64, device="cuda"),
                torch.as_tensor(cv, device="cuda"))
    # rMD ensemble (recorded), its mean path, then the tube-ratchet iteration
    xy, cv = fresh()
    frames = torch.zeros((K, n, 2), dtype=torch.float64, device="cuda")
    wall_r, per_r = timed_calls(torch, lambda _: scps.funnel_steps(p, xy, cv, n_rmd, record_every=rec,
                                                                   frames=frames), 1)
    succ = (torch.linalg.norm(xy, dim=1) < 1.0).cpu().numpy().astype(np.uint8)
    mp = scps.funnel_mean_path(frames, succ)
    ps = dict(p, bias_mode=1)
    xy, cv = fresh()
    step = [0]

    def call(_):
        scps.funnel_steps(ps, xy, cv, args.block, step0=step[0], mean_path=mp)
        step[0] += args.block

    for _ in range(args.warmup):
        call(0)
    torch.cuda.synchronize()
    wall, per_ms = timed_calls(torch, call, args.steps)
    value = n * args.block * args.steps / wall
    out = base_line(args, value, "trajectory-steps/s", wall, args.steps, {
        "workload": f"funnel_toy_model: {n} trajectories of one particle on the asymmetric funnel (Table 1), "
                    f"kT = 0.3, gamma dt = 0.02; rMD (k_R = 70 on |X|) from (0, 5) for {n_rmd} steps, mean path of "
                    f"{K} frames over the {int(succ.sum())} that reached |X| < 1, then the tube ratchets "
                    f"(lambda = 0.3, k_s = k_w = 3), {args.block} steps per benchmark step",
        "trajectories": n, "block": args.block, "path_frames": K}, dtype="f64")
    out["rmd"] = {"value": n * n_rmd / wall_r, "unit": "trajectory-steps/s", "reached_bottom": float(succ.mean())}
    out["reached_bottom_after_iteration"] = float((torch.linalg.norm(xy, dim=1) < 1.0).float().mean())
    out["roofline"] = roofline(n * args.block * (FLOPS_FUNNEL + K * FLOPS_FUNNEL_FRAME), per_ms,
                               "k_funnel_steps<1>", peak=PEAK_FP64)
    if not args.no_cpu:
        import oracle as O
        m, st = 65536, max(10, 15 * args.cpu_steps)     # about 10 s on 16 host cores
        cv0 = np.zeros((m, 8))
        cv0[:, 5] = cv0[:, 6] = np.inf
        t0 = time.perf_counter()
        O.funnel_steps(ps, np.tile(I.FUNNEL_START, (m, 1)), cv0, st, mean_path=mp.cpu().numpy(),
                       threads=host_threads())
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m * st / dt, "unit": "trajectory-steps/s", "cores": host_threads(),
                               "kind": "oracle", "sample": f"{m} trajectories x {st} tube-ratchet steps of the same "
                                                          f"workload, FP64, OpenMP over trajectories ({dt:.1f} s)"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); replicas are independent, so "
              "more GPUs would each run their own batch with no communication.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch

    from paper_1705_02180_amd import inputs as I
    from paper_1705_02180_amd import scps

    torch.cuda.set_device(0)
    fn = {"chain560": bench_chain560, "chain20": bench_chain20, "uneven512": bench_uneven512,
          "autograd3000": bench_autograd3000, "scps6000": bench_scps6000,
          "scps560": lambda *a: bench_scps6000(*a, fip=True), "cutoff6000": bench_cutoff6000, "funnel": bench_funnel}[args.workload]
    out = fn(args, torch, I, scps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
