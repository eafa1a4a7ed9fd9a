"""Throughput of batched rMD stepping on one MI355X.

Workload: 256 replicas of a 560-particle chain (35 groups of 16, contacts over
the 280 heavy particles: 39,060 contact pairs, 155,403 nonbonded pairs),
Lennard-Jones + Debye-Hueckel, BAOAB at dt = 2 fs, T = 300 K, ratchet on z.
One benchmark step = one scps_step_replicas call that advances every replica
by --block Langevin steps (one persistent kernel launch).  Inputs are seeded
and synthetic and resident in HBM before timing starts.

Printed: one JSON line with replica-steps/s (value), contact-pair evals/s,
the plain one-replica-per-launch form on the same GPU, the roofline of the
stepping kernel (algorithmic FP32 work / HIP-event time of each launch) and
the FP64 CPU oracle timed on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "replica-steps/s & contact-pair evals/s, batched vs plain, 1 MI355X, 1e-5 rel"
# algorithmic FP32 flops per unordered pair (an FMA counts 2; rcp, rsqrt, exp count 1)
FLOPS_CONTACT = 43      # C(q), C'(q), (C-R)^2 and both gradient sides
FLOPS_NONBONDED = 40    # Lennard-Jones 12-6 + Debye-Hueckel and both force sides
PEAK_FP32 = 157.3e12    # MI355X vector FP32, 256 CUs x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--block", type=int, default=100, help="Langevin steps per benchmark step")
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--plain-replicas", type=int, default=8)
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (to scale HBM byte counters)")
    return ap.parse_args()


KERNEL_SOURCE = os.path.join(ROOT, "paper_1705_02180_amd", "csrc", "scps_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rmd_persistent_traffic.json")


def source_sha256():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


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


def copy_calibration():
    import torch
    n = 64 * 1024 * 1024                     # 64 Mi float32 = 256 MiB read + 256 MiB written
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)


def pair_counts(w):
    s = w.systems[0]
    n, nc = s.n, len(s.contact_idx)
    ex = w.params["nb_excl"]
    nb = n * (n - 1) // 2 - sum(n - d for d in range(1, ex + 1))
    ci = s.contact_idx
    msep = w.params["min_seq_sep"]
    con = sum(1 for a in range(nc) for b in range(a + 1, nc) if ci[b] - ci[a] > msep)
    return con, nb


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


def cpu_baseline(w, n_steps):
    import numpy as np
    import oracle as O

    threads = len(os.sched_getaffinity(0))
    systems = [O.System.from_inputs(s, w.params) for s in w.systems]
    x = w.initial_x().astype(np.float64)
    v = w.initial_v(7).astype(np.float64)
    cv = w.initial_cvstate()
    t0 = time.perf_counter()
    _, _, _, used = O.run_batch(w.params, systems, w.replica_system, x, v, cv, n_steps, 0, threads)
    dt = time.perf_counter() - t0
    rate = w.n_replicas * n_steps / dt
    return {"value": rate, "unit": "replica-steps/s", "cores": int(used), "kind": "oracle",
            "sample": f"{w.n_replicas} replicas x {n_steps} Langevin steps of the same workload, "
                      f"FP64, OpenMP over replicas ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); replicas are independent, so "
              "more GPUs would each run their own batch with no communication.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import torch

    from paper_1705_02180_amd import inputs as I
    from paper_1705_02180_amd import scps

    torch.cuda.set_device(0)
    w = I.config2(n_replicas=args.replicas)
    sy = w.systems[0]
    n_con, n_nb = pair_counts(w)
    ctx = scps.Context.from_workload(w)
    ctx.set_reference_map(0, native_xyz=sy.native)
    x = torch.as_tensor(w.initial_x(), device="cuda")
    v = torch.as_tensor(w.initial_v(7), device="cuda")
    cv = torch.as_tensor(w.initial_cvstate(), device="cuda")
    step = 0
    for _ in range(args.warmup):
        ctx.step_replicas(x, v, cv, args.block, step0=step)
        step += args.block
    ctx.sync()

    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        ctx.step_replicas(x, v, cv, args.block, step0=step)
        step += args.block
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    per_launch_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    gpu_s = sum(per_launch_ms) / 1e3
    rep_steps = args.replicas * args.block * args.steps
    value = rep_steps / wall
    avg_launch_s = gpu_s / args.steps
    flops_launch = args.replicas * args.block * (n_con * FLOPS_CONTACT + n_nb * FLOPS_NONBONDED)
    achieved = flops_launch / avg_launch_s

    out = {
        "metric": METRIC, "value": value, "unit": "replica-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"chain560_fip35_shaped: {args.replicas} replicas x 560 particles, "
                               f"{n_con} contact pairs + {n_nb} LJ/Debye-Hueckel pairs, BAOAB dt=2 fs, "
                               f"{args.block} Langevin steps per benchmark step",
                   "replicas": args.replicas, "particles": sy.n, "block": args.block},
        "contact_pair_evals_per_s": value * n_con,
        "nonbonded_pair_evals_per_s": value * n_nb,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": measured_traffic(),
                     "kernel": "k_rmd_persistent", "avg_launch_ms": 1e3 * avg_launch_s},
    }
    if not args.no_plain:
        plain = run_plain(scps, torch, w, args.plain_replicas, args.plain_steps)
        out["plain"] = {"value": plain, "unit": "replica-steps/s",
                        "form": f"one replica per context, one launch sequence per Langevin step "
                                f"({args.plain_replicas} replicas x {args.plain_steps} steps)"}
        out["speedup_vs_plain"] = value / plain
    if not args.no_cpu:
        wc = I.config2(n_replicas=args.replicas)
        out["cpu_baseline"] = cpu_baseline(wc, args.cpu_steps)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
