#!/usr/bin/env python3
"""Throughput of the two-belt Shan-Chen D2Q9 step on one MI355X.

Workload (default): a 2048x2048 periodic lattice, FP32 populations in SoA
planes, A1 = G1 + G2 = -4.9 with G2 = 0.1 |G1|, tau = 1, rho0 = 1, initial
density 0.7 (1 + 0.01 U(-1, 1)) from a seeded generator, fluid at rest;
moments and the section V energies every 500 steps.  One "step" is one full
lattice update t -> t+1 (pull-stream, moments, psi, 24-link force, BGK
collision, store) plus its share of the logging.

Prints one JSON line: MLUPS for the whole timed region, the effective HBM
bandwidth of the step kernel against the 8 TB/s peak (average duration from
HIP events on the library's stream), and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
BYTES_PER_LU = {"f64": 144, "f32": 72, "f16dev": 36}
METRIC = "MLUPS and achieved HBM GB/s (two-belt D2Q9 step); adjoint/forward time ratio"
TRAFFIC_FILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.txt")))
KERNEL_SRC = os.path.join(ROOT, "paper_1008_2865_amd", "csrc", "lb_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(workload_key):
    """HBM bytes per launch of the dominant kernel from a committed counter
    summary, or None if none is for this workload and the current kernel."""
    for path in TRAFFIC_FILES:
        if not os.path.exists(path):
            continue
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("workload") != workload_key:
            continue
        try:
            return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, G1, G2, seed, target_s, steps=None):
    """The oracle (FP64, OpenMP) on a bounded sample of the same workload,
    driven through the same lb_* call sequence as the GPU library (its
    host-memory entry points); then a short single-thread sample."""
    import oracle as O
    from paper_1008_2865_amd import inputs

    rho = inputs.rho_noise(n, n, seed)
    lat = O.AbiLattice(rho, G1=G1, G2=G2)
    if steps is None:
        lat.step(1)  # warm the threads and pages
        t0 = time.perf_counter()
        lat.step(2)
        one = (time.perf_counter() - t0) / 2
        steps = int(max(1, min(5000, target_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    lat.step(steps)
    dt = time.perf_counter() - t0
    threads = O.threads()
    # Single thread, about a fifth of the time budget.
    O.set_threads(1)
    t1 = time.perf_counter()
    lat.step(1)
    one1 = time.perf_counter() - t1
    s1 = int(max(1, min(1000, 0.2 * target_s / max(one1, 1e-6))))
    t1 = time.perf_counter()
    lat.step(s1)
    dt1 = time.perf_counter() - t1
    O.set_threads(threads)
    lat.close()
    return {"value": round(n * n * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} FP64 oracle through its lb_init/lb_step entry points, {steps} steps "
                      f"of the same workload (r = G2/|G1|, seed {seed}), {dt:.1f} s wall on "
                      f"{threads} threads",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread_mlups": round(n * n * s1 / dt1 / 1e6, 3),
            "cpu_gbps_at_144_B_per_LU": round(n * n * steps / dt * 144 / 1e9, 2)}


def log_point_cost(sim, le, moments, B, reps=3):
    """Extra seconds of a log point (the logged step plus lb_moments) over
    a plain step, on the library's stream: (logged step + moments + one
    plain step) against two plain steps, the pairs placed where the library
    runs them so."""
    import torch

    extra = []
    for _ in range(reps):
        sim.step(le - sim.t % le)      # to the next log point (not timed)
        a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record()
        sim.step(2)                    # the logged step and one plain step
        B.lb_moments(sim.ctx, *moments, on_device=True)
        b.record()
        sim.step(2)                    # two plain steps (one launch where paired)
        c.record()
        torch.cuda.synchronize()
        extra.append((a.elapsed_time(b) - b.elapsed_time(c)) / 1e3)
    return max(0.0, sorted(extra)[len(extra) // 2])


def adjoint_ratio(n, T, every, storage, r, seed, reps):
    """Wall time of the backward pass over the forward pass of the adjoint
    workload: gradients of L = (E(T) - E*)^2 + beta A(T) with respect to
    G1, G2 and the initial density, E* = 1.01 E(T) of the same run,
    beta = 1/n^2, eps = 1e-6, a checkpoint every `every` steps."""
    import torch

    from paper_1008_2865_amd import inputs
    from paper_1008_2865_amd.adjoint import DropletLoss

    G1, G2 = inputs.couplings(r)
    rho = inputs.rho_noise(n, n, seed)
    # A stream of its own, so the backward pass replays captured segments
    # and overlaps each segment's re-step with the adjoint steps before it.
    with torch.cuda.stream(torch.cuda.Stream()):
        dl = DropletLoss(n, n, T, E_target=0.0, beta=1.0 / n ** 2, eps=1e-6, storage=storage,
                         checkpoint_every=every)
        dl.E_target = 1.01 * dl.forward(rho, G1, G2)[1]
        dl.backward()  # warm-up pass (captures the segment graphs)
        torch.cuda.synchronize()
        fw, bw = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            L, E, A, M = dl.forward(rho, G1, G2)
            t1 = time.perf_counter()
            dG1, dG2, drho = dl.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fw.append(t1 - t0)
            bw.append(t2 - t1)
            log(f"bench: adjoint forward {fw[-1] * 1e3:.1f} ms, backward {bw[-1] * 1e3:.1f} ms")
        dl.close()
    f_s, b_s = min(fw), min(bw)
    return {"ratio": round(b_s / f_s, 3), "forward_ms": round(f_s * 1e3, 3),
            "backward_ms": round(b_s * 1e3, 3),
            "forward_mlups": round(n * n * T / f_s / 1e6, 1),
            "config": f"{n}x{n} periodic two-belt D2Q9, r={r}, seed {seed}, {storage}, T={T}, "
                      f"checkpoint every {every}, L=(E(T)-1.01 E_ref)^2 + A(T)/{n}^2, "
                      f"best of {reps} (forward: T steps + checkpoints + loss; backward: "
                      f"recomputed segments, tape, adjoint steps, gradients; the re-step of "
                      f"segment s-1 on a second stream while the adjoint steps of segment s run; "
                      f"full segments replayed from captured HIP graphs)",
            "loss": [L, E, A, M], "dG": [dG1, dG2], "drho_l2": float(torch.linalg.norm(drho))}


def copy_bandwidth(nbytes, reps=10):
    """GB/s of torch's device copy of an nbytes buffer (read + write)."""
    import torch

    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (a.elapsed_time(b) / 1e3) / 1e9


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--n", type=int, default=2048, help="lattice side")
    ap.add_argument("--storage", default="f32", choices=sorted(BYTES_PER_LU))
    ap.add_argument("--r", type=float, default=0.1, help="G2 / |G1| at A1 = -4.9")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--log-every", type=int, default=500)
    ap.add_argument("--tile-x", type=int, default=0)
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--steps-per-launch", type=int, default=0,
                    help="0: library choice; 1; 2: plain FP32 or half-storage steps two per launch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle sample length; 0 skips the CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=None)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a device copy of one population buffer (counter calibration)")
    ap.add_argument("--workload", default="single", choices=["single", "batch", "adjoint", "structure"],
                    help="single: one lattice (default, the headline workload); batch: the "
                         "96-lattice sweep of independent lattices; adjoint: gradients of the "
                         "droplet functional at 512^2 (adjoint/forward time ratio); structure: "
                         "the structure factor S(k), shell average and kbar at 512^2 and 2048^2")
    ap.add_argument("--checkpoint-every", type=int, default=100)
    ap.add_argument("--tile-y2", type=int, default=0,
                    help="batch: rows per workgroup of the two-step launches (0: tuned)")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false",
                    help="single workload: skip the adjoint/forward ratio of the 512^2 adjoint "
                         "workload that the line carries by default")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the single-GPU path only: the library has no multi-GPU "
              "code (the lattice would shard as y-slabs with a 3-row halo exchange). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1008_2865_amd import binding as B
    from paper_1008_2865_amd import inputs
    from paper_1008_2865_amd.sim import LBSim

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "structure":
        return bench_structure(args)
    n, K, W, le = args.n, args.steps, args.warmup, args.log_every
    G1, G2 = inputs.couplings(args.r)
    rho0 = inputs.rho_noise(n, n, args.seed)
    total = W + K
    sim = LBSim(rho0, G1=G1, G2=G2, storage=args.storage, log_every=le,
                max_steps=total + 5 * le + 1000, tile_x=args.tile_x, tile_y=args.tile_y,
                tile_rows=args.tile_rows, steps_per_launch=args.steps_per_launch)
    tx, ty, tr, nb = sim.launch_shape()
    tx2, ty2, nb2 = B.lb_two_step_shape(sim.p)
    two = tx2 > 0
    log(f"bench: {n}x{n} {args.storage}, r={args.r}, tile {tx}x{ty}x{tr}, {nb} workgroups, "
        + (f"two-step tile {tx2}x{ty2} ({tx2 - 6} columns out), {nb2} workgroups, " if two else "")
        + f"warmup {W}, steps {K}, log every {le}")
    moments = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in range(3)]

    def run(nsteps, pairs=None):
        done = 0
        while done < nsteps:
            t = sim.t
            chunk = min(le - t % le if le else nsteps, nsteps - done)
            if pairs is not None:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                sim.step(chunk)
                b.record()
                pairs.append((a, b, chunk))
            else:
                sim.step(chunk)
            done += chunk
            if le and sim.t % le == 0:
                B.lb_moments(sim.ctx, *moments, on_device=True)

    run(W)
    torch.cuda.synchronize()
    pairs = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = sim.t
    w0 = time.perf_counter()
    e0.record()
    run(K, pairs)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    region_s = e0.elapsed_time(e1) / 1e3
    step_s = sum(a.elapsed_time(b) for a, b, _ in pairs) / 1e3
    launches = sum(c for _, _, c in pairs)
    trace = sim.trace()
    last_e = f"{trace[-1, 2] + trace[-1, 3]:.6g}" if len(trace) else "n/a"
    log(f"bench: region {region_s * 1e3:.2f} ms (host wall {wall * 1e3:.2f} ms), "
        f"step chunks {step_s * 1e3:.2f} ms over {launches} steps; "
        f"trace rows {len(trace)}, last E = {last_e}")
    # Logging (the logged step and lb_moments, one in le steps) at its
    # workload share: a timed region shorter than le steps may hold no log
    # point, or one at a 1/K share instead of 1/le.  The extra time of a log
    # point over two plain steps is measured on its own and the region is
    # charged K/le of them in place of the ones it actually held.
    logs_in_region = sum(1 for t in range(t_start, t_start + K) if le and t % le == 0)
    log_cost = log_point_cost(sim, le, moments, B) if le else 0.0
    region_amortised = region_s + ((K / le if le else 0) - logs_in_region) * log_cost

    # The dominant kernel on its own: plain steps between two log points
    # (two per launch where the library runs them so), timed with HIP events
    # on the library's stream.
    if le and sim.t % le == 0:
        sim.step(1)  # the logged step leaving this log point
    probe = 400 if not le else min(400, (le - 1 - sim.t % le) // 2 * 2)
    pa = torch.cuda.Event(enable_timing=True)
    pb = torch.cuda.Event(enable_timing=True)
    pa.record()
    sim.step(probe)
    pb.record()
    torch.cuda.synchronize()
    per_launch_steps = 2 if two else 1
    launches_probe = probe // per_launch_steps
    avg_launch = pa.elapsed_time(pb) / 1e3 / launches_probe

    if args.copy_calib:
        nbytes = 9 * n * n * 4
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration, {nbytes} bytes read + {nbytes} bytes written per copy")

    sites = n * n
    bpl = BYTES_PER_LU[args.storage]
    value = sites * K / region_amortised / 1e6
    alg_bytes = bpl * sites * per_launch_steps
    achieved = alg_bytes / avg_launch / 1e9
    workload_key = (f"{n}x{n} {args.storage} r={args.r} "
                    + (f"two-step tile {tx2}x{ty2}" if two else f"tile {tx}x{ty}x{tr}"))
    traffic = measured_traffic(workload_key)
    copy_gbps = copy_bandwidth(bpl // 2 * sites)
    kernel = ("k_step2 (two fused pull-stream + two-belt force + BGK collide steps per launch)"
              if two else "k_step (fused pull-stream + two-belt force + BGK collide)")
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(region_amortised * 1e3 / K, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {
            "workload": f"two-belt D2Q9 Shan-Chen, {n}x{n} periodic, {args.storage} SoA populations, "
                        f"A1=-4.9, G2/|G1|={args.r}, tau=1, rho0=1, rho=0.7(1+0.01U) seed {args.seed}, "
                        f"moments + pseudo-energy every {le} steps (timed region: {K} steps holding "
                        f"{logs_in_region} log point(s), charged {K / le if le else 0:g} log points "
                        f"of {log_cost * 1e6:.1f} us each)",
            "timed_region_ms": round(region_s * 1e3, 4),
            "log_points_in_region": logs_in_region,
            "log_point_extra_us": round(log_cost * 1e6, 2),
            "nx": n, "ny": n, "storage": args.storage, "G1": G1, "G2": G2, "tau": 1.0,
            "log_every": le, "tile_x": tx, "tile_y": ty, "tile_rows": tr, "workgroups": nb,
            "steps_per_launch": per_launch_steps,
            "two_step_tile": [tx2, ty2] if two else None, "two_step_workgroups": nb2 if two else None,
        },
        "effective_gbps": round(value * bpl / 1e3, 1),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4),
            "traffic": traffic,
            "kernel": kernel,
            "algorithmic_bytes_per_launch": alg_bytes,
            "lattice_updates_per_launch": sites * per_launch_steps,
            "avg_launch_us": round(avg_launch * 1e6, 3),
            "launches_timed": launches_probe,
            "traffic_gbps": round(traffic / avg_launch / 1e9, 1) if traffic else None,
            "traffic_frac_of_peak": round(traffic / avg_launch / 1e9 / PEAK_HBM_GBPS, 4) if traffic else None,
            "device_copy_gbps": round(copy_gbps, 1),
            "traffic_frac_of_device_copy": round(traffic / avg_launch / 1e9 / copy_gbps, 4) if traffic else None,
        },
    }
    if args.adjoint:
        log("bench: adjoint/forward ratio at the adjoint workload ...")
        out["adjoint"] = adjoint_ratio(n=512, T=3000, every=100, storage="f32", r=0.1, seed=1, reps=3)
        # The same gradients with the whole run taped by the forward pass (one
        # segment, 12.6 GB of tape at 512^2 and T = 3000): no re-step.
        whole = adjoint_ratio(n=512, T=3000, every=3000, storage="f32", r=0.1, seed=1, reps=3)
        out["adjoint"]["whole_tape"] = {k: whole[k] for k in ("ratio", "forward_ms", "backward_ms")}
        out["adjoint"]["whole_tape"]["checkpoint_every"] = 3000
    if args.cpu_seconds > 0 or args.cpu_steps:
        log("bench: timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(n, G1, G2, args.seed, args.cpu_seconds, args.cpu_steps)
    sim.close()
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """The batched sweep: 96 square lattices, sizes U{128..1024}, own r and
    seed each, FP32, one launch for all of them per step (per two plain
    steps when the library runs them two per launch); plain steps are
    replayed from captured HIP graphs (the batch runs on its own stream)."""
    import torch

    from paper_1008_2865_amd import autotune, inputs
    from paper_1008_2865_amd.sim import LBBatch

    K = args.steps if args.steps != 20000 else 10000
    W, le = args.warmup, args.log_every
    spec = inputs.batched_lattices()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lats = []
        for d in spec:
            G1, G2 = inputs.couplings(d["r"])
            lats.append(dict(rho_init=inputs.rho_noise(d["n"], d["n"], d["seed"]), G1=G1, G2=G2))
        if args.tile_y:
            tx, tr, ty = args.tile_x or 128, args.tile_rows or 1, args.tile_y
        else:
            tx, tr, ty = autotune.tune_batch(lats, args.storage)
        for L in lats:
            L["tile_y"] = ty
        batch = LBBatch(lats, storage=args.storage, tile_x=tx, tile_rows=tr, log_every=le,
                        max_steps=W + K + le + 1000, steps_per_launch=args.steps_per_launch)
        sites = batch.sites
        if batch.two_step_shape()[0]:
            # The two-step tile height, timed on this batch (or given).
            if args.tile_y2:
                batch.set_two_step_tile(args.tile_y2)
            else:
                autotune.tune_batch_two_step(batch)
        tx2, ty2, nb2 = batch.two_step_shape()
        two = tx2 > 0
        log(f"bench: batch of {len(lats)} lattices, {sites} sites, tile {tx}x{ty}x{tr}, "
            + (f"two-step tile {tx2}x{ty2}, {nb2} workgroups, " if two else "")
            + f"warmup {W}, steps {K}, log every {le}")

        def run(nsteps, pairs=None):
            done = 0
            while done < nsteps:
                t = batch[0].t
                chunk = min(le - t % le if le else nsteps, nsteps - done)
                if pairs is not None:
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    batch.step(chunk)
                    b.record()
                    pairs.append((a, b, chunk))
                else:
                    batch.step(chunk)
                done += chunk

        run(W)
        torch.cuda.synchronize()
        pairs = []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run(K, pairs)
        e1.record()
        torch.cuda.synchronize()
        region_s = e0.elapsed_time(e1) / 1e3
        step_s = sum(a.elapsed_time(b) for a, b, _ in pairs) / 1e3
        launches = sum(c for _, _, c in pairs)
        rows = batch[0].trace()
        log(f"bench: region {region_s * 1e3:.2f} ms, {launches} steps, trace rows {len(rows)}")
        batch.close()
    bpl = BYTES_PER_LU[args.storage]
    value = sites * K / region_s / 1e6
    # Time per launch of the dominant kernel (logged steps included, one in
    # log_every): per step, times the steps a launch advances.
    per_launch = 2 if two else 1
    avg = step_s / launches * per_launch
    workload_key = (f"batch {len(lats)} lattices {sites} sites {args.storage} "
                    + (f"two-step tile {tx2}x{ty2}" if two else f"tile {tx}x{ty}x{tr}"))
    traffic = measured_traffic(workload_key)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(region_s * 1e3 / K, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {
            "workload": f"batched sweep: {len(lats)} independent periodic two-belt D2Q9 lattices, "
                        f"sizes U{{128..1024}}^2, G2/|G1| ~ U[0, 0.15] each at A1=-4.9, own seed "
                        f"each (master seed 4), {args.storage}, one launch for all lattices per "
                        + ("two plain steps" if two else "step")
                        + f", plain steps replayed from HIP graphs, pseudo-energy every {le}",
            "lattices": len(lats), "sites": sites, "tile_x": tx, "tile_y": ty, "tile_rows": tr,
            "steps_per_launch": per_launch, "two_step_tile": [tx2, ty2] if two else None,
            "two_step_workgroups": nb2 if two else None,
        },
        "effective_gbps": round(value * bpl / 1e3, 1),
        "roofline": {
            "bound": "hbm", "achieved": round(per_launch * bpl * sites / avg / 1e9, 1),
            "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(per_launch * bpl * sites / avg / 1e9 / PEAK_HBM_GBPS, 4),
            "traffic": traffic,
            "traffic_gbps": round(traffic / avg / 1e9, 1) if traffic else None,
            "workload_key": workload_key,
            "kernel": ("k_step2_batch (all lattices, two steps per launch)" if two
                       else "k_step_batch (all lattices, one launch per step)"),
            "algorithmic_bytes_per_launch": per_launch * bpl * sites,
            "avg_launch_us": round(avg * 1e6, 3),
        },
    }
    if args.cpu_seconds > 0 or args.cpu_steps:
        log("bench: timing the CPU oracle on a bounded sample ...")
        import oracle as O

        d = max(spec, key=lambda d: d["n"])
        G1, G2 = inputs.couplings(d["r"])
        f = O.init(inputs.rho_noise(d["n"], d["n"], d["seed"]))
        f = O.step(f, 1, 1.0, 1.0, G1, G2)
        t0 = time.perf_counter()
        f = O.step(f, 2, 1.0, 1.0, G1, G2)
        one = (time.perf_counter() - t0) / 2
        steps = args.cpu_steps or int(max(1, min(5000, args.cpu_seconds / max(one, 1e-6))))
        t0 = time.perf_counter()
        O.step(f, steps, 1.0, 1.0, G1, G2)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(d["n"] ** 2 * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": O.threads(), "kind": "oracle",
            "sample": f"largest lattice of the batch ({d['n']}x{d['n']}), FP64 oracle, {steps} steps, "
                      f"{dt:.1f} s wall"}
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Gradients of L = (E(T) - E*)^2 + beta A(T) on a 512^2 lattice (r = 0.1,
    seed 1, FP32, T = 3000 steps, a checkpoint every 100 steps, E* = 1.01 E(T)
    of the same run, beta = 1/512^2, eps = 1e-6): wall time of the forward
    pass (T steps plus checkpoint copies and the loss) and of the backward
    pass (recomputation of every segment, tape, adjoint steps, gradients)."""
    import torch

    from paper_1008_2865_amd import inputs

    n = args.n if args.n != 2048 else 512
    T = args.steps if args.steps != 20000 else 3000
    log(f"bench: adjoint {n}x{n} {args.storage}, T {T}, checkpoint every {args.checkpoint_every}")
    res = adjoint_ratio(n, T, args.checkpoint_every, args.storage, args.r, args.seed, reps=3)
    f_s, b_s = res["forward_ms"] / 1e3, res["backward_ms"] / 1e3
    L, E, A, M = res["loss"]
    G1, G2 = inputs.couplings(args.r)
    rho = inputs.rho_noise(n, n, args.seed)
    out = {
        "metric": "adjoint/forward wall-time ratio (droplet functional gradients)",
        "value": res["ratio"], "unit": "x", "n_gpus": 1, "steps": T, "warmup": 1,
        "ms_per_step": round((f_s + b_s) * 1e3 / T, 6), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": "adjoint of a " + res["config"]},
        "forward_ms": res["forward_ms"], "backward_ms": res["backward_ms"],
        "forward_mlups": res["forward_mlups"],
        "gradient_mlups": round(n * n * T / (f_s + b_s) / 1e6, 1),
        "loss": res["loss"], "dG": res["dG"], "drho_l2": res["drho_l2"],
    }
    if args.cpu_seconds > 0 or args.cpu_steps:
        log("bench: timing the oracle gradient on a bounded sample ...")
        from oracle import adjoint as OA

        steps = args.cpu_steps or 20
        t0 = time.perf_counter()
        OA.loss_and_grads(rho, G1, G2, steps, 1.0, 1.01 * E, 1.0 / n ** 2, 1e-6)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(n * n * steps / dt / 1e6, 3), "unit": "MLUPS (forward + gradient)",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{n}x{n}, {steps} steps, FP64 autograd oracle, {dt:.1f} s wall"}
    print(json.dumps(out), flush=True)


def bench_structure(args):
    """The structure factor of section IV (mean, row FFTs, transpose, column
    FFTs with |.|^2 / N, shell averages, kbar) on seeded density fields of
    512^2 and 2048^2, FP64; GPU time per evaluation from HIP events on the
    library's stream, synchronous host copies of the shells included."""
    import numpy as np
    import torch

    from paper_1008_2865_amd import binding as B
    from paper_1008_2865_amd import inputs
    from paper_1008_2865_amd.structure import StructureFactor

    reps = 50
    res = {}
    for L in (512, 2048):
        sk = StructureFactor(L)
        rho = torch.tensor(inputs.rho_noise(L, L, args.seed, amp=0.2), device="cuda")
        shell = np.empty(sk.nshell)
        counts = np.empty(sk.nshell, np.int64)
        for _ in range(3):
            B.lb_sk_compute(sk.ctx, rho, shell, counts, on_device=True)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record(sk.stream)
        for _ in range(reps):
            kbar = B.lb_sk_compute(sk.ctx, rho, shell, counts, on_device=True)
        b.record(sk.stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        gpu = a.elapsed_time(b) / 1e3 / reps
        # Bytes of the two-pass transform: rho in, row spectra out (8 + 16),
        # transpose (16 + 16), column spectra in, |.|^2 out (16 + 8), shell
        # pass (8 + 4 index bytes) per mode.
        res[L] = {"us_per_eval": round(gpu * 1e6, 2), "wall_us_per_eval": round(wall * 1e6, 2),
                  "effective_gbps": round(92 * L * L / gpu / 1e9, 1), "kbar": kbar}
        log(f"bench: S(k) L={L}: {gpu * 1e6:.1f} us (GPU), {wall * 1e6:.1f} us (wall)")
        sk.close()
    out = {
        "metric": "structure factor evaluations per second (S(k), shell average, kbar)",
        "value": round(1.0 / (res[2048]["us_per_eval"] / 1e6), 1), "unit": "evaluations/s",
        "n_gpus": 1, "steps": reps, "warmup": 3,
        "ms_per_step": round(res[2048]["us_per_eval"] / 1e3, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "structure factor of a seeded 2048x2048 density field "
                               "(0.7 (1 + 0.2 U(-1, 1))), FP64 FFTs in LDS, 1449 shells; "
                               "512x512 alongside"},
        "sizes": {str(k): v for k, v in res.items()},
    }
    if args.cpu_seconds > 0 or args.cpu_steps:
        from oracle import structure as OS

        rho = inputs.rho_noise(2048, 2048, args.seed, amp=0.2)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 10.0) or n == 0:
            Sn, _ = OS.shells(rho)
            OS.kbar(Sn)
            n += 1
        dt = (time.perf_counter() - t0) / n
        out["cpu_baseline"] = {"value": round(1.0 / dt, 3), "unit": "evaluations/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"2048x2048, {n} evaluations of the numpy oracle, {dt:.2f} s each"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
