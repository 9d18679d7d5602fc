"""Benchmark of the explicit MLS-MPM substep on one MI355X.

Workload (default): the cutting-style contact scene -- 4,194,304 particles
in a 0.8 x 0.2 x 0.8 slab on a 256^3 grid, an oriented-box blade sweeping
through it and a capsule grasper pressing on it, 500 substeps of dt = 5e-5.
One benchmark step = the whole 500-substep job from the initial state:
mpm_set_particles from device-resident inputs, the tools reset to their
initial pose, mpm_step(500) (binning, P2G, grid update, G2P of every
substep, all in the HIP library). `value` = particles x substeps / second.

Also reported on the same JSON line:
* roofline: the dominant kernel (the fused G2P2G) against the HBM peak,
  from its algorithmic bytes per launch and its mean duration measured with
  HIP events on the library's stream during the timed steps (the events
  ride on the kernels' dispatches, on every PROFILE_EVERY-th substep, a
  uniform sample over the run that keeps the events' own cost, a few us per
  event, off the other substeps; every substep launches its kernels one by
  one meanwhile); `traffic` is
  the kernel's HBM bytes per launch from hardware counters
  (profiles/k_g2p2g_<scene>_counters.md), null once its sources changed;
  `atomics` is its TCC atomic requests per launch (from
  profiles/k_g2p2g_<scene>_atomics.md) over the same live launch time,
  against the measured request rate of coalesced FP32 atomics;
* substep_roofline: the whole substep against the HBM byte model
  N x 100 B + N_act x 72 B;
* cpu_baseline: the FP64 oracle timed on the host for a bounded sample of
  the same workload (a few substeps of the full scene);
* fwd_bwd: the differentiable press (65,536 particles on 64^3, a capsule
  following a 200 x 3 per-substep velocity table, E_p = exp(theta_p)):
  mpm_rollout_forward(200, checkpoints every 20) and mpm_rollout_backward
  (gradients for theta, the velocity table and the starting state), timed
  separately, with the ratio (fwd + bwd) / fwd; fwd_bwd_keep_all is the same
  with a checkpoint (and the grid) kept at every substep;
* batch (unless --no-batch): 256 independent scenes of uneven size (16^3 ..
  40^3 particle cubes, 5.85M particles, a 64^3 grid and a capsule each)
  advanced together by one mpm_step(200) per step, as aggregate
  particle-substeps/s. It runs after the headline timing and its kernel
  timing, so the headline `roofline` covers c3 launches only; a profile of
  the headline workload alone uses --no-batch.
* solver_sweep (with --solver-sweep): the paper's solver comparison shape
  (Sec. III-D): a cube falling on a fixed 56^3 grid, N = 2^14 .. 2^22
  particles, one frame = 0.02 s: MLS-MPM and standard MPM take 10 substeps
  of 2e-3, PB-MPM one step of 0.02 with 10 or 20 constraint passes; ms per
  frame over the first frames of the fall.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-substeps/s (P2G+grid+G2P) fwd & fwd+bwd; % HBM roofline at 4M particles"
# Per-kernel events on every PROFILE_EVERY-th substep of the timed steps.
PROFILE_EVERY = 8
HBM_PEAK_GBS = 8000.0
B_PARTICLE = 100.0      # x, F, E read + x, F written per particle-substep (fused path)
B_NODE_SUBSTEP = 72.0   # P2G result write+read, reset, velocity write+read per active node
B_NODE_G2P2G = 28.0     # the fused kernel's share: velocity read 12 B + P2G result write 16 B


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_fields(name, keys):
    """Machine-readable fields of a committed counter summary under
    profiles/, or None when it is missing or the kernel's sources changed
    since the counters were taken (the summary records their SHA-256)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    want = set(keys) | {"kernel_source_sha256", "kernel_sources"}
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0] in want:
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    if set(fields) != want:
        return None
    h = hashlib.sha256()
    for f in fields["kernel_sources"].split():
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != fields["kernel_source_sha256"]:
        return None
    return {k: float(fields[k]) for k in keys}


def counted_traffic(scene_name):
    """HBM bytes per launch of the fused kernel (FETCH_SIZE + WRITE_SIZE,
    calibrated by a copy of known size), or None."""
    f = profile_fields(f"k_g2p2g_{scene_name}_counters.md", ["traffic_bytes_per_launch"])
    return None if f is None else f["traffic_bytes_per_launch"]


def counted_atomics(scene_name, avg_s):
    """Global atomic requests of the fused kernel (TCC_ATOMIC per launch)
    over its live launch time, against the measured request rate of
    coalesced FP32 atomics, or None."""
    f = profile_fields(f"k_g2p2g_{scene_name}_atomics.md",
                       ["atomic_requests_per_launch", "atomic_request_peak_per_s"])
    if f is None:
        return None
    rate = f["atomic_requests_per_launch"] / avg_s
    return {"requests_per_launch": f["atomic_requests_per_launch"], "achieved_per_s": rate,
            "peak_per_s": f["atomic_request_peak_per_s"], "frac": rate / f["atomic_request_peak_per_s"],
            "unit": "TCC atomic requests/s"}


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def oracle_substeps_per_s(scene, n_sub):
    """Wall time of the FP64 oracle's substep loop alone (scene setup and the
    read-back excluded), single-threaded."""
    import oracle as O
    o = O.Oracle(scene.n_grid, scene.dt, gravity=scene.gravity, wall_band=scene.wall_band, nu=scene.nu,
                 E_default=scene.E_default)
    o.set_particles(scene.x, scene.v, scene.C, scene.F, scene.E, scene.mass, scene.vol0)
    for k, t in enumerate(scene.tools):
        o.set_tool(k, t.type, **t.kwargs())
    t0 = time.perf_counter()
    st = o.step(n_sub)
    dt = time.perf_counter() - t0
    return dt, st


def cpu_baseline(scene, n_sub):
    """The FP64 oracle (single-threaded) on the full scene for n_sub
    substeps, plus the whole c1 run (100 substeps of 8,000 particles)."""
    from paper_2502_18437_amd import scenes
    model, threads = host_cpu()
    dt, _ = oracle_substeps_per_s(scene, n_sub)
    c1 = scenes.make("c1")
    dt1, _ = oracle_substeps_per_s(c1, c1.n_substeps)
    return {"value": scene.N * n_sub / dt, "unit": "particle-substeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sub} substeps of the full {scene.name} scene ({scene.N} particles, "
                      f"{scene.n_grid}^3 grid), FP64, one host thread, substep loop only (setup excluded); "
                      f"{dt:.1f} s",
            "host_cpu": model, "host_logical_cpus": threads,
            "c1_full_run": {"substeps": c1.n_substeps, "particles": c1.N, "seconds": dt1,
                            "particle_substeps_per_s": c1.N * c1.n_substeps / dt1}}


def batch_throughput(steps, warmup=1):
    """The batched workload: 256 independent scenes of uneven size (16^3 ..
    40^3 particle cubes, each on its own 64^3 grid with one capsule), all
    stepped by one mpm_step per benchmark step (200 substeps)."""
    import torch
    from paper_2502_18437_amd import mpm, scenes
    b = scenes.batch_c4()
    n_sub = b.n_substeps
    dev = torch.device("cuda", 0)
    x_d = torch.from_numpy(b.concat("x")).to(dev)
    sim = mpm.Simulation(b.n_grid, b.dt, gravity=b.gravity, wall_band=b.wall_band, nu=b.nu, E_default=b.E_default,
                         max_particles=b.N, n_scenes=len(b.scenes))
    log(f"[bench] batch {b.name}: {len(b.scenes)} scenes, {b.N} particles, {n_sub} substeps/step")

    def step():
        sim.set_batch_particles(b.counts, x_d, None, None, None, None, b.mass, b.vol0)
        for i, sc in enumerate(b.scenes):
            for k, t in enumerate(sc.tools):
                sim.set_tool(k, t.type, scene=i, **t.kwargs())
        sim.step(n_sub)

    for _ in range(warmup):
        step()
    sim.read_state(out={})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _, st = sim.read_state(out={}, allow_errors=True)
    info = sim.info()
    sim.close()
    per_substep = elapsed / (steps * n_sub)
    n_act = int(info["active_nodes"])
    model = b.N * B_PARTICLE + n_act * B_NODE_SUBSTEP
    return {"workload": f"{b.name}: {len(b.scenes)} scenes, {b.N} particles ({int(b.counts.min())}..{int(b.counts.max())} "
                        f"per scene), 64^3 grid each, one capsule each, {n_sub} substeps of dt={b.dt}",
            "value": b.N * n_sub * steps / elapsed, "unit": "particle-substeps/s", "ms_per_step": 1e3 * elapsed / steps,
            "steps": steps, "status": int(st), "active_nodes": n_act,
            "substep_roofline": {"bound": "hbm", "model_bytes": model, "us_per_substep": 1e6 * per_substep,
                                 "achieved": model / per_substep / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": model / per_substep / 1e9 / HBM_PEAK_GBS}}


SWEEP_SIZES = (1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 21, 1 << 22)


def solver_sweep(frames=4, lead_frames=5, sizes=SWEEP_SIZES):
    """ms per 0.02 s frame of the falling cube for each solver and size,
    timed over `frames` frames after lead_frames + 1 untimed ones (the cube
    is then falling at about 1.2 m/s and reaches the floor after the timed
    frames). The launch configuration is the library autotuner's choice from
    that state. At 2^22 particles the cube holds about 370 particles per
    cell."""
    import torch
    from paper_2502_18437_amd import mpm, scenes
    dev = torch.device("cuda", 0)
    runs = (("mls", mpm.MPM_SOLVER_MLS, 1, 10, 2e-3), ("standard_pic", mpm.MPM_SOLVER_PIC, 1, 10, 2e-3),
            ("pb10", mpm.MPM_SOLVER_PB, 10, 1, 2e-2), ("pb20", mpm.MPM_SOLVER_PB, 20, 1, 2e-2))
    out = []
    for n in sizes:
        s = scenes.scene_cube(n)
        x_d = torch.from_numpy(s.x).to(dev)
        for label, kind, iters, sub, dt in runs:
            sim = mpm.Simulation(s.n_grid, dt, gravity=s.gravity, wall_band=s.wall_band, nu=s.nu,
                                 E_default=s.E_default, max_particles=s.N)
            sim.set_particles(x_d, None, None, None, None, s.mass, s.vol0)
            sim.set_solver(kind, iters, 0.5)
            for _ in range(lead_frames):
                sim.step(sub)
            # trials long enough for the re-binning interval to matter
            log(f"[bench] sweep N={s.N} {label}: autotuning")
            cfg = sim.autotune(trial_substeps=8 if kind == mpm.MPM_SOLVER_PB else 2 * sub)
            sim.step(sub)  # one more untimed frame: graphs recorded with the chosen configuration
            sim.read_state(out={})
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(frames):
                sim.step(sub)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            _, st = sim.read_state(out={}, allow_errors=True)
            sim.close()
            passes = sub * iters
            out.append({"particles": s.N, "solver": label, "substeps_per_frame": sub, "dt": dt, "launch_config": cfg,
                        "grid_updates_per_frame": passes, "ms_per_frame": 1e3 * el / frames,
                        "particle_passes_per_s": s.N * passes * frames / el, "status": int(st)})
            log(f"[bench] sweep N={s.N} {label}: {1e3 * el / frames:.3f} ms/frame {cfg}")
    return {"workload": f"falling cube (side 0.4) on a 56^3 grid, frames of 0.02 s; frames {lead_frames + 2}.."
                        f"{lead_frames + 1 + frames} timed", "frames": frames, "runs": out}


def fwd_bwd(steps, checkpoint_every=20):
    """Time the differentiable rollout of the press scene: forward with
    checkpoints, then the reverse pass, each bracketed by device syncs."""
    import torch
    from paper_2502_18437_amd import mpm, scenes
    s = scenes.make("c5")
    T = s.n_substeps
    dev = torch.device("cuda", 0)
    theta = torch.from_numpy(s.theta).to(dev)
    x_d = torch.from_numpy(s.x).to(dev)
    rng = np.random.default_rng(0)
    xb = torch.from_numpy(rng.standard_normal((s.N, 3)).astype(np.float32)).to(dev)
    sim = mpm.Simulation(s.n_grid, s.dt, gravity=s.gravity, wall_band=s.wall_band, nu=s.nu,
                         E_default=s.E_default, max_particles=s.N)
    log(f"[bench] fwd+bwd: {s.name}, {s.N} particles, {s.n_grid}^3 grid, {T} substeps, "
        f"checkpoints every {checkpoint_every}")

    def forward():
        sim.set_particles(x_d, None, None, None, None, s.mass, s.vol0)
        for k, t in enumerate(s.tools):
            sim.set_tool(k, t.type, **t.kwargs())
        for k, tab in s.vel_tables.items():
            sim.set_tool_velocity_table(k, tab)
        sim.rollout_forward(T, checkpoint_every, theta=theta)

    def backward():
        return sim.rollout_backward(xb, want_state=False)

    forward()
    g = backward()
    torch.cuda.synchronize()
    t_f = t_b = 0.0
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_f += t1 - t0
        t_b += t2 - t1
    _, st = sim.read_state(out={}, allow_errors=True)
    ok = bool(torch.isfinite(g["theta"]).all().item()) and bool(np.isfinite(g["vel"]).all())
    sim.close()
    t_f /= steps
    t_b /= steps
    ps = s.N * T
    return {"workload": f"{s.name}: {s.N} particles, {s.n_grid}^3 grid, capsule with a {T} x 3 velocity "
                        f"table, {T} substeps of dt={s.dt}, checkpoints every {checkpoint_every}",
            "fwd_ms": 1e3 * t_f, "bwd_ms": 1e3 * t_b, "fwd_particle_substeps_per_s": ps / t_f,
            "fwd_bwd_particle_substeps_per_s": ps / (t_f + t_b), "ratio_fwd_bwd_over_fwd": (t_f + t_b) / t_f,
            "checkpoint_every": checkpoint_every, "steps": steps, "status": int(st), "finite_gradients": ok}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scene", default="c3")
    ap.add_argument("--substeps", type=int, default=0, help="substeps per step (default: the scene's)")
    ap.add_argument("--resort", type=int, default=0)
    ap.add_argument("--cpu-substeps", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-diff", action="store_true", help="skip the fwd+bwd measurement")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 256-scene batch (so that a profile of the command holds only the headline "
                         "workload's fused-kernel launches)")
    ap.add_argument("--diff-steps", type=int, default=3)
    ap.add_argument("--solver-sweep", action="store_true",
                    help="also time the three solvers on the falling cube (paper's solver comparison shape)")
    ap.add_argument("--sweep-sizes", default="",
                    help="comma-separated particle counts for --solver-sweep (default: 2^14 .. 2^22)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the solver sweep (for profiling its kernels) and print its JSON")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="run only the c5 fwd+bwd leg (checkpoints every 20) and print its JSON (for profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 256-scene batch (for profiling its kernels) and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device-to-device copy of MIB MiB (a kernel of known "
                         "traffic that scales hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_18437_amd import mpm, scenes

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sizes = tuple(int(v) for v in args.sweep_sizes.split(",") if v) or SWEEP_SIZES
    if args.sweep_only:
        print(json.dumps({"solver_sweep": solver_sweep(sizes=sizes)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_throughput(args.diff_steps)}), flush=True)
        return
    if args.fwd_bwd_only:
        print(json.dumps({"fwd_bwd": fwd_bwd(args.diff_steps, checkpoint_every=20)}), flush=True)
        return
    s = scenes.make(args.scene)
    n_sub = args.substeps or s.n_substeps
    log(f"[bench] scene {s.name}: {s.N} particles, {s.n_grid}^3 grid, {n_sub} substeps/step")

    # Inputs resident in HBM before timing.
    x_d = torch.from_numpy(s.x).to(dev)
    E_d = torch.from_numpy(s.E).to(dev) if s.E is not None else None
    sim = mpm.Simulation(s.n_grid, s.dt, gravity=s.gravity, wall_band=s.wall_band, nu=s.nu,
                         E_default=s.E_default, resort_interval=args.resort, max_particles=s.N)

    def step():
        sim.set_particles(x_d, None, None, None, E_d, s.mass, s.vol0)
        for k, t in enumerate(s.tools):
            sim.set_tool(k, t.type, **t.kwargs())
        sim.step(n_sub)

    for _ in range(args.warmup):
        step()
    sim.read_state(out={})  # synchronise and surface deferred errors
    torch.cuda.synchronize()

    if not args.no_profile:
        sim.profile(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    _, st = sim.read_state(out={})
    info = sim.info()
    prof = sim.profile_read() if not args.no_profile else None
    graphs = None
    if not args.no_profile:
        # The per-kernel events above launch every kernel; the same steps with
        # runs of substeps replayed as HIP graphs (the default when not timing
        # kernels):
        sim.profile(False)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        g_el = time.perf_counter() - g0
        graphs = {"value": s.N * n_sub * args.steps / g_el, "ms_per_step": 1e3 * g_el / args.steps,
                  "graph_chunk": sim.launch_config()["graph_chunk"]}
    sim.close()
    assert st == 0, st

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ms_per_step = 1e3 * elapsed / args.steps
    value = s.N * n_sub * args.steps / elapsed
    n_act = int(info["active_nodes"])
    per_substep_s = elapsed / (args.steps * n_sub)
    model_bytes = s.N * B_PARTICLE + n_act * B_NODE_SUBSTEP
    out = {
        "metric": METRIC, "value": value, "unit": "particle-substeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{s.name}: {s.N} particles, {s.n_grid}^3 grid, {len(s.tools)} tools, "
                               f"{n_sub} substeps of dt={s.dt}", "particles": s.N, "grid": s.n_grid,
                   "substeps_per_step": n_sub, "resort_interval": info["resort_interval"],
                   "active_nodes": n_act, "occupied_blocks": info["occupied_blocks"],
                   "active_blocks": info["active_blocks"], "fallback_particle_substeps": info["n_fallback"]},
        "substep_roofline": {"bound": "hbm", "model_bytes": model_bytes, "us_per_substep": 1e6 * per_substep_s,
                             "achieved": model_bytes / per_substep_s / 1e9, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": model_bytes / per_substep_s / 1e9 / HBM_PEAK_GBS},
    }
    if prof is not None:
        ms, n = prof["g2p2g"]
        avg_s = ms / max(n, 1) / 1e3
        bytes_launch = s.N * B_PARTICLE + n_act * B_NODE_G2P2G
        achieved = bytes_launch / avg_s / 1e9
        out["roofline"] = {"kernel": "k_g2p2g", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": counted_traffic(s.name),
                           "bytes_per_launch": bytes_launch, "avg_us": avg_s * 1e6, "launches": n,
                           "timed_every": PROFILE_EVERY,
                           "atomics": counted_atomics(s.name, avg_s)}
        out["kernel_ms"] = {k: {"total_ms": v[0], "launches": v[1],
                                "avg_us": 1e3 * v[0] / v[1] if v[1] else None} for k, v in prof.items()}
    if not args.no_batch:
        out["batch"] = batch_throughput(args.diff_steps)
    if args.solver_sweep:
        out["solver_sweep"] = solver_sweep(sizes=sizes)
    if not args.no_diff:
        out["fwd_bwd"] = fwd_bwd(args.diff_steps, checkpoint_every=20)
        out["fwd_bwd_keep_all"] = fwd_bwd(args.diff_steps, checkpoint_every=1)
    if graphs is not None:
        out["graph_replay"] = graphs
    if not args.no_cpu:
        log(f"[bench] oracle CPU baseline: {args.cpu_substeps} substeps of the full scene ...")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_substeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
