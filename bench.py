"""Throughput of the batched kinematic step on one MI355X.

Default workload: 1024 environments of procedural apartments with 20k-80k
triangles each, 128x128 24-bit depth, 65 collision spheres, 8 object boxes
(the paper-scale plain step).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic(kernel_sources, record):
    """HBM bytes per launch from a committed FETCH_SIZE / WRITE_SIZE record,
    or None when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                for f in kernel_sources)).hexdigest()
    return rec["traffic_bytes_per_launch"] if rec.get("source_sha256") == h else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(cfg, robot, scenes, consts, seconds=10.0, sample_envs=32):
    """The CPU oracle, as is, on a bounded sample of the same workload."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_2306_07552_amd import scenegen as sg
    threads = max(1, min(16, os.cpu_count() or 1))
    envs = list(range(min(sample_envs, scenes.num_envs)))
    # per-env oracle objects, built in parallel (setup, not timed)
    with ThreadPoolExecutor(threads) as ex:
        obs = list(ex.map(lambda e: O.OracleBatch(robot, scenes, consts, envs=[e]), envs))
    t0 = time.perf_counter()
    done = 0
    k = 0
    with ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < seconds:
            a = sg.actions(cfg, k)
            list(ex.map(lambda i: obs[i].step(a[envs[i]:envs[i] + 1]), range(len(envs))))
            done += len(envs)
            k += 1
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{len(envs)} envs of the same workload x {k} steps ({dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against known bytes) and exit")
    ap.add_argument("--tuning", type=str, default=None,
                    help="JSON dict of raster launch settings (gal_tuning fields)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: the step shards by "
                          "environment with no communication, and only the 1-GPU figure is "
                          "measured", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2306_07552_amd import gal, scenegen as sg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_reference:
        n = args.copy_reference * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes": n * 4, "dispatches": 5}), flush=True)
        return

    cfg = sg.CONFIGS[args.config]
    t = time.perf_counter()
    scenes = sg.make_scene_set(cfg)
    robot = sg.make_robot_for(cfg)
    consts = sg.config_constants(cfg)
    log(f"scenes: {scenes.num_envs} envs, {int(scenes.tri_offset[-1])} triangles "
        f"({time.perf_counter() - t:.1f} s)")
    t = time.perf_counter()
    b = gal.Batch(robot, scenes, consts, color=cfg.color)
    log(f"gal_create_batch: {time.perf_counter() - t:.1f} s, mesh {b.mesh_info()}")
    if args.tuning:
        b.set_tuning(**json.loads(args.tuning))
    log(f"plain tuning {b.get_tuning()}")
    N = b.num_envs
    out = b.alloc_outputs()

    # actions for every step, resident in HBM before timing
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg.seed)
    lim = torch.tensor([cfg.act_lim[0], cfg.act_lim[1]] + [cfg.act_lim[2]] * 7,
                       dtype=torch.float32, device="cuda")
    total = args.warmup + args.steps
    acts = (torch.rand((total, N, 9), generator=g, device="cuda") * 2 - 1) * lim

    act_buf = torch.empty((N, 9), dtype=torch.float32, device="cuda")

    def run(k0, n):
        for k in range(k0, k0 + n):
            act_buf.copy_(acts[k], non_blocking=True)
            b.step(act_buf, out)

    def timed_pass(label):
        """Warmup, then exactly K timed steps bracketed by device syncs."""
        run(0, args.warmup)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        ev0.record(stream)
        run(args.warmup, args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        gpu_ms = ev0.elapsed_time(ev1)
        log(f"{label}: {args.steps} steps in {gpu_ms:.2f} ms device, {wall * 1e3:.2f} ms wall")
        return gpu_ms

    def kernel_times():
        """Per-kernel durations over a profiled pass (HIP events on the step stream)."""
        b.profile(True)
        run(args.warmup, args.steps)
        torch.cuda.synchronize()
        b.profile(False)
        robot_ms, raster_ms, nsteps = b.profile_read()
        return robot_ms / nsteps, raster_ms / nsteps

    # ---- plain step: default launch configuration, eager launches
    plain_ms = timed_pass("plain")
    plain_robot, plain_raster = kernel_times()
    plain = {"value": round(N * args.steps / (plain_ms / 1e3), 1),
             "ms_per_step": round(plain_ms / args.steps, 4), "tuning": b.get_tuning(),
             "robot_ms": round(plain_robot, 5), "raster_ms": round(plain_raster, 5)}

    # ---- batched step: autotuned configuration, persistent queue, graph replay
    act_buf.copy_(acts[0])
    best, best_ms = b.autotune(act_buf, out, steps=3)
    b.set_tuning(graph=1)
    log(f"autotuned {best} ({best_ms:.4f} ms/step in the tuner)")
    batched_ms = timed_pass("batched")
    robot_k, raster_k = kernel_times()
    value = N * args.steps / (batched_ms / 1e3)
    ms_per_step = batched_ms / args.steps

    mi = b.mesh_info()
    raster_bytes = mi["clusters"] * 48 + mi["cluster_verts"] * 12 + mi["tris"] * 4 + 4 * b.depth_pixels
    achieved = raster_bytes / (raster_k / 1e3) / 1e9
    traffic = None
    if args.config == 1 and not cfg.color:
        traffic = measured_traffic(["paper_2306_07552_amd/csrc/k_raster.hip",
                                    "paper_2306_07552_amd/csrc/gal_internal.h"],
                                   "k_raster_1024env_128px_traffic.json")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_raster", "algorithmic_bytes_per_launch": int(raster_bytes),
                "avg_launch_ms": round(raster_k, 5)}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(cfg, robot, scenes, consts)

    res = {"metric": "env-steps/sec @1024 envs, 128x128 depth (batched step; plain beside it)",
           "value": round(value, 1), "unit": "env-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+i32", "data": "synthetic",
           "config": {"workload": cfg.name, "tuning": b.get_tuning(), "envs": N, "res": int(cfg.res0),
                      "tris_total": int(scenes.tri_offset[-1]), "spheres": robot.num_spheres,
                      "objects": cfg.num_objects, "episode_len": cfg.episode_len,
                      "path": "batched (autotuned, persistent queue, hipGraph)"},
           "roofline": roofline, "cpu_baseline": cpu, "plain": plain,
           "batched": {"tuning": b.get_tuning(), "robot_ms": round(robot_k, 5),
                       "raster_ms": round(raster_k, 5)}}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
