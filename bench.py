"""Throughput of the batched kinematic step on one MI355X.

Default workload: 1024 environments of procedural apartments with 20k-80k
triangles each, 128x128 24-bit depth, 65 collision spheres, 8 object boxes
(the paper-scale step).  Three paths are timed on the same batch:
  plain     default launch configuration, eager kernel launches;
  batched   autotuned launch configuration, persistent work queue, hipGraph;
  batched+surrogate  as batched, with the learned static-collision pre-filter
            (trained beforehand on rollouts of other scenes, calibrated on
            held-out scenes, 1-in-16 skipped queries audited).
Prints one JSON line; `value` is the batched+surrogate throughput.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12          # 39.32
# forward flops of one surrogate query: 2112 -> 256 -> 256 -> 256 -> 256 -> 1
SURROGATE_FLOP_PER_ROW = 2 * (2112 * 256 + 3 * 256 * 256 + 256)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Tuning keys a counter record must match: every raster setting that changes
# what the kernel reads and writes or how its pixels are spread over lanes and
# waves (the queue order changes neither bytes nor instructions).
TRAFFIC_KEYS = ("block", "region", "lane_max", "small_max", "occlusion", "prologue", "refresh", "persistent",
                "split", "bin")
TUNING_DEFAULTS = {"bin": 0}   # settings that older records leave out
VALU_KEYS = TRAFFIC_KEYS


def counter_record(kernel_sources, record, tuning, field, keys=None):
    """One per-launch figure (HBM bytes from FETCH_SIZE / WRITE_SIZE, VALU
    instructions from SQ_INSTS_VALU) from a committed rocprofv3 counter
    record of the launch configuration being timed, or None when the kernel
    source changed since the counters were taken or no record has this
    configuration."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                for f in kernel_sources)).hexdigest()
    if rec.get("source_sha256") != h:
        return None
    for r in rec["records"]:
        if field in r and all(r["tuning"].get(k, TUNING_DEFAULTS.get(k)) == tuning.get(k, TUNING_DEFAULTS.get(k))
                              for k in (keys or TRAFFIC_KEYS)):
            return r[field]
    return None


# multiply-adds per env of the policy encoder and heads (128x128 depth):
# conv 8x8/4 -> 31x31x32, conv 4x4/2 -> 14x14x64, conv 3x3/1 -> 12x12x32,
# fc 4608 -> 512, heads 519 -> 9 + 1
POLICY_MAC_PER_ENV = 961 * 32 * 64 + 196 * 64 * 512 + 144 * 32 * 576 + 4608 * 512 + 519 * 10


def policy_record(gal, torch, b, out, act_buf, N, steps, stream):
    """Policy inference on the step's depth output (in place): mean time of
    one call for all envs, and the rollout loop (inference then step, the
    policy writing the actions the step reads) in env-steps/s."""
    pol = gal.Policy(N, act_dim=9, seed=1)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    reps = 50
    noise = torch.randn((max(reps, steps), N, 9), generator=g, device="cuda")
    val = torch.empty(N, device="cuda")
    lp = torch.empty(N, device="cuda")
    for k in range(5):
        pol.act(out["depth"], out["state"], act_buf, noise=noise[k], value=val, logp=lp)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(reps):
        pol.act(out["depth"], out["state"], act_buf, noise=noise[k], value=val, logp=lp)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    flop = 2.0 * N * POLICY_MAC_PER_ENV
    for k in range(5):
        pol.act(out["depth"], out["state"], act_buf, noise=noise[k])
        b.step(act_buf, out)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(steps):
        pol.act(out["depth"], out["state"], act_buf, noise=noise[k])
        b.step(act_buf, out)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    train = ppo_record(gal, torch, b, out, act_buf, N, stream)
    return {"params": pol.num_params, "envs": N, "forward_ms": round(fwd_ms, 4),
            "flop_per_call": int(flop), "achieved_tflops": round(flop / (fwd_ms / 1e3) / 1e12, 1),
            "mfma_peak_tflops": BF16_PEAK_TFLOPS,
            "mfma_frac": round(flop / (fwd_ms / 1e3) / 1e12 / BF16_PEAK_TFLOPS, 4),
            "rollout_env_steps_per_s": round(N * steps / (loop_ms / 1e3), 1),
            "rollout_ms_per_step": round(loop_ms / steps, 4),
            "rollout": "policy inference + step (the step's tuning as timed above)",
            "train": train}


def ppo_record(gal, torch, b, out, act_buf, N, stream, T=64, minibatches=2, iters=2):
    """The paper's training loop on one GPU (Section 4.2: rollouts of 64
    steps, 2 minibatches, 1 epoch per update): the policy drives the step for
    T steps, its observations kept on the device; GAE; one PPO gradient and
    Adam step per minibatch (half of the rollout each).  Reward: +0.01 per
    accepted move, -0.1 per rejected one (a stand-in; the task reward is not
    built).  Env-steps/s over whole iterations."""
    mb = T * N // minibatches
    pol = gal.Policy(mb, act_dim=9, seed=2)
    R = 128 * 128
    obs = torch.empty((T, N * R), dtype=torch.int32, device="cuda")
    st = torch.empty((T, N, 10), device="cuda")
    acts = torch.empty((T, N, 9), device="cuda")
    logp = torch.empty((T, N), device="cuda")
    val = torch.empty((T, N), device="cuda")
    rew = torch.empty((T, N), device="cuda")
    done = torch.empty((T, N), dtype=torch.uint8, device="cuda")
    last = torch.empty(N, device="cuda")
    adv = torch.empty((T, N), device="cuda")
    ret = torch.empty((T, N), device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(9)
    noise = torch.randn((T, N, 9), generator=g, device="cuda")
    stats = torch.empty(4, device="cuda")

    def iteration():
        for t in range(T):
            obs[t].copy_(out["depth"])
            st[t].copy_(out["state"])
            pol.act(out["depth"], out["state"], acts[t], noise=noise[t], value=val[t], logp=logp[t])
            act_buf.copy_(acts[t])
            b.step(act_buf, out)
            rew[t] = out["accepted"].float() * 0.11 - 0.1
            done[t] = out["done"]
        pol.act(out["depth"], out["state"], act_buf, value=last)
        gal.gae(rew, val, done, last, 0.99, 0.95, adv, ret)
        per = T // minibatches
        for k in range(minibatches):
            sl = slice(k * per, (k + 1) * per)
            pol.ppo_gradients(obs[sl], st[sl].reshape(-1, 10), acts[sl].reshape(-1, 9), logp[sl].reshape(-1),
                              adv[sl].reshape(-1), ret[sl].reshape(-1), stats=stats, samples=mb)
            pol.adam_step(2.5e-4)

    iteration()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(iters):
        iteration()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    s = stats.cpu().numpy()
    return {"rollout_len": T, "envs": N, "minibatches": minibatches, "epochs": 1, "minibatch_samples": mb,
            "ms_per_iteration": round(ms, 3), "env_steps_per_s": round(T * N / (ms / 1e3), 1),
            "last_stats": {"policy_loss": float(s[0]), "value_mse": float(s[1]), "entropy": float(s[2]),
                           "mean_ratio": float(s[3])}}


def host_threads():
    """Threads the CPU baseline may use: the cores this process may run on,
    at most 16 (the host share of one GPU on a shared box)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail)), avail


def cpu_rate(cfg, robot, scenes, consts, threads, seconds, sample_envs):
    """Env-steps/s of the CPU oracle, as is, stepping `sample_envs` envs of the
    workload (one oracle batch per env) on `threads` threads for ~`seconds`."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_2306_07552_amd import scenegen as sg
    envs = list(range(min(sample_envs, scenes.num_envs)))
    with ThreadPoolExecutor(threads) as ex:
        obs = list(ex.map(lambda e: O.OracleBatch(robot, scenes, consts, envs=[e],
                                                  color=cfg.color), envs))
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
    return done / dt, len(envs), k, dt


def cpu_baseline(cfg, robot, scenes, consts, seconds=10.0, sample_envs=32):
    """The CPU oracle, as is, on a bounded sample of the same workload: on
    every core it may use (capped at 16), and on one thread."""
    threads, avail = host_threads()
    v, n, k, dt = cpu_rate(cfg, robot, scenes, consts, threads, seconds, sample_envs)
    v1, n1, k1, dt1 = cpu_rate(cfg, robot, scenes, consts, 1, seconds / 2, min(sample_envs, 8))
    return dict(value=round(v, 1), unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n} envs of the same workload x {k} steps ({dt:.1f} s) on {threads} threads",
                nproc=os.cpu_count(), affinity_cores=avail,
                one_thread=dict(value=round(v1, 1), sample=f"{n1} envs x {k1} steps ({dt1:.1f} s)"))


def train_surrogate(cfg, robot, consts, n_train_envs=2048):
    """Surrogate trained and calibrated on rollouts of scenes the benchmark
    does not use."""
    from paper_2306_07552_amd import surrogate
    base = cfg.num_envs
    return surrogate.fit(robot, consts, cfg, range(base, base + n_train_envs),
                         range(base + n_train_envs, base + n_train_envs + 512),
                         max_rows=max(4096, cfg.num_envs))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed passes of --steps steps per path; the median is reported")
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-policy", action="store_true",
                    help="skip the policy-inference and rollout-loop measurement")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against known bytes) and exit")
    ap.add_argument("--tuning", type=str, default=None,
                    help="JSON dict of raster launch settings (gal_tuning fields) for the plain path")
    ap.add_argument("--batched-tuning", type=str, default=None,
                    help="JSON dict of gal_tuning fields for the batched paths instead of running "
                         "the autotuner (profiling runs use this so every raster dispatch of the "
                         "batched paths has one configuration)")
    ap.add_argument("--sweep-tunings", type=str, default=None,
                    help="JSON list of gal_tuning dicts: run --steps untimed steps with each (after "
                         "--warmup) and exit; for counter runs (rocprofv3 --pmc) over several "
                         "launch configurations in one process, raster dispatches in list order")
    ap.add_argument("--sweep-surrogate", action="store_true",
                    help="with --sweep-tunings: attach an untrained surrogate that skips nothing")
    ap.add_argument("--work-counters", action="store_true",
                    help="with --sweep-tunings: print the raster's on-device work counters per step")
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
    N = b.num_envs
    out = b.alloc_outputs()

    # actions for every step, resident in HBM before timing; each step copies
    # its actions into the one buffer the policy would write
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg.seed)
    lim = torch.tensor([cfg.act_lim[0], cfg.act_lim[1]] + [cfg.act_lim[2]] * 7,
                       dtype=torch.float32, device="cuda")
    total = args.warmup + args.steps
    acts = (torch.rand((total, N, 9), generator=g, device="cuda") * 2 - 1) * lim
    if cfg.manip:
        # grasp / release intent on 60 % of steps, a stop action on 0.2 %
        u = torch.rand((total, N, 2), generator=g, device="cuda")
        acts = torch.cat([acts, torch.stack([(u[..., 0] < 0.6), (u[..., 1] < 0.002)], -1).float()], -1)
    act_buf = torch.empty((N, acts.shape[-1]), dtype=torch.float32, device="cuda")

    def run(k0, n):
        for k in range(k0, k0 + n):
            act_buf.copy_(acts[k], non_blocking=True)
            b.step(act_buf, out)

    if args.sweep_tunings:
        sweep = json.loads(args.sweep_tunings)
        if args.sweep_surrogate:
            # an untrained network that skips nothing: the inference kernel's
            # cost does not depend on the weights
            mlp = gal.Mlp(max_rows=N, seed=1)
            b.attach_surrogate(mlp, 0.0, audit_period=0)
        counts = []
        for tun in sweep:
            b.set_tuning(**tun)
            if args.work_counters:
                b.counters(True)
            run(0, args.warmup + args.steps)
            torch.cuda.synchronize()
            if args.work_counters:
                c = b.counters_read()
                b.counters(False)
                counts.append({k: v / (args.warmup + args.steps) for k, v in c.items()})
        print(json.dumps({"sweep": [b_t for b_t in sweep], "warmup": args.warmup,
                          "steps": args.steps, "surrogate": bool(args.sweep_surrogate),
                          "work_counters_per_step": counts or None}), flush=True)
        return

    def timed_pass(label):
        """Warmup, then `repeats` passes of exactly K timed steps, each
        bracketed by device syncs; the median pass is reported."""
        run(0, args.warmup)
        torch.cuda.synchronize()
        times = []
        for rep in range(args.repeats):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            w0 = time.perf_counter()
            ev0.record(stream)
            run(args.warmup, args.steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - w0
            times.append(ev0.elapsed_time(ev1))
            log(f"{label} pass {rep}: {args.steps} steps in {times[-1]:.2f} ms device, "
                f"{wall * 1e3:.2f} ms wall")
        pass_ms[label] = [round(t, 3) for t in times]
        return sorted(times)[len(times) // 2]

    pass_ms = {}

    def kernel_times():
        """Per-stage durations over a profiled pass (HIP events on the step stream):
        the surrogate's kernels, the robot step and the raster kernel."""
        b.profile(True)
        run(args.warmup, args.steps)
        torch.cuda.synchronize()
        b.profile(False)
        sur_ms, robot_ms, raster_ms, nsteps = b.profile_read_stages()
        return sur_ms / nsteps, robot_ms / nsteps, raster_ms / nsteps

    def path_record(ms, tuning, sur_ms, robot_ms, raster):
        return {"value": round(N * args.steps / (ms / 1e3), 1),
                "ms_per_step": round(ms / args.steps, 4), "tuning": tuning,
                "surrogate_ms": round(sur_ms, 5), "robot_ms": round(robot_ms, 5),
                "pre_raster_ms": round(sur_ms + robot_ms, 5), "raster_ms": round(raster, 5)}

    # ---- plain step
    plain_ms = timed_pass("plain")
    plain = path_record(plain_ms, b.get_tuning(), *kernel_times())

    # ---- batched step: autotuned configuration, persistent queue, graph replay
    act_buf.copy_(acts[0])
    if args.batched_tuning:
        b.set_tuning(**json.loads(args.batched_tuning))
        log(f"batched tuning given: {b.get_tuning()}")
    else:
        best, best_ms = b.autotune(act_buf, out, steps=5)
        log(f"autotuned {best} ({best_ms:.4f} ms/step in the tuner)")
    b.set_tuning(graph=1)
    batched_ms = timed_pass("batched")
    sur_k, robot_k, raster_k = kernel_times()
    batched = path_record(batched_ms, b.get_tuning(), sur_k, robot_k, raster_k)

    # ---- batched + surrogate
    sur = None
    headline_ms = batched_ms
    launch = (("persistent queue" if batched["tuning"]["persistent"] else "one workgroup per item")
              + (f", {batched['tuning']['split']} envs split" if batched["tuning"].get("split") else ""))
    path = f"batched (autotuned: {launch}, hipGraph)"
    if not args.no_surrogate and not cfg.manip:
        mlp, skip_below, info = train_surrogate(cfg, robot, consts)
        log(f"surrogate: {info}")
        b.attach_surrogate(mlp, skip_below, audit_period=16)
        b.surrogate_stats(reset=True)
        sur_ms = timed_pass("batched+surrogate")
        st = b.surrogate_stats(reset=True)
        sur_s, robot_s, raster_s = kernel_times()
        sur = path_record(sur_ms, b.get_tuning(), sur_s, robot_s, raster_s)
        sur.update(skip_below=skip_below, calibration=info,
                   stats_timed_region=st,
                   skipped_fraction=round(st["skipped"] / max(st["queries"], 1), 4),
                   mismatch_rate=st["mismatches"] / max(st["audited"], 1))
        headline_ms = sur_ms
        path = f"batched+surrogate (autotuned: {launch}, hipGraph, 1/16 audit)"

    value = N * args.steps / (headline_ms / 1e3)
    raster_head = sur["raster_ms"] if sur else raster_k
    tuning = b.get_tuning()
    mi = b.mesh_info()
    # algorithmic bytes of one raster launch (what a rasteriser without a
    # culling hierarchy reads and writes): 12 B per triangle (3 indices) and
    # per scene vertex (3 floats), 4 B per depth pixel (+ 3 B of colour)
    tris = int(scenes.tri_offset[-1])
    verts = int(scenes.vert_offset[-1])
    raster_bytes = 12 * tris + 12 * verts + (7 if cfg.color else 4) * b.depth_pixels
    achieved = raster_bytes / (raster_head / 1e3) / 1e9
    kernel = "k_raster_persistent" if tuning["persistent"] else "k_raster"
    traffic = valu = None
    if args.config == 1 and not cfg.color:
        srcs = ["paper_2306_07552_amd/csrc/k_raster.hip", "paper_2306_07552_amd/csrc/gal_raster.h"]
        traffic = counter_record(srcs, "k_raster_1024env_128px_traffic.json", tuning,
                                 "traffic_bytes_per_launch")
        valu = counter_record(srcs, "k_raster_1024env_128px_sq.json", tuning,
                              "sq_insts_valu_per_launch", VALU_KEYS)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel, "algorithmic_bytes_per_launch": int(raster_bytes),
                "algorithmic_bytes": "12 B x triangles + 12 B x scene vertices + "
                                     + ("7" if cfg.color else "4") + " B x pixels",
                "avg_launch_ms": round(raster_head, 5),
                "culled_traffic_frac": (round(traffic / raster_bytes, 4) if traffic else None),
                "mesh": mi}
    # issue-rate bound: one wave64 VALU instruction per CU per clock
    # (4 SIMDs x 16 lanes), 256 CUs at 2.4 GHz = 39.3 T lane-ops/s
    alu_peak = VALU_PEAK_TOPS
    if valu:
        alu_ach = valu * 64 / (raster_head / 1e3) / 1e12
        roofline["alu"] = {"achieved": round(alu_ach, 2), "peak": alu_peak,
                           "unit": "T VALU lane-ops/s", "frac": round(alu_ach / alu_peak, 4),
                           "sq_insts_valu_per_launch": valu}
    else:
        roofline["alu"] = None
    if roofline["alu"] and roofline["alu"]["frac"] > roofline["frac"]:
        roofline["binding"] = "alu"
    else:
        roofline["binding"] = "hbm"
    if sur:
        flop = N * SURROGATE_FLOP_PER_ROW
        roofline["surrogate"] = {
            "bound": "mfma", "kernels": "features + MLP inference + routing",
            "flop_per_step": flop, "stage_ms": sur["surrogate_ms"],
            "achieved": round(flop / (sur["surrogate_ms"] / 1e3) / 1e12, 2),
            "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(flop / (sur["surrogate_ms"] / 1e3) / 1e12 / BF16_PEAK_TFLOPS, 5)}

    # ---- the policy that consumes the depth stack in place, and the rollout
    # loop it drives (policy inference + step)
    policy = None
    if not args.no_policy and not cfg.manip and int(max(scenes.res)) == int(min(scenes.res)) == 128:
        policy = policy_record(gal, torch, b, out, act_buf, N, args.steps, stream)
        log(f"policy: {policy}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(cfg, robot, scenes, consts)

    res = {"metric": "env-steps/sec @1024 envs, 128x128 depth: plain vs batched+surrogate, "
                     "0 mismatches",
           "value": round(value, 1), "unit": "env-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(headline_ms / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+i32 (surrogate bf16)", "data": "synthetic",
           "config": {"workload": cfg.name, "envs": N, "res": int(cfg.res0),
                      "tris_total": int(scenes.tri_offset[-1]), "spheres": robot.num_spheres,
                      "objects": cfg.num_objects, "episode_len": cfg.episode_len,
                      "path": path},
           "roofline": roofline, "cpu_baseline": cpu,
           "plain": plain, "batched": batched, "batched_surrogate": sur, "policy": policy,
           "timing": {"repeats": args.repeats, "reported": "median pass",
                      "pass_ms": pass_ms}}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
