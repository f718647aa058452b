#!/usr/bin/env python3
"""Throughput of the batched XPBD step on one MI355X.

A "step" is one simulation step (dt = 1/60 s: 10 substeps, each with the
prediction, `iterations` colour sweeps over the edge-distance and
tetrahedral-volume constraints, the tool push-out and the velocity update)
of every environment of the batch.  The default workload is 1024 identical
16x10x4 slabs (935 particles, 3200 tetrahedra), per-environment compliances
log-uniform in [1e-7, 1e-5], per-environment seeded tool paths, 8 iterations,
1000 steps.  Inputs are resident in GPU memory before the timed region; the
timed region is K consecutive xpbd_step launches bracketed by HIP events on
the batch's stream.

Prints one JSON line with the throughput in environment-substeps per second,
the roofline of the step kernel and the FP64 oracle timed on the host cores
on a bounded sample of the same workload.

    python bench.py [--steps 1000] [--warmup 20] [--workload batch|uneven|single|rl]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "env-substeps/s at fixed constraint residual, plain vs learned warm-start"

# Algorithmic work of one projection / particle update, as written in the kernel
# (an FMA counts 2 flops; rsq and rcp count 1):
FLOPS_EDGE = 34        # distance constraint (Eq. 1, compliance form)
FLOPS_TET = 115        # volume constraint (Eqs. 2-3, compliance form)
FLOPS_PARTICLE = 18    # prediction + velocity update of a free particle, per substep
# Algorithmic LDS bytes: particle records (position + inverse mass, 16 B) read,
# positions (12 B) written, multiplier read + written, constraint record read.
LDS_EDGE = 2 * 16 + 2 * 12 + 2 * 4 + 8      # 72 B
LDS_TET = 4 * 16 + 4 * 12 + 2 * 4 + 12      # 132 B
LDS_PARTICLE = 16 + 16 + 16 + 16            # predict read + write, velocity read, + lambda reset share
# of which written (positions, the multiplier; the particle's position and velocity)
LDS_EDGE_W = 2 * 12 + 4
LDS_TET_W = 4 * 12 + 4
LDS_PARTICLE_W = 32
# Algorithmic HBM bytes per environment and launch: positions and velocities in
# and out (48 B per particle), inverse masses (4 B), tool poses (12 B per tool and step).
HBM_PARTICLE = 48 + 4

CLOCK = 2.4e9                                # peak engine clock, Hz
CUS = 256
PEAK_FP32 = 157.3e12                         # published FP32 vector peak (packed FP32 issue)
PEAK_FP32_NONPACKED = CUS * 64 * 2 * CLOCK   # 78.6 TFLOP/s: 256 CU x 64 lanes x FMA x 2.4 GHz
PEAK_HBM = 8.0e12                            # B/s
COLOURINGS = ["greedy", "largest-first", "waves", "capped-256", "capped-128", "capped-256-where-it-fits"]
LDS_PEAK_RECORD = "lds_peak.json"            # measured LDS bytes per clock per CU (--lds-peak)
LDS_ASSUMED_B_PER_CLK = 128.0                # used only when no measurement is recorded


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed steps")
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps first")
    ap.add_argument("--workload", choices=["batch", "uneven", "single", "rl"], default="batch",
                    help="rl: the RL-style step (observations, policy network, tool motion, "
                         "grasping and the simulation step of 12x8x3 slabs with two tools)")
    ap.add_argument("--envs", type=int, default=0,
                    help="environments (0: 1024 for the batch workload, 4096 for the uneven one, "
                         "8192 for the RL-style step)")
    ap.add_argument("--seed", type=int, default=0,
                    help="seed of the workload's draws (compliances, tool paths, RL starts and "
                         "policy); the learned leg trains on seed + 1")
    ap.add_argument("--steps-per-launch", type=int, default=1)
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0 = library's choice)")
    ap.add_argument("--variant", type=int, default=0,
                    help="0 = library's choice, 1 = multipliers in registers, 2 = multipliers in LDS")
    ap.add_argument("--packing", type=int, default=0,
                    help="0 = library's choice, 1 = id order, 2 = 8-lane bank groups, 3 = 16-lane, "
                         "4 = scattered + 16-lane, 5 = searched")
    ap.add_argument("--colouring", type=int, default=None,
                    help="constraint colouring (a Gauss-Seidel order; the oracle takes the same): "
                         "0 = greedy (the library's default), 1 = largest first, 2 = largest "
                         "first with colours of 65..100 cut to one wave of 64, 3 = largest first "
                         "with colours capped at 256 members, 4 = the same capped at 128, "
                         "5 = per mesh: 3 where its colours fit the register variant's 64 "
                         "rounds, else 1 (default: one colour per round of the workload's "
                         "workgroups: 3 for the batch and single workloads (256 threads), 4 "
                         "for the RL workload (128 threads), 1 for the uneven workload, whose "
                         "largest meshes a cap would push past 64 rounds; 5 measured slower "
                         "there)")
    ap.add_argument("--group", type=int, default=0,
                    help="environments per workgroup (0 = library's choice, 1 or 2)")
    ap.add_argument("--cpu-envs", type=int, default=64, help="oracle sample: environments")
    ap.add_argument("--cpu-steps", type=int, default=100, help="oracle sample: steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", type=int, default=0, metavar="STEPS",
                    help="time the library's launch configurations for STEPS steps each "
                         "(xpbd_autotune) and bench the fastest (0: the default configuration)")
    ap.add_argument("--tool-shape", choices=["sphere", "capsule"], default="sphere",
                    help="spheres against particles, or 2 cm capsules against the surface "
                         "faces (one environment per workgroup)")
    ap.add_argument("--tool-lift", type=float, default=0.0, metavar="M",
                    help="raise every tool pose by M metres (1.0: no contact anywhere)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm-start leg (training + timed learned steps)")
    ap.add_argument("--learned-steps", type=int, default=100, help="timed learned steps")
    ap.add_argument("--learned-min", type=int, default=2,
                    help="sweeps before the residual check of the learned solver")
    ap.add_argument("--learned-stall", type=float, default=0.9,
                    help="the fallback sweeps stop once one lowers the residual by less than "
                         "this factor (0: run to the maximum)")
    ap.add_argument("--learned-quantile", type=float, default=0.99,
                    help="the fallback threshold is this quantile of the plain solver's "
                         "residual over the warm-up steps")
    ap.add_argument("--train-envs", type=int, default=128, help="environments of the training run")
    ap.add_argument("--train-records", type=int, default=24,
                    help="recorded substeps (one per step) of the training run")
    ap.add_argument("--train-steps", type=int, default=1500, help="Adam steps")
    ap.add_argument("--lds-peak", action="store_true",
                    help="only run the LDS bandwidth probe (16-byte reads, 12-byte writes) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one plain device copy of MIB mebibytes (reference for the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.colouring is None:
        args.colouring = {"uneven": 1, "rl": 4}.get(args.workload, 3)
    return args


def lds_peaks():
    """(read, write) LDS bytes per clock per CU: the conflict-free 16-byte read
    and 12-byte write rates measured by the library's probe (recorded in
    profiles/), else the assumed figure for both."""
    path = os.path.join(ROOT, "profiles", LDS_PEAK_RECORD)
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        return float(rec["read_b128_bytes_per_clk_per_cu"]), float(rec["write_b96_bytes_per_clk_per_cu"]), True
    return LDS_ASSUMED_B_PER_CLK, LDS_ASSUMED_B_PER_CLK, False


def host_threads(work_items):
    """Threads for the oracle's CPU baseline: every CPU this process may run on,
    capped by OMP_NUM_THREADS where the host sets it (a shared host may set it
    to the core share one GPU's jobs get), and by the work items.  Returns the
    count and a description of the host."""
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    share = os.environ.get("OMP_NUM_THREADS")
    cap = int(share) if share and share.isdigit() and int(share) > 0 else allowed
    threads = max(1, min(allowed, cap, work_items))
    return threads, {"host_cpus": os.cpu_count(), "cpus_allowed": allowed,
                     "omp_num_threads": share, "threads": threads}


def lds_roofline(total, written, launch_s):
    """LDS line of a launch that moves `total` algorithmic bytes, `written` of
    them written: the shortest time the measured read and write rates allow
    for that mix, as a fraction of the launch."""
    rd, wr, measured = lds_peaks()
    t_min = (total - written) / (rd * CUS * CLOCK) + written / (wr * CUS * CLOCK)
    return {"achieved": total / launch_s / 1e9, "unit": "GB/s",
            "peak": total / t_min / 1e9, "frac": t_min / launch_s, "bytes_per_launch": total,
            "written_bytes_per_launch": written,
            "peak_read_bytes_per_clk_per_cu": rd, "peak_write_bytes_per_clk_per_cu": wr,
            "peak_source": "measured (profiles/" + LDS_PEAK_RECORD + ")" if measured
            else "assumed 128 B/clk/CU"}


def lds_peak_probe():
    """Run the LDS probe (include/xpbd_probe.h) for both access forms and print
    one JSON line: bytes per clock per CU from the workgroups' own cycle counts
    and from the event time at the 2.4 GHz peak clock."""
    import torch
    from paper_2503_18616_amd import xpbd
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    groups, per_cu = 2 * CUS, 2
    out = {}
    for name, kind in (("read_b128", xpbd.PROBE_LDS_READ_B128), ("write_b96", xpbd.PROBE_LDS_WRITE_B96)):
        ms, nbytes, cycles, ticks = xpbd.xpbd_lds_probe(kind, groups, 20000, stream)
        out[name] = {"ms": ms, "bytes": nbytes, "workgroups": groups, "reps": 20000,
                     "cycles_per_workgroup": cycles, "clock_ghz": cycles / ticks * 0.1,
                     "bytes_per_clk_per_cu": nbytes / groups * per_cu / cycles,
                     "bytes_per_clk_per_cu_at_2p4ghz": nbytes / (ms * 1e-3) / CLOCK / CUS}
        progress(f"LDS {name}: {out[name]}")
    print(json.dumps(out), flush=True)


def copy_calibration(mib):
    """One device-to-device copy of a known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB", flush=True)


def source_sha(name):
    import hashlib
    with open(os.path.join(ROOT, "paper_2503_18616_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload, steps_per_launch, args, record="xpbd_step_traffic.json"):
    """HBM bytes per step launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes
    recorded in profiles/, if they were taken on this kernel source, this launch
    selection (the runtime source), this colouring, the default launch shape and
    the default tools (spheres on their paths)."""
    path = os.path.join(ROOT, "profiles", record)
    if (not os.path.exists(path) or steps_per_launch != 1 or args.variant or args.packing
            or args.block or args.group or args.tool_shape != "sphere" or args.tool_lift):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (rec.get("kernel_source_sha256") != source_sha("xpbd_kernels.hip")
            or rec.get("runtime_source_sha256") != source_sha("xpbd_runtime.hip")
            or rec.get("workload") != workload or rec.get("colouring", 0) != args.colouring):
        return None
    return rec["traffic_bytes_per_launch"]


def loss_summary(losses, window=50):
    """Training loss over the first and the last `window` Adam steps (mean and
    median: a minibatch's loss is heavy-tailed where a few rows carry large
    corrections)."""
    import numpy as np
    first, last = np.asarray(losses[:window]), np.asarray(losses[-window:])
    return {"loss_first": float(first.mean()), "loss_last": float(last.mean()),
            "loss_first_median": float(np.median(first)),
            "loss_last_median": float(np.median(last)), "loss_window": int(window)}


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def lifted(tool_pos, args):
    """Tool poses raised by --tool-lift metres along z (every point of a pose)."""
    if args.tool_lift:
        tool_pos = tool_pos.copy()
        for k in range(2, tool_pos.shape[-1], 3):
            tool_pos[..., k] += args.tool_lift
    return tool_pos


def learned_leg(args, wl_fn, mesh, make_batch, I, S):
    """The learned warm start on the same workload: train the network on
    recorded substeps of a separate training run (untimed), then time
    learned stepping with the residual check against the plain solver's
    residual from the same start state."""
    import numpy as np
    import torch

    from paper_2503_18616_amd import warmstart as trainer
    from paper_2503_18616_amd import xpbd

    t0 = time.perf_counter()
    # training run: its own seeds, the same mesh and compliance distribution
    warm = 20
    tw = wl_fn(args.train_envs, seed=args.seed + 1, num_steps=warm + args.train_records)
    ttools = torch.from_numpy(lifted(tw.tools(warm + args.train_records), args)).cuda()
    subs = [k % S for k in range(args.train_records)]
    with make_batch(tw, 0) as tb:
        tb.step(warm, ttools[:warm])
        x0, v0 = tb.positions(), tb.velocities()
        with xpbd.Mlp(None, None, np.ones(xpbd.MLP_FEATURES), None, np.ones(3)) as pilot:
            f0, t0_ = trainer.record(tb, pilot, ttools[warm:], subs, I)
        norm = trainer.normalisation(f0, t0_)
        del f0, t0_
        tb.write(xpbd.FIELD_POS, x0)
        tb.write(xpbd.FIELD_VEL, v0)
        net = xpbd.Mlp(trainer.he_init(0), *norm)
        feats, targets = trainer.record(tb, net, ttools[warm:], subs, I)
    rows = int((feats[:, 31].float() > 0).sum())
    torch.cuda.synchronize()
    t_adam = time.perf_counter()
    losses = trainer.train(net, feats, targets, args.train_steps)
    torch.cuda.synchronize()
    adam_s = time.perf_counter() - t_adam
    del feats, targets
    train_s = time.perf_counter() - t0
    progress(f"learned warm start: trained in {train_s:.1f} s ({args.train_steps} Adam steps "
             f"in {adam_s:.3f} s)")

    # evaluation: plain and learned from the same state of the benchmark workload
    N = args.envs
    total = args.warmup + args.learned_steps
    wl = wl_fn(N, seed=args.seed, num_steps=total)
    tools = torch.from_numpy(lifted(wl.tools(total), args)).cuda()
    L = args.learned_steps
    with make_batch(wl, xpbd.F_RESIDUAL) as pb, make_batch(wl, xpbd.F_RESIDUAL) as lb:
        warm_res = []
        for s in range(args.warmup):
            pb.step(1, tools[s:s + 1])
            warm_res.append(pb.read(xpbd.FIELD_RESIDUAL).reshape(N, 2)[:, 0].copy())
        threshold = float(np.quantile(np.concatenate(warm_res), args.learned_quantile))
        x0, v0 = pb.positions(), pb.velocities()

        def restore(b):
            b.write(xpbd.FIELD_POS, x0)
            b.write(xpbd.FIELD_VEL, v0)

        # residual after k sweeps from the same state, plain and learned, no fallback
        by_sweeps = {"plain": {}, "learned": {}}
        probe = min(10, L)
        for k in (1, 2, 4, I):
            for mode in ("plain", "learned"):
                restore(lb)
                r = []
                for s in range(args.warmup, args.warmup + probe):
                    lb.step_learned(net, 1, tools[s:s + 1], k, k, np.inf,
                                    apply_correction=mode == "learned")
                    r.append(lb.read(xpbd.FIELD_RESIDUAL).reshape(N, 2)[:, 0].copy())
                by_sweeps[mode][str(k)] = float(np.concatenate(r).mean())

        # the three solvers from the same state: plain (xpbd_step), learned with
        # the stall rule, learned with fallback whenever the residual is above
        # the threshold (stall ratio 0)
        legs = {"learned": args.learned_stall, "learned_stall0": 0.0}
        stream = torch.cuda.current_stream()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        ms = {}
        for name, stall in legs.items():
            restore(lb)
            torch.cuda.synchronize()
            start.record(stream)
            lb.step_learned(net, L, tools[args.warmup:total], args.learned_min, I, threshold,
                            stall_ratio=stall)
            end.record(stream)
            torch.cuda.synchronize()
            ms[name] = start.elapsed_time(end)
        restore(pb)
        torch.cuda.synchronize()
        start.record(stream)
        pb.step(L, tools[args.warmup:total])
        end.record(stream)
        torch.cuda.synchronize()
        ms["plain"] = start.elapsed_time(end)
        # the same runs again, untimed, with every env-substep's sweeps and final
        # residual recorded (the runs are deterministic: the same trajectories;
        # plain through the learned entry point without correction, bit for bit
        # the plain step)
        its = torch.zeros(L * S * N, dtype=torch.int32, device="cuda")
        res = torch.zeros(L * S * N, dtype=torch.float32, device="cuda")
        stats = {}
        for name in ("plain", *legs):
            restore(lb)
            if name == "plain":
                lb.step_learned(None, L, tools[args.warmup:total], I, I, np.inf,
                                apply_correction=False, iterations=its, residuals=res)
            else:
                lb.step_learned(net, L, tools[args.warmup:total], args.learned_min, I, threshold,
                                stall_ratio=legs[name], iterations=its, residuals=res)
            it, r = its.cpu().numpy(), res.cpu().numpy().astype(np.float64)
            stats[name] = {"sweeps_mean": float(it.mean()),
                           "fallback_fraction": float((it > args.learned_min).mean())
                           if name != "plain" else 0.0,
                           "residual_mean": float(r.mean()),
                           "residual_p50": float(np.quantile(r, 0.5)),
                           "residual_p99": float(np.quantile(r, 0.99)),
                           "residual_max": float(r.max()),
                           "above_threshold": float((r > threshold).mean())}
    net.close()

    def rate(t):
        return N * L * S / (t / 1e3)

    def matched(name):
        return bool(stats[name]["residual_mean"] <= stats["plain"]["residual_mean"] and
                    stats[name]["residual_p99"] <= stats["plain"]["residual_p99"])
    st = stats["learned"]
    return {"value": rate(ms["learned"]), "unit": "env-substeps/s",
            "ms_per_step": ms["learned"] / L, "steps": L,
            "plain_value_same_steps": rate(ms["plain"]),
            "min_iterations": args.learned_min, "max_iterations": I,
            "stall_ratio": args.learned_stall,
            "threshold": threshold, "threshold_rule": f"plain {I}-sweep residual, "
            f"{args.learned_quantile:g} quantile over {args.warmup} warm-up steps",
            "sweeps_mean": st["sweeps_mean"], "fallback_fraction": st["fallback_fraction"],
            "residual_rms_mean": st["residual_mean"],
            "plain_residual_rms_mean": stats["plain"]["residual_mean"],
            "residual_matched": matched("learned"),
            "residual_matched_rule": "mean and 0.99 quantile of the per-env-substep residual "
                                     "at most the plain solver's, over the same steps",
            "residual_ratio": st["residual_mean"] / stats["plain"]["residual_mean"],
            "stall0": {"value": rate(ms["learned_stall0"]), "ms_per_step": ms["learned_stall0"] / L,
                       "residual_matched": matched("learned_stall0"),
                       "sweeps_mean": stats["learned_stall0"]["sweeps_mean"],
                       "fallback_fraction": stats["learned_stall0"]["fallback_fraction"]},
            "per_substep_residual": stats,
            "residual_by_sweeps": by_sweeps,
            "training": {"envs": args.train_envs, "recorded_substeps": args.train_records,
                         "free_rows": rows, "adam_steps": args.train_steps,
                         **loss_summary(losses), "seconds": train_s,
                         "adam_seconds": adam_s},
            "network": "27-128-128-3 ReLU, bf16 MFMA, fp32 accumulate"}


def mesh_sizes(xpbd, m):
    """(kept edges, kept tets, particles, free particles) of a mesh."""
    info = xpbd.xpbd_prepare_mesh(m.rest_pos, m.inv_mass, m.tets)
    return (int(info["edges"].shape[0]), int(info["tets"].shape[0]), m.num_vertices,
            int((m.inv_mass > 0).sum()))


def rl_learned_leg(args, make_batch, policy, rp, S, I):
    """The learned warm start inside the RL-style step: train the network on
    substeps recorded from RL steps of a separate training batch (untimed),
    then time RL steps with the learned warm start against plain RL steps
    from the same state (positions, velocities, tool centres, grasps)."""
    import numpy as np
    import torch

    from paper_2503_18616_amd import warmstart as trainer
    from paper_2503_18616_amd import workloads as W
    from paper_2503_18616_amd import xpbd

    def rl_state(n, seed):
        tools0, target = W.rl_start(n, seed)
        return (torch.from_numpy(tools0).cuda(), torch.full((n,), -1, dtype=torch.int32,
                                                             device="cuda"),
                torch.from_numpy(target).cuda())

    def snapshot(b, tp, gr):
        return b.positions(), b.velocities(), tp.clone(), gr.clone()

    def restore(b, tp, gr, snap):
        b.write(xpbd.FIELD_POS, snap[0])
        b.write(xpbd.FIELD_VEL, snap[1])
        tp.copy_(snap[2])
        gr.copy_(snap[3])

    t0 = time.perf_counter()
    warm, n_rec = 20, args.train_records
    tw = W.rl_workload(args.train_envs, seed=args.seed + 1)
    NP = args.train_envs * tw.meshes[0].num_vertices
    subs = [k % S for k in range(n_rec)]

    def record(b, net, tp, gr, tg):
        feats = torch.zeros((n_rec * NP, xpbd.MLP_FEATURE_STRIDE), dtype=torch.bfloat16,
                            device="cuda")
        targets = torch.zeros((n_rec * NP, 4), dtype=torch.float32, device="cuda")
        for k, sub in enumerate(subs):
            b.rl_step_learned(policy, rp, net, 1, tp, gr, tg, I, I, np.inf,
                              apply_correction=False, record_substep=sub,
                              record_features=feats[k * NP:(k + 1) * NP],
                              record_targets=targets[k * NP:(k + 1) * NP])
        return feats, targets

    with make_batch(tw, 0) as tb:
        tp, gr, tg = rl_state(args.train_envs, args.seed + 1)
        for _ in range(warm):
            tb.rl_step(policy, rp, 1, tp, gr, tg)
        snap = snapshot(tb, tp, gr)
        with xpbd.Mlp(None, None, np.ones(xpbd.MLP_FEATURES), None, np.ones(3)) as pilot:
            f0, t0_ = record(tb, pilot, tp, gr, tg)
        norm = trainer.normalisation(f0, t0_)
        del f0, t0_
        restore(tb, tp, gr, snap)
        net = xpbd.Mlp(trainer.he_init(0), *norm)
        feats, targets = record(tb, net, tp, gr, tg)
    rows = int((feats[:, 31].float() > 0).sum())
    losses = trainer.train(net, feats, targets, args.train_steps)
    del feats, targets
    train_s = time.perf_counter() - t0
    progress(f"RL learned warm start: trained in {train_s:.1f} s")

    N = args.envs or 8192
    steps = args.learned_steps
    wl = W.rl_workload(N, seed=args.seed)
    its = torch.zeros(steps * S * N, dtype=torch.int32, device="cuda")
    with make_batch(wl, xpbd.F_RESIDUAL) as pb, make_batch(wl, xpbd.F_RESIDUAL) as lb:
        tp, gr, tg = rl_state(N, args.seed)
        warm_res = []
        for _ in range(args.warmup):
            pb.rl_step(policy, rp, 1, tp, gr, tg)
            warm_res.append(pb.read(xpbd.FIELD_RESIDUAL).reshape(N, 2)[:, 0].copy())
        threshold = float(np.quantile(np.concatenate(warm_res), args.learned_quantile))
        snap = snapshot(pb, tp, gr)
        ltp, lgr = tp.clone(), gr.clone()
        restore(lb, ltp, lgr, snap)
        stream = torch.cuda.current_stream()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for s in range(steps):
            lb.rl_step_learned(policy, rp, net, 1, ltp, lgr, tg, args.learned_min, I, threshold,
                               iterations=its[s * S * N:(s + 1) * S * N],
                               stall_ratio=args.learned_stall)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        # the learned RL step captured in a graph, replayed from where it stopped
        lp = xpbd.make_learned_params(args.learned_min, I, threshold, stall_ratio=args.learned_stall)
        with lb.rl_graph(policy, rp, ltp, lgr, tg, net=net, learned=lp) as g:
            g.launch(2)
            torch.cuda.synchronize()
            start.record(stream)
            g.launch(steps)
            end.record(stream)
            torch.cuda.synchronize()
        graph_ms = start.elapsed_time(end) / steps
        start.record(stream)
        for s in range(steps):
            pb.rl_step(policy, rp, 1, tp, gr, tg)
        end.record(stream)
        torch.cuda.synchronize()
        ms_plain = start.elapsed_time(end)
        # the residual of every step (last substep), untimed, from the same state
        r_l, r_p = [], []
        for b, out in ((lb, r_l), (pb, r_p)):
            restore(b, tp, gr, snap)
            for s in range(steps):
                if b is lb:
                    b.rl_step_learned(policy, rp, net, 1, tp, gr, tg, args.learned_min, I,
                                      threshold, stall_ratio=args.learned_stall)
                else:
                    b.rl_step(policy, rp, 1, tp, gr, tg)
                out.append(b.read(xpbd.FIELD_RESIDUAL).reshape(N, 2)[:, 0].copy())
        r_l, r_p = np.concatenate(r_l), np.concatenate(r_p)
    net.close()
    it = its.cpu().numpy()
    return {"value": N * steps * S / (ms / 1e3), "unit": "env-substeps/s",
            "ms_per_step": ms / steps, "steps": steps, "graph_ms_per_step": graph_ms,
            "plain_value_same_steps": N * steps * S / (ms_plain / 1e3),
            "min_iterations": args.learned_min, "max_iterations": I,
            "stall_ratio": args.learned_stall, "threshold": threshold,
            "threshold_rule": f"plain {I}-sweep residual, {args.learned_quantile:g} quantile "
                              f"over {args.warmup} warm-up steps",
            "sweeps_mean": float(it.mean()),
            "fallback_fraction": float((it > args.learned_min).mean()),
            "residual_rms_mean": float(r_l.mean()),
            "plain_residual_rms_mean": float(r_p.mean()),
            "residual_p99": float(np.quantile(r_l, 0.99)),
            "plain_residual_p99": float(np.quantile(r_p, 0.99)),
            "residual_matched": bool(r_l.mean() <= r_p.mean()
                                     and np.quantile(r_l, 0.99) <= np.quantile(r_p, 0.99)),
            "residual_matched_rule": "mean and 0.99 quantile of the per-env-step residual (last "
                                     "substep) at most the plain solver's, over the same steps",
            "residual_ratio": float(r_l.mean() / r_p.mean()),
            "training": {"envs": args.train_envs, "recorded_substeps": n_rec,
                         "free_rows": rows, "adam_steps": args.train_steps,
                         **loss_summary(losses), "seconds": train_s},
            "network": "27-128-128-3 ReLU, bf16 MFMA, fp32 accumulate"}


def rl_bench(args):
    """The RL-style step (include/xpbd_rl.h): per step and environment the
    observations, the 64-256-256-7 policy, the tool motion, the grasp and the
    simulation step.  The timed region is K xpbd_rl_step calls of one step
    each (as an RL loop that reads every step's observations), all on the
    batch's stream, bracketed by HIP events."""
    import numpy as np
    import torch

    from paper_2503_18616_amd import workloads as W
    from paper_2503_18616_amd import xpbd

    N = args.envs or 8192
    total = args.warmup + args.steps
    wl = W.rl_workload(N, seed=args.seed, num_steps=total)
    m = wl.meshes[0]
    S, I = wl.substeps, wl.iterations
    E, T, V, v_free = mesh_sizes(xpbd, m)
    stream = torch.cuda.current_stream()
    params = xpbd.make_params(wl.dt, S, I, wl.gravity, 2, wl.tool_radius, block_size=args.block,
                              solver_variant=args.variant, colour_packing=args.packing,
                              envs_per_group=args.group, colouring=args.colouring)
    t_create = time.perf_counter()
    batch = xpbd.Batch([(m.rest_pos, m.inv_mass, m.tets)], wl.env_mesh, wl.compliance, params,
                       stream=stream.cuda_stream)
    policy = xpbd.Policy(W.rl_policy_params(args.seed), stream=stream.cuda_stream)
    t_create = time.perf_counter() - t_create
    launch = batch.info()
    lo, hi = W.rl_box()
    rp = xpbd.make_rl_params(W.RL_GRASP_RADIUS, W.RL_GRASP_OFFSET, W.RL_MAX_SPEED,
                             W.RL_OBS_SCALE, W.rl_origin(), lo, hi, W.rl_tracked(m))
    tools0, target = W.rl_start(N, args.seed)
    tp = torch.from_numpy(tools0).cuda()
    gr = torch.full((N,), -1, dtype=torch.int32, device="cuda")
    tg = torch.from_numpy(target).cuda()
    obs = torch.zeros((1, N, xpbd.RL_OBS), dtype=torch.float32, device="cuda")
    act = torch.zeros((1, N, xpbd.RL_ACTIONS), dtype=torch.float32, device="cuda")
    progress(f"{wl.name}: set up in {t_create:.1f} s")
    batch.set_flags(xpbd.F_RESIDUAL)   # allocate the multiplier buffer before the timed region
    batch.set_flags(0)
    for _ in range(args.warmup):
        batch.rl_step(policy, rp, 1, tp, gr, tg, obs, act)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for s in range(args.steps):
        if s == args.steps - 1:
            batch.set_flags(xpbd.F_RESIDUAL)
        batch.rl_step(policy, rp, 1, tp, gr, tg, obs, act)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    progress(f"timed {args.steps} RL steps: {ms / args.steps:.3f} ms per step")
    holding = int((gr >= 0).sum())
    resid = batch.read(xpbd.FIELD_RESIDUAL).reshape(N, 2)
    # the same RL step captured in a graph (include/xpbd_graph.h) and replayed
    # from the state the timed steps left
    batch.set_flags(0)
    graph_steps = min(args.steps, 100)
    with batch.rl_graph(policy, rp, tp, gr, tg, obs, act) as g:
        g.launch(2)
        torch.cuda.synchronize()
        start.record(stream)
        g.launch(graph_steps)
        end.record(stream)
        torch.cuda.synchronize()
    graph_ms = start.elapsed_time(end) / graph_steps
    progress(f"graph replays: {graph_ms:.3f} ms per step")
    batch.close()

    learned = None
    if not args.no_learned and args.variant in (0, 1) and not args.group:
        def make(w, flags):
            p = xpbd.make_params(w.dt, S, I, w.gravity, 2, w.tool_radius, flags=flags,
                                 block_size=args.block, solver_variant=xpbd.VARIANT_REGISTERS,
                                 colour_packing=args.packing, envs_per_group=1,
                                 colouring=args.colouring)
            return xpbd.Batch([(m.rest_pos, m.inv_mass, m.tets)], w.env_mesh, w.compliance, p,
                              stream=stream.cuda_stream)
        learned = rl_learned_leg(args, make, policy, rp, S, I)
    policy.close()

    step_s = ms / 1e3 / args.steps
    flops = N * S * (I * (E * FLOPS_EDGE + T * FLOPS_TET) + v_free * FLOPS_PARTICLE)
    policy_flops = N * 2 * (xpbd.RL_OBS * xpbd.RL_HIDDEN + xpbd.RL_HIDDEN * xpbd.RL_HIDDEN +
                            xpbd.RL_HIDDEN * xpbd.RL_ACTIONS)
    roofline = {"bound": "alu", "achieved": flops / step_s / 1e12,
                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                "frac": flops / step_s / PEAK_FP32,
                "frac_nonpacked_issue": flops / step_s / PEAK_FP32_NONPACKED,
                "traffic": measured_traffic(wl.name, 1, args, "rl_step_traffic.json"),
                "kernel": "xpbd_step_reg_kernel (grasping), timed with the policy kernel "
                          "of the same step",
                "launch_ms": step_s * 1e3, "flops_per_launch": flops}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        import oracle.rl as R
        from concurrent.futures import ThreadPoolExecutor
        f32 = lambda v: float(np.float32(v))
        om = oracle.prepare_mesh(m.rest_pos, m.inv_mass, m.tets, colouring=args.colouring)
        op = oracle.OracleParams(f32(wl.dt), S, I, tuple(f32(g) for g in wl.gravity), 2,
                                 tuple(f32(r) for r in wl.tool_radius))
        vec = lambda v: tuple(f32(x) for x in v)
        orl = R.RlParams(f32(W.RL_GRASP_RADIUS), vec(W.RL_GRASP_OFFSET), f32(W.RL_MAX_SPEED),
                         f32(W.RL_OBS_SCALE), vec(W.rl_origin()), vec(lo), vec(hi),
                         W.rl_tracked(m))
        net = R.unpack_policy(W.rl_policy_params(args.seed))
        envs = list(range(0, N, max(1, N // args.cpu_envs)))[:args.cpu_envs]
        steps = min(args.cpu_steps, 30)
        threads, host = host_threads(len(envs))
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as pool:
            list(pool.map(lambda e: R.run_env_rl(om, wl.compliance[e], op, orl, net, tools0[e],
                                                 target[e], steps), envs))
        dt = time.perf_counter() - t0
        progress(f"oracle sample: {dt:.1f} s")
        cpu = {"value": len(envs) * steps * S / dt, "unit": "env-substeps/s", "cores": threads,
               "kind": "oracle", "host": host,
               "sample": f"{len(envs)} of the {N} environments x {steps} RL steps "
                         f"({len(envs) * steps * S} env-substeps, FP64, {dt:.1f} s wall)"}

    out = {
        "metric": METRIC, "value": N * args.steps * S / (ms / 1e3), "unit": "env-substeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "seed": args.seed, "envs": N, "grid": [m.nx, m.ny, m.nz],
                   "particles": V,
                   "edges": E, "tets": T, "substeps": S, "iterations": I, "tools": 2,
                   "create_s": round(t_create, 3), "solver": "plain (no warm start)",
                   "launch": launch,
                   "colouring": COLOURINGS[args.colouring],
                   "policy": "64-256-256-7 bf16 (random init)",
                   "env_steps_per_s": N * args.steps / (ms / 1e3),
                   "policy_gflop_per_step": policy_flops / 1e9,
                   "holding_at_end": holding,
                   "graph_ms_per_step": graph_ms,
                   "residual_rms_mean": float(resid[:, 0].mean()),
                   "residual_max": float(resid[:, 1].max())},
        "roofline": roofline, "cpu_baseline": cpu, "learned": learned,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "environments are independent, so a multi-GPU run is N copies of this one",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.lds_peak:
        lds_peak_probe()
        return
    if args.steps % args.steps_per_launch or args.warmup % args.steps_per_launch:
        sys.exit("--steps and --warmup must be multiples of --steps-per-launch")

    import numpy as np
    import torch

    from paper_2503_18616_amd import workloads as W
    from paper_2503_18616_amd import xpbd

    torch.cuda.set_device(0)
    if args.workload == "rl":
        rl_bench(args)
        return
    total = args.warmup + args.steps
    if args.workload == "batch":
        args.envs = args.envs or 1024
        wl = W.batch_workload(args.envs, seed=args.seed, num_steps=total)
    elif args.workload == "uneven":
        args.envs = args.envs or 4096
        wl = W.uneven_workload(args.envs, seed=args.seed, num_steps=total)
    else:
        wl = W.single_env_workload(seed=args.seed)
        wl.num_steps = total
        args.envs = 1
    m = wl.meshes[0]
    N, S, I = wl.num_envs, wl.substeps, wl.iterations
    # per-mesh sizes (kept edges and tets, free particles), summed over the environments
    sizes = []
    for mm in wl.meshes:
        info = xpbd.xpbd_prepare_mesh(mm.rest_pos, mm.inv_mass, mm.tets)
        sizes.append((int(info["edges"].shape[0]), int(info["tets"].shape[0]), mm.num_vertices,
                      int((mm.inv_mass > 0).sum())))
    env_sizes = np.array([sizes[int(k)] for k in wl.env_mesh], np.int64)   # [N][E, T, V, free]
    E, T, V, v_free = (int(x) for x in sizes[0])

    capsules = args.tool_shape == "capsule"
    if capsules:
        tools = torch.from_numpy(lifted(W.capsule_path(total, N, wl.seed), args)).cuda()
    else:
        tools = torch.from_numpy(lifted(wl.tools(total), args)).cuda()
    params = xpbd.make_params(wl.dt, S, I, wl.gravity, wl.num_tools, wl.tool_radius,
                              flags=0, block_size=args.block,
                              solver_variant=args.variant, colour_packing=args.packing,
                              envs_per_group=args.group, colouring=args.colouring,
                              tool_shape=xpbd.TOOL_CAPSULE if capsules else xpbd.TOOL_SPHERE)
    stream = torch.cuda.current_stream()
    tuned = None
    if args.autotune:
        t_tune = time.perf_counter()
        best, default = xpbd.xpbd_autotune(
            [(mm.rest_pos, mm.inv_mass, mm.tets) for mm in wl.meshes], wl.env_mesh, wl.compliance,
            params, args.autotune, tools[:args.autotune], stream=stream.cuda_stream)
        tuned = {"ms_per_step_tuned": best, "ms_per_step_default": default,
                 "solver_variant": params.solver_variant, "block_size": params.block_size,
                 "envs_per_group": params.envs_per_group, "colour_packing": params.colour_packing,
                 "seconds": round(time.perf_counter() - t_tune, 1)}
        progress(f"autotune: {tuned}")
    t_create = time.perf_counter()
    batch = xpbd.Batch([(mm.rest_pos, mm.inv_mass, mm.tets) for mm in wl.meshes], wl.env_mesh,
                       wl.compliance, params, stream=stream.cuda_stream)
    t_create = time.perf_counter() - t_create
    launch = batch.info()
    progress(f"{wl.name}: {N} environments of {len(wl.meshes)} meshes set up in {t_create:.1f} s; "
             f"launch {launch}")
    # The learned leg (its own batches: training and the timed learned and plain
    # steps) runs first.  Its seconds of GPU work also bring the GPU to its
    # steady clock: after an idle spell the first step launches run up to 18 %
    # slower (2.48 ms falling to 2.11 ms over the first 8 launches in a kernel
    # trace), longer than a few warm-up steps cover.
    learned = None
    if not args.no_learned and args.workload == "batch" and not capsules and args.variant in (0, 1):
        def make(w, flags):
            p = xpbd.make_params(w.dt, S, I, w.gravity, w.num_tools, w.tool_radius, flags=flags,
                                 solver_variant=xpbd.VARIANT_REGISTERS, colouring=args.colouring)
            return xpbd.Batch([(m.rest_pos, m.inv_mass, m.tets)], w.env_mesh, w.compliance, p,
                              stream=stream.cuda_stream)
        learned = learned_leg(args, W.batch_workload, m, make, I, S)

    spl = args.steps_per_launch
    # the residual of the last timed launch needs the multiplier buffer: enable
    # it once here, so that switching the flag on inside the timed region
    # allocates nothing
    batch.set_flags(xpbd.F_RESIDUAL)
    batch.set_flags(0)
    for s in range(0, args.warmup, spl):
        batch.step(spl, tools[s:s + spl])
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for s in range(args.warmup, total, spl):
        if s + spl == total:   # the residual of the final state, computed on the last launch
            batch.set_flags(xpbd.F_RESIDUAL)
        batch.step(spl, tools[s:s + spl])
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    progress(f"timed {args.steps} steps: {ms / args.steps:.3f} ms per step")
    launches = args.steps // spl
    env_substeps = N * args.steps * S
    value = env_substeps / (ms / 1e3)
    resid = batch.read(xpbd.FIELD_RESIDUAL).reshape(N, 2)
    # the same step captured in a graph (include/xpbd_graph.h; a batch of
    # several size classes as parallel branches) and replayed from the state
    # the timed steps left, on a copy of the last step's tool poses
    batch.set_flags(0)
    graph_steps = min(args.steps, 100)
    graph_tools = tools[total - 1].clone()
    with batch.step_graph(graph_tools) as g:
        g.launch(2)
        torch.cuda.synchronize()
        start.record(stream)
        g.launch(graph_steps)
        end.record(stream)
        torch.cuda.synchronize()
    graph_ms = start.elapsed_time(end) / graph_steps
    progress(f"graph replays: {graph_ms:.3f} ms per step")
    batch.close()

    # roofline of the step kernel (the only kernel in the timed region)
    launch_s = ms / 1e3 / launches
    Es, Ts, Vs, Fs = (env_sizes[:, k] for k in range(4))
    flops = int(spl * S * (I * (Es * FLOPS_EDGE + Ts * FLOPS_TET) + Fs * FLOPS_PARTICLE).sum())
    lds = int(spl * S * (I * (Es * LDS_EDGE + Ts * LDS_TET) + Vs * LDS_PARTICLE).sum())
    lds_w = int(spl * S * (I * (Es * LDS_EDGE_W + Ts * LDS_TET_W) + Vs * LDS_PARTICLE_W).sum())
    hbm = int((Vs * HBM_PARTICLE + spl * wl.num_tools * 12).sum())
    roofline = {"bound": "alu", "achieved": flops / launch_s / 1e12,
                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                "frac": flops / launch_s / PEAK_FP32,
                "traffic": measured_traffic(wl.name, spl, args),
                "kernel": "xpbd_step_reg_kernel", "launch_ms": launch_s * 1e3,
                "flops_per_launch": flops,
                "frac_nonpacked_issue": flops / launch_s / PEAK_FP32_NONPACKED}
    lds_line = lds_roofline(lds, lds_w, launch_s)
    hbm_line = {"achieved": hbm / launch_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": hbm / launch_s / PEAK_HBM, "bytes_per_launch": hbm}

    cpu = None
    if not args.no_cpu_baseline and not capsules and args.variant != 3:
        import oracle
        sample_envs = list(range(0, N, max(1, N // args.cpu_envs)))[:args.cpu_envs]
        f32 = lambda v: float(np.float32(v))
        used = sorted({int(wl.env_mesh[e]) for e in sample_envs})
        om = [oracle.prepare_mesh(wl.meshes[k].rest_pos, wl.meshes[k].inv_mass, wl.meshes[k].tets,
                                  colouring=args.colouring)
              if k in used else None for k in range(len(wl.meshes))]
        op = oracle.OracleParams(f32(wl.dt), S, I, tuple(f32(g) for g in wl.gravity),
                                 wl.num_tools, tuple(f32(r) for r in wl.tool_radius))
        cpu_tools = lifted(wl.tools(args.cpu_steps, env_ids=sample_envs), args)
        threads, host = host_threads(len(sample_envs))
        t0 = time.perf_counter()
        oracle.run_batch(om, wl.env_mesh, wl.compliance, op, cpu_tools, args.cpu_steps,
                         env_ids=sample_envs, threads=threads)
        dt = time.perf_counter() - t0
        progress(f"oracle sample: {dt:.1f} s")
        cpu = {"value": len(sample_envs) * args.cpu_steps * S / dt, "unit": "env-substeps/s",
               "cores": threads, "kind": "oracle", "host": host,
               "sample": f"{len(sample_envs)} of the {N} environments x {args.cpu_steps} steps "
                         f"({len(sample_envs) * args.cpu_steps * S} env-substeps, FP64, "
                         f"{dt:.1f} s wall)"}

    out = {
        "metric": METRIC, "value": value, "unit": "env-substeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "seed": args.seed, "envs": N, "meshes": len(wl.meshes),
                   "grid": [m.nx, m.ny, m.nz] if len(wl.meshes) == 1 else "per environment",
                   "particles": V if len(wl.meshes) == 1 else int(Vs.sum()),
                   "edges": E if len(wl.meshes) == 1 else int(Es.sum()),
                   "tets": T if len(wl.meshes) == 1 else int(Ts.sum()),
                   "substeps": S, "iterations": I, "create_s": round(t_create, 3),
                   "steps_per_launch": spl, "solver": "plain (no warm start)",
                   "tool_lift_m": args.tool_lift, "autotune": tuned,
                   "tool_shape": args.tool_shape,
                   "solver_variant": ["auto", "registers", "lds", "jacobi"][args.variant],
                   "colouring": COLOURINGS[args.colouring],
                   "launch": launch,
                   "graph_ms_per_step": graph_ms,
                   "residual_rms_mean": float(resid[:, 0].mean()),
                   "residual_max": float(resid[:, 1].max())},
        "roofline": roofline, "lds": lds_line, "hbm": hbm_line, "cpu_baseline": cpu,
        "learned": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
