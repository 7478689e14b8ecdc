#!/usr/bin/env python3
"""Throughput of the BR-MPPI control update on one MI355X.

Default workload (the reverse-parking closed loop): S = 8192 samples, horizon
T = 50, Ts = 0.05 s, eight parked-vehicle ellipses, 200 receding-horizon
updates.  A "step" is one control update: Philox noise + S rollouts with
barrier-rate guidance and contouring cost + weights + weighted average +
warm-start shift, followed by the FP64 plant step that closes the loop.  The
whole loop is device-resident: the path, warm start, obstacles and plant state
live in HBM and no host round trip happens between updates.

  value = S * T * steps / wall time of the timed loop   [sample-steps/s]

Printed as one JSON line; extra fields carry the plain-solve latency
percentiles, the batched and served forms against plain per-instance solves,
the paper's own problem shape, the roofline of the rollout kernel and the CPU
oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X vector FP32 (packed), AMD spec
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
KERNEL_SRC = os.path.join(ROOT, "paper_2508_05773_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rollout_c2_traffic.json")
LEGS = ("latency", "batched", "served", "paper", "large")


# ---------------------------------------------------------------------------
# algorithmic work of the rollout kernel (counted from its source: add, sub,
# mul = 1 flop, fma = 2, each transcendental / reciprocal / division = 1;
# FP64 accumulations included; Philox integer ops excluded)
# ---------------------------------------------------------------------------
def flops_per_sample_step(n_obs: int, hitch: bool = True, guided: bool = True) -> int:
    if not guided:
        return 6 + 11 + 59 + 18 + 24          # inputs, trig, cost, dynamics, one noise block
    nb = (5 + n_obs + 3) // 4                  # Philox blocks per step
    base = 6 + 11 + 20 + 59 + 18               # inputs, trig, 2x2 solve, cost, dynamics
    return base + 24 * nb + (120 if hitch else 0) + 125 * n_obs


def noise_flops_per_sample_step(n_obs: int, guided: bool = True) -> int:
    """Box-Muller part of the count (24 per Philox block)"""
    return 24 * ((5 + n_obs + 3) // 4 if guided else 1)


def rollout_flops(S: int, T: int, n_obs: int, hitch=True, guided=True, noise_in_kernel=True) -> float:
    f = flops_per_sample_step(n_obs, hitch, guided)
    if not noise_in_kernel:
        f -= noise_flops_per_sample_step(n_obs, guided)
    return float(S) * (T * f + 48)


def kernel_sha() -> str:
    """hash of the kernel source's code: line comments, trailing blanks and
    empty lines do not count, so that a comment edit keeps the measured
    traffic valid"""
    code = []
    for line in open(KERNEL_SRC, encoding="utf-8").read().splitlines():
        line = line.split("//", 1)[0].rstrip()
        if line:
            code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


def load_traffic():
    """HBM bytes per rollout launch from the committed rocprofv3 counter runs,
    valid only while the kernel source is unchanged."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q)) if len(a) else None


def note(msg):
    """progress line on stderr (the JSON result is the only stdout line)"""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="control updates in the timed loop")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-solves", type=int, default=300)
    ap.add_argument("--served-seconds", type=float, default=0.3, help="simulated seconds of the served leg")
    ap.add_argument("--served-sweep", default="32,64,96,128,160",
                    help="controller counts of the served leg's latency sweep below capacity")
    ap.add_argument("--sweep-seconds", type=float, default=1.0, help="simulated seconds per sweep point")
    ap.add_argument("--sustain-seconds", type=float, default=5.0,
                    help="simulated seconds of the served run at the highest load the sweep kept under the tick")
    ap.add_argument("--cpu-seconds", type=float, default=24.0)
    ap.add_argument("--no-extras", action="store_true", help="only the timed closed loop")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch shapes")
    ap.add_argument("--tune-file", default=None,
                    help="launch-shape table: used as is when it exists, else written by the autotune")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="extra legs to run after the timed loop (comma list of %s)" % ", ".join(LEGS))
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a 256 MiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the control update on one MI355X; runs on several GPUs are not "
              "supported. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calib_copy:
        n = 256 << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n, "launches": 5}))
        return

    from paper_2508_05773_amd import brmppi as B
    from paper_2508_05773_amd import workloads as W

    prob = W.config2()
    S, T, n_obs = prob.S, prob.T, prob.n_obs
    import tempfile

    tune_file = args.tune_file or os.path.join(tempfile.mkdtemp(prefix="brmppi_tune_"), "launch.json")
    have_table = os.path.exists(tune_file)
    ctx = B.Context(arena_bytes=3 << 30, n_streams=2, max_controllers=600,
                    profile=False, flags_extra=B.CTX_PROFILE_ROLLOUT, autotune_cache=tune_file)
    h = ctx.h
    shape = None
    if not args.no_autotune:
        if not have_table:
            note("autotuning launch shapes")
            B.brmppi_autotune(h)
        shape = json.load(open(tune_file)).get("plain_8_1")   # 8-obstacle bucket, S <= 8192
    # the value is timed on a context that records no events (a pair of HIP
    # events around every launch puts stream markers between the kernels and
    # costs about 9 us per update); the same loop then runs on the profiling
    # context, which times every rollout launch with HIP events on its stream
    ctx2 = B.Context(arena_bytes=3 << 30, n_streams=2, max_controllers=600, profile=False,
                     autotune_cache=tune_file)

    def timed_loop(c):
        c.set_path(0, prob.path, prob.ds)
        pb = B.ProblemBuffers(prob, controller=0)
        # ---- warm-up, then the timed closed loop from the start state ----
        if args.warmup > 0:
            B.brmppi_closed_loop(c.h, pb, args.warmup, want_x=False, want_u=False)
        B.brmppi_profile_reset(c.h)
        info0 = B.brmppi_get_info(c.h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.brmppi_closed_loop(c.h, pb, args.steps, want_x=False, want_u=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        info1 = B.brmppi_get_info(c.h)
        # buffers the library had to re-allocate inside the timed call (the loop's
        # scratch and staging do not depend on its length: this is 0)
        grows = sum(info1[k] - info0[k] for k in ("scratch_grows", "pinned_grows"))
        return el, B.brmppi_get_state(c.h, 0), grows

    wall, x_end, grows = timed_loop(ctx2)
    if grows:
        note(f"warning: {grows} buffer re-allocations inside the timed loop")
    value = S * T * args.steps / wall
    wall_prof, _, _ = timed_loop(ctx)
    prof = B.brmppi_profile_read(h)
    roll_ms = prof["rollout"]["ms"] / max(prof["rollout"]["count"], 1)
    # the closed loop draws the normals of several updates per noise launch
    noise_ms = prof["noise"]["ms"] / args.steps if prof["noise"]["count"] else 0.0
    # variants 1-4 draw the normals in the separate noise kernel: the rollout
    # kernel's own algorithmic work then excludes the Box-Muller flops
    noise_in_kernel = prof["noise"]["count"] == 0
    flops = rollout_flops(S, T, n_obs, noise_in_kernel=noise_in_kernel)
    achieved = flops / (roll_ms * 1e-3) / 1e12
    traffic = load_traffic()
    out = {
        "metric": "sample-steps/s; MPPI solves/s + p50/p99 solve latency, batched vs plain",
        "value": value,
        "unit": "sample-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"reverse parking closed loop: S=8192, T=50, Ts=0.05 s, 8 parked-vehicle "
                               f"ellipses, {args.steps} receding-horizon updates timed after {args.warmup} "
                               f"untimed ones, device-resident",
                   "S": S, "T": T, "n_obs": n_obs, "updates": args.steps},
        "buffer_regrowths_in_timed_loop": grows,
        "solves_per_s": args.steps / wall,
        "ms_per_step_with_launch_events": wall_prof * 1e3 / args.steps,
        "final_state_finite": bool(np.all(np.isfinite(x_end))),
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
            "kernel": "k_rollout (8-obstacle bucket)", "launch_shape": {"block_variant": shape},
            "noise_kernel_ms_per_update": noise_ms, "noise_launches": prof["noise"]["count"], "flops_per_launch": flops, "avg_launch_ms": roll_ms,
            "launches": prof["rollout"]["count"], "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
            "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
            "flops_per_sample_step": flops_per_sample_step(n_obs),
        },
    }

    legs = set() if args.no_extras else {x for x in args.legs.split(",") if x}
    bad = legs - set(LEGS)
    if bad:
        ap.error(f"unknown legs {sorted(bad)}")
    if "large" in legs:
        out["large"] = large_leg(B, W, ctx, tune_file if not args.no_autotune else None)
    ctx.close()
    if legs - {"large"}:
        # the other legs run on the context without kernel timing: with timing
        # on, a batch is launched directly instead of replayed from its HIP
        # graph, and every timed launch records two events
        out.update(extras(args, B, W, ctx2, prob, legs))
    ctx2.close()

    if not args.no_cpu:
        note("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(W, prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def extras(args, B, W, ctx, prob, legs):
    res = {}
    if "latency" in legs:
        note("plain-solve latency")
        res.update(latency_leg(args, B, ctx, prob))
    if "batched" in legs:
        note("batched vs plain")
        res["batched"] = batched_leg(B, W, ctx)
    if "served" in legs:
        note("served")
        # ---- served: continuous batching of 256 controllers vs sequential plain ----
        res["served"] = served_leg(args, B, W, ctx)
    if "paper" in legs:
        note("paper shape")
        res["paper_shape"] = paper_leg(B, W, ctx)
    return res


def latency_leg(args, B, ctx, prob):
    h = ctx.h
    res = {}
    # ---- plain blocking solve latency (host in, host out) ----
    ctx.set_path(1, prob.path, prob.ds)
    lat = []
    for k in range(args.latency_solves + 10):
        pbk = B.ProblemBuffers(prob, controller=1, with_nominal=(k == 0), seed=prob.seed + k)
        _, st, _ = B.brmppi_solve(h, pbk)
        if k >= 10:
            lat.append(st["latency_us"] * 1e-3)
    res["p50_ms"] = pct(lat, 50)
    res["p99_ms"] = pct(lat, 99)
    res["plain_solves_per_s"] = 1e3 / float(np.mean(lat))
    res["pcie_inclusive_sample_steps_per_s"] = prob.S * prob.T * res["plain_solves_per_s"]
    return res


def batched_leg(B, W, ctx):
    import torch

    h = ctx.h
    # ---- batched (one persistent launch in a HIP graph) vs plain per-instance ----
    insts = W.config3()
    for i, p in enumerate(insts):
        ctx.set_path(100 + i, p.path, p.ds)
    pbs = [B.ProblemBuffers(p, controller=100 + i) for i, p in enumerate(insts)]
    for pbi in pbs:
        B.brmppi_solve(h, pbi)
    torch.cuda.synchronize()
    reps_p = 3
    t0 = time.perf_counter()
    for _ in range(reps_p):
        for pbi in pbs:
            B.brmppi_solve(h, pbi)
    t_plain = (time.perf_counter() - t0) / reps_p
    bb = B.BatchBuffers(pbs)      # the call's arguments marshalled once, reused
    for _ in range(2):
        B.brmppi_solve_batch(h, bb)
    reps_b = 10
    t0 = time.perf_counter()
    for _ in range(reps_b):
        B.brmppi_solve_batch(h, bb)
    t_batch = (time.perf_counter() - t0) / reps_b
    ss = sum(p.S * p.T for p in insts)
    # algorithmic flops of the batch (one-lane rollouts, noise drawn in the
    # kernel) over the whole call's time: a lower bound on the rollout's rate
    fl = sum(rollout_flops(p.S, p.T, p.n_obs, hitch=not (p.flags & W.FLAG_HITCH_OFF),
                           guided=not (p.flags & W.FLAG_GUIDANCE_OFF)) for p in insts)
    return {
        "workload": "64 uneven instances: S in {1024..16384}, T in [20, 80], 0-16 obstacles",
        "tflops": fl / t_batch / 1e12, "frac": fl / t_batch / 1e12 / PEAK_FP32_TFLOPS,
        "frac_nonpacked": fl / t_batch / 1e12 / PEAK_FP32_NONPACKED_TFLOPS,
        "instances": len(insts), "plain_ms": t_plain * 1e3, "batched_ms": t_batch * 1e3,
        "plain_solves_per_s": len(insts) / t_plain, "batched_solves_per_s": len(insts) / t_batch,
        "speedup": t_plain / t_batch, "batched_sample_steps_per_s": ss / t_batch,
        "sample_steps": ss, "reduce_read_bytes": sum(12 * p.S * p.T + 4 * p.S for p in insts),
    }


def paper_leg(B, W, ctx):
    h = ctx.h
    # ---- the paper's experiment shape (Sec. V): 5000 rollouts, H = 120 steps,
    # its vehicle, seven e = 4 parked vehicles and a crossing e = 2 pedestrian,
    # on the reverse-parking scene; with the two MPPI baselines of its
    # comparison (plain MPPI, MPPI with a collision penalty) timed the same way
    pp = W.paper_shape()
    ps = {}
    for name, flags in (("br_mppi", 0), ("mppi", W.FLAG_GUIDANCE_OFF),
                        ("mppi_col", W.FLAG_GUIDANCE_OFF | W.FLAG_COLLISION_PENALTY)):
        q = pp.copy(flags=flags)
        ctx.set_path(2, q.path, q.ds)
        lat = []
        for k in range(40):
            _, st, _ = B.brmppi_solve(h, B.ProblemBuffers(q, controller=2, with_nominal=(k == 0), seed=k))
            if k >= 5:
                lat.append(st["latency_us"] * 1e-3)
        ps[name] = {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                    "paper_ms": W.PAPER_TIME_MS["backward"][name],
                    "paper_ms_forward": W.PAPER_TIME_MS["forward"][name]}
    return {"S": pp.S, "T": pp.T, "n_obs": pp.n_obs, **ps["br_mppi"], "paper_hw": "unnamed single GPU, JAX",
            "baselines": {"mppi": ps["mppi"], "mppi_col": ps["mppi_col"]},
            "note": "paper_ms: backward-parking times of the paper's comparison (its table of MPPI, MPPI + "
                    "collision cost, BR-MPPI); the scene here is reverse parking"}


def large_leg(B, W, ctx, tune_file):
    import torch

    h = ctx.h
    note("large solve")
    # ---- one large update (S = 65536, T = 100, 32 obstacles): enough waves to
    # fill every SIMD, so the rollout's fraction of peak is not occupancy-bound ----
    big = W.config5()
    ctx.set_path(3, big.path, big.ds)
    for k in range(2):
        B.brmppi_solve(h, B.ProblemBuffers(big, controller=3, with_nominal=(k == 0), seed=k))
    torch.cuda.synchronize()
    B.brmppi_profile_reset(h)
    lat = []
    for k in range(10):
        _, st, _ = B.brmppi_solve(h, B.ProblemBuffers(big, controller=3, with_nominal=False, seed=10 + k))
        lat.append(st["latency_us"] * 1e-3)
    prof = B.brmppi_profile_read(h)
    roll_ms = prof["rollout"]["ms"] / max(prof["rollout"]["count"], 1)
    noise_in_kernel = prof["noise"]["count"] == 0
    fl = rollout_flops(big.S, big.T, big.n_obs, noise_in_kernel=noise_in_kernel)
    ach = fl / (roll_ms * 1e-3) / 1e12
    shape = None
    try:
        shape = json.load(open(tune_file)).get("plain_32_3") if tune_file else None
    except (OSError, ValueError):
        pass
    # a table entry with precomputed normals falls back to the one-lane form
    # with in-kernel normals when the noise buffer does not fit: no noise launch
    if shape and noise_in_kernel and shape[1] != 0:
        shape = [shape[0], 0]
    return {"workload": "S=65536, T=100, 32 ellipses, three-piece spline path with cusps",
            "launch_shape": {"block_variant": shape},
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "sample_steps_per_s": big.S * big.T / (pct(lat, 50) * 1e-3),
            "rollout_ms": roll_ms, "noise_ms": prof["noise"]["ms"] / max(len(lat), 1),
            "rollout_tflops": ach, "rollout_frac": ach / PEAK_FP32_TFLOPS,
            "rollout_frac_nonpacked": ach / PEAK_FP32_NONPACKED_TFLOPS,
            "flops_per_launch": fl}


def served_replay(args, B, W, ctx, ctrls, n_active, seconds, base_id=300):
    """Real-time replay of the arrival process of the first n_active controllers
    (one request per 10 ms tick each, Exp(1 ms) jitter, a random phase), served
    by continuous batching; every controller runs its closed loop on the device.
    Returns the solves, the sample-steps, the algorithmic flops (one-lane
    rollouts, noise drawn in the kernel) and the latency of every request
    (submit to result ready, the library's clock)."""
    h = ctx.h
    pbs = []
    for c in range(n_active):
        p = ctrls[c]
        ctx.set_path(base_id + c, p.path, p.ds)
        B.brmppi_set_state(h, base_id + c, p.x0.astype(np.float64))
        flags = B.X0_RESIDENT | B.ADVANCE_PLANT
        pbs.append([B.ProblemBuffers(p, controller=base_id + c, with_nominal=True, flags=flags),
                    B.ProblemBuffers(p, controller=base_id + c, with_nominal=False, flags=flags)])
    events = W.config4_arrivals(n_active, seconds)
    started = [False] * n_active
    outstanding = []          # (ticket, T, sample-steps, flops)
    lat = []
    ss_total = 0
    fl_total = 0.0
    t_start = time.perf_counter()

    def take(block):
        nonlocal ss_total, fl_total
        t, T, ssk, flk = outstanding[0]
        if block:
            u, st, rc = B.brmppi_wait(h, t, T, timeout_ms=120000, allow=(B.OK, B.ENONFINITE))
        else:
            u, st, rc = B.brmppi_poll(h, t, T, allow=(B.OK, B.PENDING, B.ENONFINITE))
            if rc == B.PENDING:
                return False
        outstanding.pop(0)
        lat.append(st["latency_us"] * 1e-3)
        ss_total += ssk
        fl_total += flk
        return True

    for (te, c, k) in events:
        while time.perf_counter() - t_start < te:
            while outstanding and take(False):
                pass
        pb = pbs[c][1 if started[c] else 0]
        pb.c.seed = (4000 + c * 100003 + k) & (2**64 - 1)
        while True:
            t, rc = B.brmppi_submit(h, pb, allow=(B.OK, B.EAGAIN))
            if rc == B.OK:
                break
            take(True)        # back-pressure: the queue is full, wait for the oldest request
        started[c] = True
        p = ctrls[c]
        outstanding.append((t, pb.c.T, pb.c.S * pb.c.T, rollout_flops(p.S, p.T, p.n_obs)))
        while outstanding and take(False):
            pass
    while outstanding:
        take(True)
    wall = time.perf_counter() - t_start
    return events, pbs, lat, ss_total, fl_total, wall


def served_leg(args, B, W, ctx):
    ctrls = W.config4_controllers()
    n = len(ctrls)
    events, pbs, lat, ss_total, fl_total, wall = served_replay(args, B, W, ctx, ctrls, n, args.served_seconds)
    done = len(lat)
    # sequential plain solves of the same kind of requests (first 512 events)
    seq_events = events[:512]
    t0 = time.perf_counter()
    for (te, c, k) in seq_events:
        B.brmppi_solve(ctx.h, pbs[c][1], allow=(B.OK, B.ENONFINITE))
    t_seq = time.perf_counter() - t0
    out = {
        "workload": "256 controllers, S in {2048, 8192, 32768}, T in {30, 50, 100}, 0-32 obstacles "
                    "(10 % moving), one request per 10 ms tick + Exp(1 ms) jitter, closed loop on the device",
        "simulated_s": args.served_seconds, "requests": len(events), "wall_s": wall,
        "offered_per_s": len(events) / args.served_seconds,
        "solves_per_s": done / wall, "sample_steps_per_s": ss_total / wall,
        # algorithmic flops of the completed requests over the wall time (host
        # and reduce included): a lower bound on the rollouts' own rate
        "tflops": fl_total / wall / 1e12, "frac": fl_total / wall / 1e12 / PEAK_FP32_TFLOPS,
        "frac_nonpacked": fl_total / wall / 1e12 / PEAK_FP32_NONPACKED_TFLOPS,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "sequential_plain_solves_per_s": len(seq_events) / t_seq,
        "speedup_vs_sequential": (done / wall) / (len(seq_events) / t_seq),
    }
    # latency below capacity: the same mix with fewer controllers (offered load
    # n x 100 requests/s); the highest load whose p99 stays under the 10 ms tick
    sweep = []
    for n_active in [int(x) for x in args.served_sweep.split(",") if x]:
        ev, _, lt, ss, _, wl = served_replay(args, B, W, ctx, ctrls, min(n_active, n), args.sweep_seconds)
        sweep.append({"controllers": min(n_active, n), "offered_per_s": len(ev) / args.sweep_seconds,
                      "solves_per_s": len(lt) / wl, "p50_ms": pct(lt, 50), "p99_ms": pct(lt, 99),
                      "max_ms": float(np.max(lt)) if lt else None, "sample_steps_per_s": ss / wl})
        note(f"served at {sweep[-1]['offered_per_s']:.0f} requests/s: p50 {sweep[-1]['p50_ms']:.2f} ms, "
             f"p99 {sweep[-1]['p99_ms']:.2f} ms")
    out["load_sweep"] = sweep
    ok = [r for r in sweep if r["p99_ms"] is not None and r["p99_ms"] < 10.0]
    best = max(ok, key=lambda r: r["offered_per_s"]) if ok else None
    out["max_load_p99_under_tick"] = best
    # that load held for the 5 s the served workload specifies
    if best is not None and args.sustain_seconds > 0:
        ev, _, lt, ss, _, wl = served_replay(args, B, W, ctx, ctrls, best["controllers"], args.sustain_seconds)
        out["sustained"] = {"controllers": best["controllers"], "seconds": args.sustain_seconds,
                            "requests": len(ev), "offered_per_s": len(ev) / args.sustain_seconds,
                            "solves_per_s": len(lt) / wl, "p50_ms": pct(lt, 50), "p99_ms": pct(lt, 99),
                            "max_ms": float(np.max(lt)) if lt else None, "sample_steps_per_s": ss / wl}
        note(f"served for {args.sustain_seconds:.0f} s at {out['sustained']['offered_per_s']:.0f} requests/s: "
             f"p50 {out['sustained']['p50_ms']:.2f} ms, p99 {out['sustained']['p99_ms']:.2f} ms")
    return out


def host_cpu():
    """CPU model and thread counts of the host the oracle runs on"""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    # the machine's CPU share: OMP_NUM_THREADS when set (16 on the GPU host), else
    # every core this process may run on
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or avail
    return {"model": model, "nproc": os.cpu_count(), "affinity_cpus": avail, "threads": min(share, avail)}


def cpu_baseline(W, prob, seconds):
    """The FP64 oracle as it stands on the host cores: one c2 update (all
    S = 8192 samples) on every host thread of the share and on one thread, the
    c1 update likewise, and the 32-obstacle large update on a 512-sample
    subset.  value = the c2 update on all threads."""
    from oracle import oracle as O

    cpu = host_cpu()
    threads = cpu["threads"]
    O.solve(W.config1().copy(S=64), nthreads=threads)          # build + warm
    legs = {}

    def run(name, p, nthreads, budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            O.solve(p.copy(seed=p.seed + reps), nthreads=nthreads)
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                break
        legs[name] = {"sample_steps_per_s": p.S * p.T * reps / el, "solves_per_s": reps / el,
                      "threads": nthreads, "updates": reps, "seconds": el, "S": p.S, "T": p.T,
                      "n_obs": p.n_obs}

    share = seconds / 6.0
    run("c2_update_all_threads", prob, threads, share)
    run("c2_update_1_thread", prob, 1, share)
    c1 = W.config1()
    run("c1_update_all_threads", c1, threads, share / 2)
    run("c1_update_1_thread", c1, 1, share / 2)
    big = W.config5().copy(S=512)
    run("c5_512_samples_all_threads", big, threads, share)
    run("c5_512_samples_1_thread", big, 1, share)
    v = legs["c2_update_all_threads"]["sample_steps_per_s"]
    return {"value": v, "unit": "sample-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{legs['c2_update_all_threads']['updates']} full updates of the reverse-parking problem "
                      f"(S=8192, T=50, 8 obstacles) on {threads} threads; also one thread, the c1 update "
                      f"and 512 samples of the S=65536, T=100, 32-obstacle update (legs)",
            "host": cpu, "legs": legs}


if __name__ == "__main__":
    main()
