"""Benchmark: RandNet-Parareal on one MI355X.

One step = one complete RandNet-Parareal solve of the 192 x 192 shallow-water
workload (Rusanov finite volumes, reflective walls, g = 9.81, d = 110592,
N = 256 slices on t in [0, 1], F = RK4 with 1000 steps per slice, G = RK1
with 8 steps, 300 ReLU neurons, lambda = 1e-6): coarse sweep, then
iterations of fine solves of every unfinished slot (one launch over all of
them), training pairs, random features, ridge statistics, Cholesky solve,
predictor-corrector sweep and stopping rule, in mixed precision (FP32
states, split-bfloat16 features on the matrix cores, FP64 statistics,
Cholesky and change norms), run to the common accuracy tau: the solve stops
after the first iteration k whose iterate U^k satisfies E <= tau, with
E = mean over slices of max |U_i - U_ref,i| against the FP64 serial fine
solution and tau = 10 x E of the FP32 serial fine solution.  Inputs are
seeded synthetic data already in device memory when the timed region starts.

value = fine state-steps per second of that solve: (slot, fine RK4 step)
pairs it performs, sum over its iterations of the unfinished slots times
1000, divided by its wall time.  Beside it: the same accuracy reached by the
plain FP64 solve (time, k, E) and the ratio of the two times, both solves run
to the stopping rule eps = 1e-6, the roofline of the dominant kernel (the
one-pass RK4 fine propagator, timed live with HIP events on its launch
stream), the 64 x 64 diffusion-reaction workload in FP64, and the CPU oracle
timed on the host cores.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-cpu-baseline]
                    [--extra] [--copy-calibration] [--f-only swe_192x192|bruss_128x128 [--shape S]]
                    [--solve-only NAME] [--gemm] [--robustness] [--model-only]
                    [--sweep-only 256|1024] [--trace-summary CSV] [--segment-summary CSV]
                    [--trace-window CSV NAME GRID SKIP COUNT]

--extra adds one FP64 and one mixed-precision solve of the other workloads
(Burgers d = 128; Brusselator 128 x 128; the 3D Brusselator 20^3 with the
eighth-order fine solver; the batch of 64 Burgers problems),
which takes minutes.  --copy-calibration runs a device copy of 256 MiB, the
reference a hardware-counter run uses to scale its byte counters.  --f-only
times only the fine propagator of the named workload (all N slot states,
--steps RK4 steps, FP64 and FP32; --shape pins a tile shape of the one-pass
kernel where the precision has it) and prints its roofline, for counter runs;
--model-only times the model phase's FP64 matrix products (features, ridge
fit) at the shallow-water shape, for counter runs; --sweep-only runs the
reduced shallow-water solve for one iteration with its sweeps in work-groups
of the given size, for kernel traces (--segment-summary reads them).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # MI355X HBM3E bytes/s (AMD specification)
FP64_VECTOR_PEAK = 78.6e12   # MI355X FP64 vector FLOP/s (AMD specification)
FP32_VECTOR_PEAK = 157.3e12  # MI355X FP32 vector FLOP/s (AMD specification; packed FP32)
# Algorithmic FP64 operations per degree of freedom and classical RK4 step of
# the diffusion-reaction stencil, counted from the formulas (a fused
# multiply-add counts as two): per cell and stage, two 5-point Laplacians
# 2 x 9, the u reaction 7, the v reaction 3, the stage updates 2 x 3.25 on
# average over the four stages = 34.5 per cell-stage = 17.25 per DOF-stage.
# Shallow water, per cell and stage (3 DOF): per-cell quantities 16 (1/h, two
# velocities, sqrt(g h) 2, g h^2 / 2 2, three flux terms and a wave speed per
# direction 8), one x face and one y face 13 each (speed max 1, three
# components of (f_L + f_R)/2 - a (q_R - q_L)/2 at 4), flux differences and
# slopes 15, stage update 12 = 69 per cell-stage = 92 per DOF-step.
FLOPS_PER_DOF_STEP = {"diffreact": 4 * 17.25, "swe": 4 * 69 / 3}
# Algorithmic HBM bytes per DOF and RK4 step of the fine propagator: read the
# state and write it once (the minimum of any F); the FP32 compensation the
# one-pass kernels also carry is traffic beyond it.
ALGO_BYTES_PER_DOF_STEP = {8: 16, 4: 8}

# HBM bytes per launch (one RK4 step of the 256 FP32 shallow-water states) of
# the one-pass fine propagator, from one FETCH_SIZE and one WRITE_SIZE
# hardware-counter run (KiB per dispatch), each scaled by what the counter
# reads for a device copy of known size.  Valid only for the kernel sources
# they were taken on (hash below); any change to them makes the field null
# until the counters are taken again.
PROP_SOURCES = ("paper_2411_06225_amd/csrc/swefused.h", "paper_2411_06225_amd/csrc/tiled.hip",
                "paper_2411_06225_amd/csrc/tiledprop.h", "paper_2411_06225_amd/csrc/slotprop.h",
                "paper_2411_06225_amd/csrc/common.h")
PROP_TRAFFIC = {"sources": "0e929cc303205708", "fetch_scale": 2.0, "write_scale": 1.0,
                # tile shape -> (FETCH_SIZE, WRITE_SIZE) KiB per steady-state
                # dispatch (compensation read and written), FP32, 256 states
                "shapes": {"R5NW8": (110682.5, 221285.3), "R4NW8": (110670.7, 221190.2)}}


def sources_hash(paths):
    """First 16 hex digits of the SHA-1 of the files' SHA-1 digests in order."""
    import hashlib
    digests = "".join(hashlib.sha1(open(os.path.join(ROOT, p), "rb").read()).hexdigest() for p in paths)
    return hashlib.sha1(digests.encode()).hexdigest()[:16]


def measured_traffic(shape):
    """HBM bytes per dispatch of the fine propagator in tile shape `shape`,
    or None when no counters were taken on these sources for that shape."""
    t = PROP_TRAFFIC
    if t["sources"] is None or sources_hash(PROP_SOURCES) != t["sources"] or shape not in t["shapes"]:
        return None
    fetch_kib, write_kib = t["shapes"][shape]
    return (fetch_kib * t["fetch_scale"] + write_kib * t["write_scale"]) * 1024


def swe_kernel_name(shape, real="float"):
    """The kernel that a one-pass shallow-water tile shape launches."""
    import re
    m = re.fullmatch(r"rows:C(\d+)R(\d+)NW(\d+)", shape)
    if m:
        return f"k_prop_swe_rows<{real}, {m[1]}, {m[2]}, {m[3]}>"
    m = re.fullmatch(r"R(\d+)NW(\d+)", shape)
    return f"k_prop_swe_fused<{real}, {m[1]}, {m[2]}>" if m else shape


def chosen_shape(rpr, w, prec):
    """The tile shape the autotuner chose for workload w's fine propagator
    (the default shape when it has not run)."""
    v = rpr.rpr_tune_get(rpr.prop_tune_key(w.kind, w.nx, w.ny, prec, w.F[0]) + ":v")
    return rpr.tile_shapes(w.kind, prec)[v or 0]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extra", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--solve-only", choices=["burgers_d128", "bruss_128x128", "swe_192x192", "bruss3d_20"],
                    default=None,
                    help="only run the --extra solves of this workload (for traces)")
    ap.add_argument("--gemm", action="store_true",
                    help="only time the random-feature GEMMs at the workloads' shapes and a compute-bound one")
    ap.add_argument("--robustness", action="store_true",
                    help="only run the sweep over neighbour counts, neurons and weight draws (App. D)")
    ap.add_argument("--robustness-grid", choices=["reduced", "paper"], default="reduced",
                    help="reduced: 8 m x 6 M x 10 draws in one batch per system; paper: App. D's "
                         "19 m x 49 M x 100 draws, one batch per draw")
    ap.add_argument("--sweep-only", type=int, choices=[256, 1024], default=None,
                    help="one-iteration reduced shallow-water solve, sweeps on 256 work-groups of this size")
    ap.add_argument("--segment-summary", default=None,
                    help="summarise the sweep segments of a kernel trace of --sweep-only (CSV path)")
    ap.add_argument("--trace-window", nargs=5, metavar=("CSV", "NAME", "GRID", "SKIP", "COUNT"), default=None,
                    help="mean duration of COUNT dispatches of a kernel, ending SKIP before its last one")
    ap.add_argument("--shape", default=None,
                    help="with --f-only: pin this tile shape of the one-pass kernel (names: rpr.tile_shapes)")
    ap.add_argument("--f-only", choices=["swe_192x192", "bruss_128x128"], default=None,
                    help="only time the fine propagator of this workload in FP64 and FP32 (for counter runs)")
    ap.add_argument("--trace-summary", metavar="CSV", default=None,
                    help="summarise a rocprofv3 kernel trace (CSV) per kernel and grid size, then exit")
    ap.add_argument("--model-only", action="store_true",
                    help="only time the model phase's FP64 matrix products at the shallow-water shape "
                         "(for counter runs)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def trace_summary(path, top=25):
    """Per kernel name and grid size of a rocprofv3 kernel trace: dispatches,
    mean and spread of the duration (the launches of one kernel over slot
    batches of different sizes have different grids, so a plan's launches
    and single-state ones are told apart)."""
    import csv
    from collections import defaultdict
    groups = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            if "Grid_Size" in r:
                grid = int(r["Grid_Size"])
            else:
                grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            groups[(r["Kernel_Name"], grid)].append(dur)
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]
    print("| kernel | grid (threads) | dispatches | mean us | min us | max us | total ms |")
    print("|---|---|---|---|---|---|---|")
    for (name, grid), v in rows:
        short = name.split("(")[0].replace("void ", "")
        print(f"| `{short}` | {grid} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {min(v) / 1e3:.2f} | "
              f"{max(v) / 1e3:.2f} | {sum(v) / 1e6:.3f} |")


def trace_window(path, name, grid, skip, count):
    """Mean and median duration of `count` dispatches of the kernel whose
    name contains `name` at grid size `grid`, ending `skip` dispatches before
    its last one (in time order): the launches of one timed solve."""
    import csv
    import statistics as stt
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    g = lambda r: int(r["Grid_Size"]) if "Grid_Size" in r else \
        int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows
         if name in r["Kernel_Name"] and g(r) == grid]
    win = d[len(d) - skip - count:len(d) - skip]
    print(json.dumps({"kernel": name, "grid": grid, "dispatches": len(d), "window": [len(d) - skip - count,
                      len(d) - skip], "mean_us": stt.mean(win), "median_us": stt.median(win)}))


def segment_summary(path, N=256):
    """The sweep's segment kernels in a kernel trace of `bench.py
    --sweep-only`, in dispatch order: a sweep of N slots is a prologue, N - 1
    pairs (phase 1: coarse pass and hidden layer of slot i; phase 2: readout,
    update, change norm, hidden-layer partial sums of slot i) and the
    stopping rule; the k = 0 sweep's coarse passes are k_sweep_pass."""
    import csv
    import statistics as stt
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    seg = [r for r in rows if "k_chain_seg" in r["Kernel_Name"]]
    sw = [dur(r) for r in rows if "k_sweep_pass" in r["Kernel_Name"]]
    print("| sweep | kernel | prologue us | phase 1 us (mean / median) | phase 2 us (mean / median) | "
          "stopping rule us | sweep ms |")
    print("|---|---|---|---|---|---|---|")
    for s0 in range(0, len(seg) - 2 * N + 1, 2 * N):
        sweep = seg[s0:s0 + 2 * N]
        p1 = [dur(r) for r in sweep[1:-1:2]]
        p2 = [dur(r) for r in sweep[2:-1:2]]
        name = sweep[1]["Kernel_Name"].split("(")[0].replace("void ", "")
        print(f"| {s0 // (2 * N) + 1} | `{name}` | {dur(sweep[0]):.1f} | {stt.mean(p1):.2f} / {stt.median(p1):.2f} | "
              f"{stt.mean(p2):.2f} / {stt.median(p2):.2f} | {dur(sweep[-1]):.1f} | "
              f"{sum(map(dur, sweep)) / 1e3:.2f} |")
    if sw:
        print(f"\nk = 0 sweep coarse passes (k_sweep_pass): {len(sw)} dispatches, mean {stt.mean(sw):.2f} us")


def sweep_only(torch, rpr, W, dev, block):
    """The reduced-precision shallow-water solve stopped after one
    iteration, its sweeps in segment kernels on 256 work-groups of `block`
    threads (pinned in the autotuner's table), run twice: the trace of it
    shows each segment's duration."""
    w = W.SWE_192
    h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params)
    A, z = W.random_weights(w)
    u0 = torch.tensor(W.initial_condition(w), dtype=torch.float64, device=dev)
    key = rpr.chain_tune_key(w.kind, w.nx, w.ny, rpr.RPR_MIXED, w.M, w.N)
    rpr.rpr_tune_set(key, 256)
    rpr.rpr_tune_set(key + ":B", block)
    p = rpr.Plan(h, w.d, w.t0, w.tN, w.N, F=w.F, G=w.G, tol=w.eps, M=w.M, activation=w.act, lam=w.lam, A=A,
                 zeta=z, precision=rpr.RPR_MIXED, k_max=1, autotune=1)
    U = torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev)
    for _ in range(2):
        p.execute(u0, U)
        torch.cuda.synchronize()
    info = p.info()
    p.close()
    return {"block": block, "sweep_s": info["t_sweep"], "total_s": info["t_total"]}


def main():
    args = parse()
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.segment_summary:
        segment_summary(args.segment_summary)
        return
    if args.trace_window:
        path, name, grid, skip, count = args.trace_window
        trace_window(path, name, int(grid), int(skip), int(count))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2411_06225_amd as rpr
    from paper_2411_06225_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.gemm:
        print(json.dumps({"feature_gemm": gemm_demo(torch, rpr, dev)}))
        return
    if args.solve_only:
        print(json.dumps({"extra": extra_workloads(torch, rpr, W, dev, only=args.solve_only)}))
        return
    if args.robustness:
        if args.robustness_grid == "paper":
            # App. D: m = 2..20, M = 20..500 in steps of 10, 100 weight draws;
            # one batch per draw
            res = robustness_sweep(torch, rpr, W, dev, n_seeds=100, ms=tuple(range(2, 21)),
                                   Ms=tuple(range(20, 501, 10)), seeds_per_batch=1)
        else:
            res = robustness_sweep(torch, rpr, W, dev)
        print(json.dumps({"robustness": res}))
        return
    if args.sweep_only:
        print(json.dumps({"sweep_only": sweep_only(torch, rpr, W, dev, args.sweep_only)}))
        return
    if args.model_only:
        print(json.dumps({"model_fp64": model_roofline(torch, rpr, W, dev, reps=max(args.steps, 1))}))
        return
    if args.f_only:
        wf = W.WORKLOADS[args.f_only]
        if args.shape:
            for prec in (rpr.RPR_FP64, rpr.RPR_MIXED):
                names = rpr.tile_shapes(wf.kind, prec)
                if args.shape in names:
                    rpr.rpr_tune_set(rpr.prop_tune_key(wf.kind, wf.nx, wf.ny, prec, wf.F[0]) + ":v",
                                     names.index(args.shape))
        cb = copy_bandwidth(torch, dev)
        res = {"workload": wf.name, "F_roofline": {
            "fp64": f_roofline(torch, rpr, wf, rpr.RPR_FP64, dev, steps=args.steps, copy_bw=cb),
            "fp32": f_roofline(torch, rpr, wf, rpr.RPR_MIXED, dev, steps=args.steps, copy_bw=cb)}}
        if args.copy_calibration:
            res["copy_calibration_bytes"] = copy_calibration(torch, dev)
        print(json.dumps(res))
        return

    w = W.SWE_192
    h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params)
    u0h = W.initial_condition(w)
    A, zeta = W.random_weights(w)
    u0 = torch.tensor(u0h, dtype=torch.float64, device=dev)
    T = (w.tN - w.t0) / w.N
    plans = []

    def make_plan(prec, k_max=0):
        p = rpr.Plan(h, w.d, w.t0, w.tN, w.N, F=w.F, G=w.G, tol=w.eps, M=w.M, activation=w.act, lam=w.lam,
                     A=A, zeta=zeta, precision=prec, autotune=1, k_max=k_max)
        plans.append(p)
        return p

    def timed_solves(plan, steps, warmup):
        U = torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev)
        for _ in range(warmup):
            plan.execute(u0, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(steps, 1)):
            plan.execute(u0, U)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / max(steps, 1), U

    def fine_state_steps(plan):
        Lh, _ = plan.history()
        K = plan.info()["K"]
        return sum(w.N - int(Lh[k - 1]) for k in range(1, K + 1)) * w.F[1]

    # serial fine reference on the GPU (same F kernel, slot after slot) in
    # FP64 (the reference of E) and FP32 (its error sets tau)
    def serial_fine(prec_dtype, prec_code):
        cur = u0.to(prec_dtype)[None].contiguous()
        out = [cur[0].double().clone()]
        for _ in range(w.N):
            nxt = torch.empty_like(cur)
            rpr.rpr_propagate(h, w.d, w.F[0], w.F[1], prec_code, T / w.F[1], 1, cur, nxt)
            cur = nxt
            out.append(cur[0].double().clone())
        torch.cuda.synchronize()
        return torch.stack(out)

    t_sf = time.perf_counter()
    Uf = serial_fine(torch.float64, rpr.RPR_FP64)
    t_sf = time.perf_counter() - t_sf
    E = lambda U: float((U[1:] - Uf[1:]).abs().amax(dim=1).mean())
    E32floor = E(serial_fine(torch.float32, rpr.RPR_MIXED))
    tau = 10.0 * E32floor
    log(f"serial fine {t_sf:.2f} s; FP32 floor E = {E32floor:.3e}, tau = {tau:.3e}")

    # both precisions to the stopping rule (eps = 1e-6): K, E, time
    natural = {}
    for name, prec in (("fp64", rpr.RPR_FP64), ("mixed", rpr.RPR_MIXED)):
        p = make_plan(prec)
        t, U = timed_solves(p, 1, 1)
        natural[name] = {"s": t, "K": p.info()["K"], "E": E(U)}
        log(f"{name} to eps: {t:.3f} s, K = {natural[name]['K']}, E = {natural[name]['E']:.3e}")

    def first_k_to_tau(prec, k_stop):
        """First k whose iterate U^k has E <= tau (a solve stopped after k
        iterations does exactly the work of the first k)."""
        for k in range(1, k_stop + 1):
            p = make_plan(prec, k_max=k)
            _, Uk = timed_solves(p, 1, 0)
            if E(Uk) <= tau:
                return k, p
        return None, None

    k64, p64 = first_k_to_tau(rpr.RPR_FP64, natural["fp64"]["K"])
    k32, p32 = first_k_to_tau(rpr.RPR_MIXED, natural["mixed"]["K"])
    if k32 is None:
        print(json.dumps({"error": f"the mixed-precision solve does not reach tau = {tau:.3e}"}))
        sys.exit(1)
    # the timed steps: the mixed solve to tau
    sec, Um = timed_solves(p32, args.steps, args.warmup)
    info = p32.info()
    value = fine_state_steps(p32) / sec
    log(f"mixed to tau: k = {k32}, {sec * 1e3:.1f} ms per solve")
    t64 = None
    if k64 is not None:
        t64, U64 = timed_solves(p64, 2, 1)
        log(f"fp64 to tau: k = {k64}, {t64 * 1e3:.1f} ms per solve")

    # roofline of the dominant kernel, the one-pass fine propagator, live
    # over the timed region: the plan records HIP events on its stream around
    # the fine-solve launches of each iteration (info t_fine); launch j of
    # iteration k advances the N - L_{k-1} unfinished slot states by one RK4
    # step, so its algorithmic bytes are 8 B (read and write an FP32 value)
    # per DOF of those states
    fine_launches = k32 * w.F[1]
    f_launch = info["t_fine"] / fine_launches
    algo_bytes = ALGO_BYTES_PER_DOF_STEP[4] * w.d * fine_state_steps(p32) / fine_launches
    achieved = algo_bytes / f_launch
    flops = FLOPS_PER_DOF_STEP["swe"] * w.d * fine_state_steps(p32) / fine_launches
    # the same kernel alone over all N states, 20 launches, for reference
    X = Um[:-1].float().contiguous()
    Y = torch.empty_like(X)
    stream = torch.cuda.current_stream()
    f_steps = 20
    rpr.rpr_propagate(h, w.d, w.F[0], 2, rpr.RPR_MIXED, T / w.F[1], w.N, X, Y, stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    rpr.rpr_propagate(h, w.d, w.F[0], f_steps, rpr.RPR_MIXED, T / w.F[1], w.N, X, Y, stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    alone = ev[0].elapsed_time(ev[1]) / 1e3 / f_steps
    shape = chosen_shape(rpr, w, rpr.RPR_MIXED)
    traffic = measured_traffic(shape)
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK,
                "traffic": traffic * algo_bytes / (ALGO_BYTES_PER_DOF_STEP[4] * w.d * w.N) if traffic else None,
                "kernel": swe_kernel_name(shape) + " (fine RK4, one launch per step, shallow water 192x192)",
                "tile_shape": shape,
                "launch": {"launches": fine_launches, "ms": f_launch * 1e3, "algorithmic_bytes": algo_bytes,
                           "bytes_per_dof_step": ALGO_BYTES_PER_DOF_STEP[4],
                           "alu_TFLOPs": flops / f_launch / 1e12,
                           "alu_frac_of_fp32_peak": flops / f_launch / FP32_VECTOR_PEAK,
                           "flops_per_dof_step": FLOPS_PER_DOF_STEP["swe"],
                           "all_N_states_ms": alone * 1e3}}

    out = {
        "metric": "time-to-tolerance (s) & fine state-steps/s, mixed vs FP64 plain, 1 MI355X",
        "value": value,
        "unit": "fine state-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "d": w.d, "N": w.N, "t": [w.t0, w.tN], "F": f"RK4x{w.F[1]}",
                   "G": f"RK1x{w.G[1]}", "M": w.M, "activation": "relu", "lambda": w.lam, "eps": w.eps,
                   "precision": "mixed (FP32 states, split-bf16 MFMA features, FP64 ridge and norms)",
                   "stop": "first iterate with E <= tau"},
        "time_to_tolerance_s": sec,
        "tau": tau,
        "fp32_serial_fine_error_floor": E32floor,
        "mixed": {"k": k32, "s": sec, "E": E(Um), "dof_steps_per_s": value * w.d,
                  "phases_s": {"total": info["t_total"], "fine": info["t_fine"], "model": info["t_model"],
                               "sweep": info["t_sweep"]}},
        "fp64": {"k": k64, "s": t64, "E": E(U64) if t64 else None},
        "fp64_over_mixed_time_to_tau": (t64 / sec) if t64 else None,
        "to_eps": natural,
        "serial_fine_fp64_s": t_sf,
        "speedup_vs_serial_fine": t_sf / sec,
        "roofline": roofline,
    }
    for p in plans:
        p.close()
    plans.clear()

    # the 64 x 64 diffusion-reaction workload, plain FP64, to the stopping rule
    out["diffreact_64x64_fp64"] = diffreact_line(torch, rpr, W, dev)

    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration(torch, dev)
    if args.extra:
        out["extra"] = extra_workloads(torch, rpr, W, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, u0h, T, natural["fp64"]["K"], k64)
    print(json.dumps(out))


def diffreact_line(torch, rpr, W, dev):
    """One FP64 solve of the diffusion-reaction workload (d = 8192, N = 64):
    time, K, fine state-steps/s and E against its FP64 serial fine solution."""
    w = W.DIFFREACT_64
    h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params)
    A, zeta = W.random_weights(w)
    u0 = torch.tensor(W.initial_condition(w), dtype=torch.float64, device=dev)
    T = (w.tN - w.t0) / w.N
    def timed(graph):
        plan = rpr.Plan(h, w.d, w.t0, w.tN, w.N, F=w.F, G=w.G, tol=w.eps, M=w.M, activation=w.act, lam=w.lam,
                        A=A, zeta=zeta, autotune=1, graph=graph)
        U = torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev)
        plan.execute(u0, U)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.execute(u0, U)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        Lh, _ = plan.history()
        K = plan.info()["K"]
        plan.close()
        return sec, U, K, sum(w.N - int(Lh[k - 1]) for k in range(1, K + 1)) * w.F[1]

    sec, U, K, steps = timed(0)
    # the same solve with each block of iterations captured as a graph (the
    # sweeps as segment kernels on the same grid: bitwise the same result)
    gsec, Ug, gK, _ = timed(1)
    same = bool(torch.equal(Ug, U))
    cur = u0[None].contiguous()
    ref = [cur[0].clone()]
    for _ in range(w.N):
        nxt = torch.empty_like(cur)
        rpr.rpr_propagate(h, w.d, w.F[0], w.F[1], rpr.RPR_FP64, T / w.F[1], 1, cur, nxt)
        cur = nxt
        ref.append(cur[0].clone())
    Uf = torch.stack(ref)
    E = float((U[1:] - Uf[1:]).abs().amax(dim=1).mean())
    return {"s": sec, "K": K, "fine_state_steps_per_s": steps / sec, "E_vs_serial_fine": E,
            "graph": {"s": gsec, "K": gK, "bitwise_equal_to_plain_launches": same}}


def host_cpus():
    """CPUs this process may run on, the OpenMP-style thread cap the host
    sets (if any), and the CPU model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    threads = min(avail, int(cap)) if cap and cap.isdigit() and int(cap) > 0 else avail
    model = platform.processor() or ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "affinity": avail, "threads": threads, "model": model}


def cpu_baseline(w, u0h, T, K64, k64):
    """The FP64 C oracle on the host: fine slot solves of the benchmark
    workload (RK4 x 1000 steps on d = 110592), on every CPU the process may
    use (one slot per thread, as the paper runs one fine solve per core) and
    on one thread; bounded samples, scaled to fine state-steps/s.  A whole
    oracle solve is extrapolated from the measured rates: per iteration k the
    fine solves of the unfinished slots on all threads, plus the coarse sweep
    (N forward-Euler slices, one thread, timed on one slice)."""
    import oracle
    cpus = host_cpus()
    threads = cpus["threads"]
    pb = oracle.problem(w.kind, w.nx, w.ny, w.domain, w.params)
    dtF, dtG = T / w.F[1], T / w.G[1]
    # all threads: one slot each, 1500 RK4 steps (about 7 s)
    steps_all = 1500
    X = np.tile(u0h, (threads, 1))
    t0 = time.perf_counter()
    oracle.propagate_many(pb, w.F[0], steps_all, dtF, X, nthreads=threads)
    t_all = time.perf_counter() - t0
    rate_all = threads * steps_all / t_all
    # one thread: one slot, 1000 RK4 steps (about 5 s)
    steps_one = 1000
    t0 = time.perf_counter()
    oracle.propagate(pb, w.F[0], steps_one, dtF, u0h)
    t_one = time.perf_counter() - t0
    rate_one = steps_one / t_one
    t0 = time.perf_counter()
    oracle.propagate(pb, w.G[0], w.G[1], dtG, u0h)
    t_g = time.perf_counter() - t0
    # whole solve to the stopping rule and to tau (no slot final before its
    # exact iteration: at most N - k + 1 slots at iteration k)
    def solve_s(K):
        fine = sum(w.N - k + 1 for k in range(1, K + 1)) * w.F[1] / rate_all
        return fine + (K + 1) * w.N * t_g
    return {"value": rate_all, "unit": "fine state-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} fine slot solves of {steps_all} RK4 steps (d = {w.d}) by the FP64 C oracle on "
                      f"{threads} threads, {t_all:.1f} s; one thread: 1 slot x {steps_one} steps, {t_one:.1f} s",
            "one_thread": {"value": rate_one, "unit": "fine state-steps/s"},
            "host": cpus,
            "extrapolated_solve_s": {"to_eps_K": K64, "to_eps": solve_s(K64),
                                     "to_tau_k": k64, "to_tau": solve_s(k64) if k64 else None,
                                     "note": "extrapolated from the sampled rates, not run whole; the fine "
                                             "solves bound it from below"}}


def copy_calibration(torch, dev):
    """A plain device copy of 256 MiB: a counter run scales FETCH_SIZE and
    WRITE_SIZE by what they read for it."""
    a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    return a.numel() * 8


def copy_bandwidth(torch, dev, mib=1024, reps=5):
    """Device-to-device copy rate (bytes read + bytes written per second) of
    a mib-MiB buffer, HIP events: the measured HBM ceiling beside the
    specification's."""
    a = torch.ones(mib * 1024 * 1024 // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        b.copy_(a)
    ev[1].record()
    torch.cuda.synchronize()
    return 2 * a.numel() * 8 * reps / (ev[0].elapsed_time(ev[1]) / 1e3)


def f_roofline(torch, rpr, w, prec, dev, steps=20, copy_bw=None):
    """Time one launch of the fine propagator over all N slot states of
    workload w (steps RK4 steps, one launch per step: the one-pass RK4 tile
    kernels of the Laplacian systems and of shallow water) with HIP events on
    its stream, and relate its algorithmic bytes (read and write the state
    once per step) to the HBM peak; the FP32 compensation the kernels also
    read and write, and the halo re-reads, are traffic beyond them."""
    h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params)
    from paper_2411_06225_amd import workloads as W
    dtype = torch.float64 if prec == rpr.RPR_FP64 else torch.float32
    esz = 8 if prec == rpr.RPR_FP64 else 4
    X = torch.tensor(W.initial_condition(w), dtype=dtype, device=dev)[None].repeat(w.N, 1).contiguous()
    Y = torch.empty_like(X)
    dt = (w.tN - w.t0) / w.N / w.F[1]
    stream = torch.cuda.current_stream()
    # the tiled form, also where a state would fit one work-group's LDS
    rpr.rpr_propagate(h, w.d, w.F[0], 2, prec, dt, w.N, X, Y, stream, threads=256)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    rpr.rpr_propagate(h, w.d, w.F[0], steps, prec, dt, w.N, X, Y, stream, threads=256)
    ev[1].record(stream)
    torch.cuda.synchronize()
    sec = ev[0].elapsed_time(ev[1]) / 1e3
    bpd = ALGO_BYTES_PER_DOF_STEP[esz]
    bytes_ = w.N * w.d * steps * bpd
    achieved = bytes_ / sec
    if w.kind == rpr.RPR_SWE2D:
        shape = chosen_shape(rpr, w, prec)
        kernel = swe_kernel_name(shape, "double" if prec == rpr.RPR_FP64 else "float")
    else:
        shape, kernel = None, "k_prop_rk4_fused"
    kernel += " (fine RK4, one launch per step)"
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "kernel": kernel, "tile_shape": shape,
            "measured_copy_GBps": copy_bw / 1e9 if copy_bw else None,
            "frac_of_copy": achieved / copy_bw if copy_bw else None,
            "launch": {"slots": w.N, "steps": steps, "ms_per_step": sec * 1e3 / steps,
                       "algorithmic_bytes_per_dof_step": bpd}}


BF16_MFMA_PEAK = 2.5e15  # MI355X dense bf16 matrix FLOP/s (AMD specification)
FP64_MFMA_PEAK = 78.6e12  # MI355X dense FP64 matrix FLOP/s (AMD specification)


def model_roofline(torch, rpr, W, dev, reps=5):
    """The model phase's FP64 matrix products at the shallow-water 192 x 192
    shape (n = N = 256 training rows, M = 300 neurons, d = 110592): the
    feature GEMM Phi = sigma(X A^T / s + zeta) (rpr_randnet_features, 2 n M d
    FLOP) and the ridge fit (rpr_ridge_fit: Gram 2 n M^2, B = Phi^T Y 2 n M d,
    Cholesky M^3 / 3 and the two triangular solves 2 M^2 d FLOP), each
    timed over `reps` calls with HIP events and related to the FP64
    matrix-core peak on those algorithmic FLOP.  Whole calls: workspace
    allocation and the one-work-group Cholesky are included (the kernels'
    own times are in the profiles)."""
    w = W.SWE_192
    n, M, d = w.N, w.M, w.d
    g = torch.Generator(device="cpu").manual_seed(n + M + d)
    A = (torch.rand((M, d), generator=g, dtype=torch.float64) * 2 - 1).to(dev)
    z = (torch.rand((M,), generator=g, dtype=torch.float64) * 2 - 1).to(dev)
    X = (torch.rand((n, d), generator=g, dtype=torch.float64) * 2).to(dev)
    Y = (torch.randn((n, d), generator=g, dtype=torch.float64) * 1e-3).to(dev)
    Phi = torch.empty((n, M), dtype=torch.float64, device=dev)
    Wt = torch.empty((M, d), dtype=torch.float64, device=dev)

    def timed(fn):
        fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / 1e3 / reps

    t_feat = timed(lambda: rpr.rpr_randnet_features(M, d, n, rpr.RPR_RELU, 2.0, A, z, X, Phi))
    t_fit = timed(lambda: rpr.rpr_ridge_fit(M, d, n, Phi, Y, w.lam, Wt))
    f_feat = 2.0 * n * M * d
    f_fit = 2.0 * n * M * M + 2.0 * n * M * d + M ** 3 / 3.0 + 2.0 * M * M * d
    out = {"shape": {"n": n, "M": M, "d": d},
           "features": {"ms": t_feat * 1e3, "TFLOPs": f_feat / t_feat / 1e12,
                        "frac_of_fp64_mfma_peak": f_feat / t_feat / FP64_MFMA_PEAK},
           "ridge_fit": {"ms": t_fit * 1e3, "TFLOPs": f_fit / t_fit / 1e12,
                         "frac_of_fp64_mfma_peak": f_fit / t_fit / FP64_MFMA_PEAK}}
    log(f"model shapes: features {t_feat * 1e3:.3f} ms, ridge fit {t_fit * 1e3:.3f} ms")
    return out


def gemm_demo(torch, rpr, dev, reps=5):
    """The random-feature GEMM Z = (X / s) A^T (eq. "HA"; n rows, M neurons,
    K = d) through rpr_randnet_features_bf16 (split bfloat16, six MFMA
    products per output) and rpr_randnet_features (FP64), at the shapes of
    the diffusion-reaction and shallow-water workloads and at a compute-bound
    shape.  Times are whole calls (weight splitting and workspace included;
    kernel times are in the profiles); 'useful' counts 2 n M d FLOP, 'mfma'
    the 6 x 2 n M d the matrix cores execute."""
    res = []
    for n, M, d in ((64, 200, 8192), (256, 300, 110592), (512, 512, 32768), (1024, 512, 65536)):
        g = torch.Generator(device="cpu").manual_seed(n + M + d)
        A = (torch.rand((M, d), generator=g, dtype=torch.float64) * 2 - 1).to(dev)
        z = (torch.rand((M,), generator=g, dtype=torch.float64) * 2 - 1).to(dev)
        X64 = (torch.rand((n, d), generator=g, dtype=torch.float64) * 2 - 1).to(dev)
        X32 = X64.float()
        Phi = torch.empty((n, M), dtype=torch.float64, device=dev)
        row = {"n": n, "M": M, "d": d}
        for name, fn, X in (("bf16_split", rpr.rpr_randnet_features_bf16, X32),
                            ("fp64", rpr.rpr_randnet_features, X64)):
            fn(M, d, n, 1, 1.0, A, z, X, Phi)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(reps):
                fn(M, d, n, 1, 1.0, A, z, X, Phi)
            ev[1].record()
            torch.cuda.synchronize()
            sec = ev[0].elapsed_time(ev[1]) / 1e3 / reps
            useful = 2.0 * n * M * d
            r = {"ms": sec * 1e3, "useful_TFLOPs": useful / sec / 1e12}
            if name == "bf16_split":
                r["mfma_TFLOPs"] = 6 * useful / sec / 1e12
                r["mfma_frac_of_peak"] = 6 * useful / sec / BF16_MFMA_PEAK
            else:
                r["frac_of_fp64_peak"] = useful / sec / FP64_VECTOR_PEAK
            row[name] = r
        res.append(row)
        print(f"gemm n={n} M={M} d={d}: bf16 {row['bf16_split']['ms']:.3f} ms, fp64 {row['fp64']['ms']:.3f} ms",
              file=sys.stderr, flush=True)
        del A, X64, X32
    return res


def robustness_sweep(torch, rpr, W, dev, n_seeds=10, ms=(2, 3, 4, 6, 8, 12, 16, 20),
                     Ms=(20, 50, 100, 200, 300, 500), seeds_per_batch=None):
    """Iterations to convergence K of RandNet-Parareal with the per-prediction
    refit on the m nearest pairs (eq. "randnet"), over neighbour counts m,
    neuron counts M and independent draws of the weights A, zeta: the study
    of App. D, on a Burgers system with d = 128 and a diffusion-reaction
    system with d = 722 (19 x 19 cells, two species).  Every (draw, m, M)
    combination is one instance of one batch plan (same initial state, its
    own weights), so each system is a single batched solve, or one per
    `seeds_per_batch` weight draws when the grid is large.  Returns, per
    system, the histograms of K by m and by M, and K of classical Parareal
    on the same problem for reference.  Progress goes to stderr."""
    from collections import Counter

    def hist(c):
        return dict(sorted(c.items(), key=lambda kv: int(kv[0]) if kv[0].isdigit() else 1 << 30))

    systems = {
        "burgers_d128": W.BURGERS_D128_STABLE,
        "diffreact_19x19": W.small(W.DIFFREACT_64, nx=19, ny=19, F=(4, 200), G=(1, 4)),
    }
    out = {}
    per_batch = seeds_per_batch or n_seeds
    for name, w in systems.items():
        u0 = torch.tensor(W.initial_condition(w), dtype=torch.float64, device=dev)
        h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params)
        k_max = min(w.N, 32)
        combos, Ks, conv = [], [], []
        t_create = t_solve = 0.0
        for s0 in range(0, n_seeds, per_batch):
            problems = []
            for sd in range(s0, min(n_seeds, s0 + per_batch)):
                for M in Ms:
                    wM = w.replace(M=M)
                    A, z = W.random_weights(wM, seed=1000 + sd)
                    for m in ms:
                        combos.append((sd, m, M))
                        problems.append(dict(h=h, d=w.d, t0=w.t0, tN=w.tN, N=w.N, F=w.F, G=w.G, M=M,
                                             activation=w.act, lam=w.lam, A=A, zeta=z, m_nn=m))
            t0 = time.perf_counter()
            plan = rpr.BatchPlan(problems, tol=[w.eps] * len(problems), correction=rpr.RPR_CORR_RANDNET_NN,
                                 k_max=k_max)
            outs = [torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev) for _ in problems]
            t1 = time.perf_counter()
            plan.execute([u0] * len(problems), outs)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            Ks += [plan.instance(b).info()["K"] for b in range(len(problems))]
            conv += [plan.instance(b).info()["converged"] for b in range(len(problems))]
            plan.close()
            del outs
            t_create += t1 - t0
            t_solve += t2 - t1
            if per_batch < n_seeds:
                print(f"robustness {name}: draws {s0}..{min(n_seeds, s0 + per_batch) - 1} done "
                      f"({len(problems)} instances, solve {t2 - t1:.2f} s)", file=sys.stderr, flush=True)
        t1, t2 = t_create, t_create + t_solve
        t0 = 0.0
        by_m = {m: Counter() for m in ms}
        by_M = {M: Counter() for M in Ms}
        for (sd, m, M), K, c in zip(combos, Ks, conv):
            key = str(K) if c else f">{k_max}"
            by_m[m][key] += 1
            by_M[M][key] += 1
        Up = torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev)
        pp = rpr.Plan(h, w.d, w.t0, w.tN, w.N, F=w.F, G=w.G, tol=w.eps, correction=rpr.RPR_CORR_PARAREAL)
        pp.execute(u0, Up)
        torch.cuda.synchronize()
        K_para = pp.info()["K"]
        pp.close()
        out[name] = {"d": w.d, "N": w.N, "instances": len(combos), "weight_draws": n_seeds, "k_max": k_max,
                     "create_s": t1 - t0, "solve_s": t2 - t1, "K_classical_parareal": K_para,
                     "K_median": float(np.median(Ks)),
                     "K_by_m": {str(m): hist(c) for m, c in by_m.items()},
                     "K_by_M": {str(M): hist(c) for M, c in by_M.items()}}
        print(f"robustness {name}: {len(combos)} instances, solve {t2 - t1:.2f} s, median K "
              f"{np.median(Ks)}, classical K {K_para}", file=sys.stderr, flush=True)
    return out


def extra_workloads(torch, rpr, W, dev, only=None):
    """One FP64 and one mixed-precision solve of each of the other workloads
    with the global-fit correction, and the same with the refit on the 4
    nearest pairs: time to tolerance, fine state-steps per second and the
    accuracy of the mixed solve against the FP64 one (per slot max
    |U_mixed - U_fp64|, averaged over slots); for shallow water also the time
    to a common accuracy.  Progress goes to stderr."""
    res = {}

    def fine_rate(plan, w, sec):
        Lh, _ = plan.history()
        K = plan.info()["K"]
        return sum(w.N - int(Lh[k - 1]) for k in range(1, K + 1)) * w.F[1] / sec

    def serial_fine(w, h, u0, prec):
        """F slice after slice from u0 (the serial fine solution), as FP64."""
        dtype = torch.float64 if prec == rpr.RPR_FP64 else torch.float32
        dt = (w.tN - w.t0) / w.N / w.F[1]
        cur = u0.to(dtype)[None].contiguous()
        out = [cur[0].double().clone()]
        for _ in range(w.N):
            nxt = torch.empty_like(cur)
            rpr.rpr_propagate(h, w.d, w.F[0], w.F[1], prec, dt, 1, cur, nxt)
            cur = nxt
            out.append(cur[0].double().clone())
        torch.cuda.synchronize()
        return torch.stack(out)

    def single(w, with_tau=False):
        h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params, nz=w.nz if w.kind == rpr.RPR_BRUSS3D else 0)
        A, z = W.random_weights(w)
        u0 = torch.tensor(W.initial_condition(w), dtype=torch.float64, device=dev)
        r = {"d": w.d, "N": w.N}
        Us = {}

        def solve(prec, k_max=0, correction=rpr.RPR_CORR_RANDNET):
            plan = rpr.Plan(h, w.d, w.t0, w.tN, w.N, F=w.F, G=w.G, tol=w.eps, M=w.M, activation=w.act, lam=w.lam,
                            A=A, zeta=z, precision=prec, autotune=1, k_max=k_max, correction=correction, m_nn=4)
            U = torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.execute(u0, U)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            res = {"s": sec, "K": plan.info()["K"], "fine_state_steps_per_s": fine_rate(plan, w, sec)}
            plan.close()
            return U, res

        for name, prec in (("fp64", rpr.RPR_FP64), ("mixed", rpr.RPR_MIXED)):
            Us[name], r[name] = solve(prec)
            print(f"extra {w.name} {name}: {r[name]['s']:.3f} s, K = {r[name]['K']}", file=sys.stderr, flush=True)
        r["mixed"]["E_vs_fp64"] = float((Us["mixed"][1:] - Us["fp64"][1:]).abs().amax(dim=1).mean())
        # the paper's correction: a refit per prediction on the 4 nearest pairs
        for name, prec in (("nn_fp64", rpr.RPR_FP64), ("nn_mixed", rpr.RPR_MIXED)):
            Us[name], r[name] = solve(prec, correction=rpr.RPR_CORR_RANDNET_NN)
            print(f"extra {w.name} {name}: {r[name]['s']:.3f} s, K = {r[name]['K']}", file=sys.stderr, flush=True)
        if with_tau:
            # the common accuracy of the benchmark line: tau = 10 x the error
            # of the FP32 serial fine solution against the FP64 one
            Uf = serial_fine(w, h, u0, rpr.RPR_FP64)
            Uf32 = serial_fine(w, h, u0, rpr.RPR_MIXED)
            E = lambda U: float((U[1:] - Uf[1:]).abs().amax(dim=1).mean())
            tau = 10.0 * E(Uf32)
            tt = {"tau": tau, "fp32_serial_fine_error_floor": E(Uf32)}
            for name in ("nn_fp64", "nn_mixed"):
                r[name]["E_vs_fp64_serial_fine"] = E(Us[name])
            for name, prec in (("fp64", rpr.RPR_FP64), ("mixed", rpr.RPR_MIXED)):
                r[name]["E_vs_fp64_serial_fine"] = E(Us[name])
                tt[name] = {"k": None, "s": None, "E": None}
                for k in range(1, r[name]["K"] + 1):
                    Uk, rk = solve(prec, k_max=k)
                    if E(Uk) <= tau:
                        tt[name] = {"k": k, "s": rk["s"], "E": E(Uk)}
                        break
                print(f"extra {w.name} {name}: tau {tau:.2e} reached at k = {tt[name]['k']}", file=sys.stderr,
                      flush=True)
            tt["fp64_over_mixed"] = (tt["fp64"]["s"] / tt["mixed"]["s"]) if tt["fp64"]["s"] and tt["mixed"]["s"] \
                else None
            r["time_to_tau"] = tt
        return r

    singles = {"burgers_d128": (W.BURGERS_D128, False), "bruss_128x128": (W.BRUSS_128, False),
               "swe_192x192": (W.SWE_192, False), "bruss3d_20": (W.BRUSS3D_20, False)}
    if only is not None:
        return {only: single(*singles[only])}
    for name, (w, tau) in singles.items():
        res[name] = single(w, with_tau=tau)
    cb = copy_bandwidth(torch, dev)
    res["swe_192x192"]["F_roofline"] = {"fp64": f_roofline(torch, rpr, W.SWE_192, rpr.RPR_FP64, dev, copy_bw=cb),
                                        "fp32": f_roofline(torch, rpr, W.SWE_192, rpr.RPR_MIXED, dev, copy_bw=cb)}

    bw = W.burgers_batch()
    problems = []
    for w in bw.instances:
        A, z = W.random_weights(w)
        problems.append(dict(h=rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params), d=w.d, t0=w.t0, tN=w.tN,
                             N=w.N, F=w.F, G=w.G, M=w.M, activation=w.act, lam=w.lam, A=A, zeta=z))
    u0s = [torch.tensor(W.initial_condition(w), dtype=torch.float64, device=dev) for w in bw.instances]
    r = {"instances": len(problems), "slots": sum(w.N for w in bw.instances)}
    for name, prec, graph in (("fp64", rpr.RPR_FP64, 0), ("mixed", rpr.RPR_MIXED, 0), ("mixed_graph", rpr.RPR_MIXED, 1)):
        plan = rpr.BatchPlan(problems, tol=[w.eps for w in bw.instances], precision=prec, graph=graph,
                             autotune=1)
        outs = [torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev) for w in bw.instances]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status = plan.execute(u0s, outs)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        steps = 0
        for b, w in enumerate(bw.instances):
            inst = plan.instance(b)
            Lh, _ = inst.history()
            steps += sum(w.N - int(Lh[k - 1]) for k in range(1, inst.info()["K"] + 1)) * w.F[1]
        i0 = plan.instance(0).info()  # the batch's phase times (eager runs; -1 with graphs)
        r[name] = {"s": sec, "status": status, "fine_state_steps_per_s": steps / sec,
                   "phases_s": {"fine": i0["t_fine"], "model": i0["t_model"], "sweep": i0["t_sweep"]}}
        plan.close()
        print(f"extra burgers_batch64 {name}: {sec:.3f} s", file=sys.stderr, flush=True)
    res["burgers_batch64"] = r
    return res


if __name__ == "__main__":
    main()
