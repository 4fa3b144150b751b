"""Benchmark: RandNet-Parareal on one MI355X.

One step = one complete RandNet-Parareal solve (coarse sweep, then iterations
of: fine solves of every unfinished slot, training pairs, random features,
Gram/readout statistics, Cholesky ridge solve, predictor-corrector chain and
stopping rule, until every slot is final) of the 64 x 64 FitzHugh-Nagumo
diffusion-reaction workload: d = 8192, N = 64 slices on t in [0, 20], F = RK4
with 4000 steps per slice, G = RK1 with 10 steps, 200 ReLU neurons,
lambda = eps = 1e-6, plain FP64.  Inputs are seeded synthetic data already in
device memory when the timed region starts.

value = fine state-steps per second of the whole solve: the number of
(slot, fine RK4 step) pairs the run performs, sum over iterations of the
unfinished slots times 4000, divided by the wall time of the solve.

Also reported: the roofline of the dominant kernel (the fine propagator,
timed live with HIP events on its launch stream), the same solve in mixed
precision (FP32 states) with its accuracy, and the CPU oracle timed on the
host cores on the same workload.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK = 78.6e12  # MI355X FP64 vector FLOP/s (AMD specification)
# Algorithmic FP64 operations per degree of freedom and classical RK4 step of
# the diffusion-reaction stencil, counted from the formulas (a fused
# multiply-add counts as two): per cell and stage, two 5-point Laplacians
# 2 x 9, the u reaction 7, the v reaction 3, the stage updates 2 x 3.25 on
# average over the four stages = 34.5 per cell-stage = 17.25 per DOF-stage.
FLOPS_PER_DOF_STEP = {"diffreact": 4 * 17.25}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2411_06225_amd as rpr
    from paper_2411_06225_amd import workloads as W

    w = W.DIFFREACT_64
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params)
    u0h = W.initial_condition(w)
    A, zeta = W.random_weights(w)
    u0 = torch.tensor(u0h, dtype=torch.float64, device=dev)
    T = (w.tN - w.t0) / w.N

    def make_plan(prec):
        return rpr.Plan(h, w.d, w.t0, w.tN, w.N, F=w.F, G=w.G, tol=w.eps, M=w.M, activation=w.act, lam=w.lam,
                        A=A, zeta=zeta, precision=prec, correction=rpr.RPR_CORR_RANDNET, autotune=1)

    def timed_solves(plan, steps, warmup):
        U = torch.empty((w.N + 1, w.d), dtype=torch.float64, device=dev)
        for _ in range(warmup):
            plan.execute(u0, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.execute(u0, U)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / max(steps, 1), U

    plan = make_plan(rpr.RPR_FP64)
    sec, U = timed_solves(plan, args.steps, args.warmup)
    info = plan.info()
    Lh, _ = plan.history()
    K = info["K"]
    active = [w.N - int(Lh[k - 1]) for k in range(1, K + 1)]
    state_steps = sum(active) * w.F[1]
    value = state_steps / sec

    # serial fine reference on the GPU (same F kernel, slot after slot) for the accuracy E
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

    Uf = serial_fine(torch.float64, rpr.RPR_FP64)
    E = float((U[1:] - Uf[1:]).abs().amax(dim=1).mean())

    # roofline of the dominant kernel: the fine propagator over all N slots
    # (the first iteration's launch), HIP events on the stream it runs on
    X = U[:-1].contiguous()
    Y = torch.empty_like(X)
    stream = torch.cuda.current_stream()
    reps = 3
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rpr.rpr_propagate(h, w.d, w.F[0], w.F[1], rpr.RPR_FP64, T / w.F[1], w.N, X, Y, stream)
    ev[0].record(stream)
    for _ in range(reps):
        rpr.rpr_propagate(h, w.d, w.F[0], w.F[1], rpr.RPR_FP64, T / w.F[1], w.N, X, Y, stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    f_sec = ev[0].elapsed_time(ev[1]) / 1e3 / reps
    f_flops = w.N * w.F[1] * w.d * FLOPS_PER_DOF_STEP["diffreact"]
    achieved = f_flops / f_sec
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK, "traffic": None,
                "kernel": "k_prop_onchip (fine RK4, diffusion-reaction 64x64, FP64)",
                "launch": {"slots": w.N, "steps": w.F[1], "flops_per_dof_step": FLOPS_PER_DOF_STEP["diffreact"],
                           "ms": f_sec * 1e3, "active_cu_fraction": w.N / 256}}

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "d": w.d, "N": w.N, "t": [w.t0, w.tN], "F": f"RK4x{w.F[1]}",
                   "G": f"RK1x{w.G[1]}", "M": w.M, "activation": "relu", "lambda": w.lam, "eps": w.eps,
                   "precision": "fp64"},
        "time_to_tolerance_s": sec,
        "K": K,
        "L_hist": [int(v) for v in Lh],
        "E_vs_serial_fine": E,
        "dof_steps_per_s": value * w.d,
        "roofline": roofline,
    }

    if not args.no_mixed:
        mplan = make_plan(rpr.RPR_MIXED)
        msec, Um = timed_solves(mplan, args.steps, 1)
        minfo = mplan.info()
        Em = float((Um[1:] - Uf[1:]).abs().amax(dim=1).mean())
        Uf32 = serial_fine(torch.float32, rpr.RPR_MIXED)
        E32floor = float((Uf32[1:] - Uf[1:]).abs().amax(dim=1).mean())
        out["mixed"] = {"ms_per_solve": msec * 1e3, "K": minfo["K"], "E_vs_fp64_serial_fine": Em,
                        "fp32_serial_fine_error_floor": E32floor, "fp64_over_mixed_time": sec / msec}
        mplan.close()
    plan.close()

    if not args.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        pb = oracle.problem(w.kind, w.nx, w.ny, w.domain, w.params)
        net = oracle.Net(A, zeta, w.act, w.lam, 0.0)
        t0 = time.perf_counter()
        _, oi = oracle.parareal(pb, u0h, N=w.N, t0=w.t0, tN=w.tN, F=w.F, G=w.G, eps=w.eps, net=net, nthreads=threads)
        csec = time.perf_counter() - t0
        o_active = [w.N - int(oi["L_hist"][k - 1]) for k in range(1, oi["K"] + 1)]
        out["cpu_baseline"] = {"value": sum(o_active) * w.F[1] / csec, "unit": "fine state-steps/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"the full solve of the same workload by the FP64 C oracle "
                                         f"(K={oi['K']}, {sum(o_active)} fine slot solves), fine solves on "
                                         f"{threads} threads, {csec:.1f} s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
