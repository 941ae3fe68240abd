#!/usr/bin/env python3
"""Benchmark: DOF-updates/s of the ADER-DG step on one MI355X.

Workload: the 2D cosine warm bubble on 81x81 cells of 12.35 m, order N=6,
no-slip walls, FP64 (6561 cells, 1,285,956 DOF).  One timed step is the whole
hot path: predictor, boundary and face fluxes, corrector, CFL time step, and
the TV refinement indicator with its statistics and flags every 10th step
(the regrid cadence of the adaptive workload).  Inputs are resident in HBM
before timing starts.  The predictor's average duration is measured with HIP
events on the launch stream inside the timed region and priced against the
FP64 vector peak.  The CPU oracle is timed on a bounded sample of the same
workload on the host cores.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # 256 CU * 4 SIMD * 16 lanes * 2 flop * 2.4 GHz
HBM_PEAK_GBS = 8000.0
TV_EVERY = 10


def cpu_baseline(w, budget_s=15.0):
    """Oracle (as it stands) on the same workload: whole steps of the 81x81
    grid on all host threads until about budget_s seconds of CPU work."""
    from oracle import oracle as O
    from paper_1905_05524_amd import model
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    used = O.set_threads(threads)
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    dt = O.dt(w["phys"], w["mesh"], Q)
    t0 = time.perf_counter()
    Q, _ = O.run(w["phys"], w["mesh"], Q, 0.0, 1, dt)
    one = time.perf_counter() - t0
    steps = 1
    extra = max(0, int(budget_s / max(one, 1e-9)) - 1)
    extra = min(extra, 400)
    if extra:
        t1 = time.perf_counter()
        O.run(w["phys"], w["mesh"], Q, dt, extra, dt)
        steps += extra
        total = one + (time.perf_counter() - t1)
    else:
        total = one
    C = w["mesh"]["nx"] * w["mesh"]["nz"]
    rate = model.dofs(C, w["phys"]["N"]) * steps / total
    return {"value": rate, "unit": "DOF-updates/s", "cores": used, "kind": "oracle",
            "sample": f"{steps} full step(s) of the 81x81 N=6 bubble workload, {total:.1f} s, "
                      f"OpenMP threads={used}"}


def batched_leg(steps=20, warmup=3):
    """64 independent bubble scenarios (grids 9..81, N in 3..6): one HIP-graph
    launch per step of the whole batch (autotuned launch shapes), against the
    same 64 scenarios run one after another with plain adg_step calls."""
    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I
    ws = I.batch_scenarios(64)
    b = adg.Batch(ws)
    for s_, w in enumerate(ws):
        b.init_state(s_, "bubbles", w["bubbles"])
    b.compute_dt()
    torch.cuda.synchronize()
    cpw, wpb = b.autotune(reps=3)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        for _ in range(warmup):
            b.step_graph(st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(st):
        e0.record(st)
        for _ in range(steps):
            b.step_graph(st)
        e1.record(st)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3
    # sequential plain runs, same kernels, default launch shape
    meshes = []
    for w in ws:
        m = adg.Mesh(w["phys"], w["mesh"])
        m.init_state("bubbles", w["bubbles"])
        m.compute_dt()
        meshes.append(m)
    torch.cuda.synchronize()
    s0 = torch.cuda.current_stream()
    for m in meshes:
        for _ in range(warmup):
            m.step(s0)
    torch.cuda.synchronize()
    e0.record(s0)
    for m in meshes:
        for _ in range(steps):
            m.step(s0)
    e1.record(s0)
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) / 1e3
    dof = sum(model.dofs(w["mesh"]["nx"] * w["mesh"]["nz"], w["phys"]["N"]) for w in ws)
    flops = sum(model.step_flops(w["phys"]["N"]) * w["mesh"]["nx"] * w["mesh"]["nz"] for w in ws)
    return {"workload": "batch64: 64 cosine-bubble scenarios from seed 190505524, k x k grids k in 9..81, "
                        "N in 3..6, walls, mu=1e-3, CFL 0.5 each with its own clock",
            "cells": sum(w["mesh"]["nx"] * w["mesh"]["nz"] for w in ws), "dof": dof, "steps": steps,
            "batched_graph_s_per_step": t_batch / steps, "sequential_s_per_step": t_seq / steps,
            "speedup_batched_vs_sequential": t_seq / t_batch,
            "batched_dof_updates_per_s": dof * steps / t_batch,
            "batched_fp64_frac": flops * steps / t_batch / 1e12 / FP64_PEAK_TFLOPS,
            "autotuned_cells_per_wave": cpw, "autotuned_waves_per_block": wpb}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the data-parallel path shards by domain decomposition, not measured here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I

    w = I.bubble81()
    N = w["phys"]["N"]
    m = adg.Mesh(w["phys"], w["mesh"])
    C = m.C
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    tv = torch.zeros(C, dtype=torch.float64, device="cuda")
    fl = torch.zeros(C, dtype=torch.int8, device="cuda")
    st = torch.zeros(3, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()

    def one_step(k):
        m.step(s)
        if k % TV_EVERY == TV_EVERY - 1:
            m.tv_indicator(adg.ADG_VAR_THETA, 1.5, -0.5, tv, fl, st, s)

    for k in range(args.warmup):
        one_step(k)
    torch.cuda.synchronize()

    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(s)
    for k in range(K):
        a, b, c = ev[k]
        a.record(s)
        m.predictor(s)
        b.record(s)
        m.corrector(s)
        c.record(s)
        if k % TV_EVERY == TV_EVERY - 1:
            m.tv_indicator(adg.ADG_VAR_THETA, 1.5, -0.5, tv, fl, st, s)
    stop.record(s)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    pred_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / K
    corr_ms = sum(b.elapsed_time(c) for _, b, c in ev) / K
    m.check_health(s)

    dof = model.dofs(C, N)
    ms_step = total_ms / K
    value = dof * K / (total_ms / 1e3)
    pflops = model.predictor_flops(N) * C
    achieved = pflops / (pred_ms / 1e3) / 1e12
    cbytes = model.corrector_bytes(N) * C
    out = {
        "metric": "DOF-updates/s per ADER-DG step, order 6 2D NS",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bubble81x81_N6: cosine warm bubble, 81x81 cells of 12.35 m, N=6, "
                               "no-slip walls, mu=1e-3, CFL 0.5; TV indicator every 10 steps",
                   "cells": C, "order": N, "dof": dof, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": f"k_predictor<{N + 1}>", "kernel_ms": pred_ms,
                     "flops_per_launch": pflops},
        "extra": {"corrector_ms": corr_ms,
                  "corrector_GBps": cbytes / (corr_ms / 1e3) / 1e9,
                  "wall_s_timed_region": t_wall,
                  "sim_time_s": m.t, "dt_s": m.dt},
    }
    if not args.no_batch:
        out["extra"]["batched"] = batched_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
