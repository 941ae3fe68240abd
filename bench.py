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
SAMPLE_EVERY = 10   # headline steps between the launches timed with events
KERNEL_SOURCES = ("paper_1905_05524_amd/csrc/step.hip", "paper_1905_05524_amd/csrc/adg_internal.h",
                  "paper_1905_05524_amd/build.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bubble81_N6.json")


def kernel_source_hash():
    """Digest of the sources the step kernels are built from; counter data
    taken on other sources no longer describe the kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE counter summary (already scaled by the copy calibration), or
    None when the summary is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash() or kernel not in d:
        return None
    return d[kernel]["traffic_bytes"]


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(O, model, w, threads, budget_s):
    """Whole oracle steps of workload w on the given number of threads until
    about budget_s seconds; returns (DOF-updates/s, steps, seconds, threads used)."""
    used = O.set_threads(threads)
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    dt = O.dt(w["phys"], w["mesh"], Q)
    t0 = time.perf_counter()
    Q, _ = O.run(w["phys"], w["mesh"], Q, 0.0, 1, dt)
    one = time.perf_counter() - t0
    steps = 1
    extra = min(max(0, int(budget_s / max(one, 1e-9)) - 1), 400)
    total = one
    if extra:
        t1 = time.perf_counter()
        O.run(w["phys"], w["mesh"], Q, dt, extra, dt)
        steps += extra
        total = one + (time.perf_counter() - t1)
    C = w["mesh"]["nx"] * w["mesh"]["nz"]
    return model.dofs(C, w["phys"]["N"]) * steps / total, steps, total, used


def _timed(fn):
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def cpu_other_workloads(O, model):
    """The oracle on the other measured workloads (bounded samples, all host
    threads): the 9x9, N=2 density wave (10 whole steps); one forward step
    with its forward-mode derivative along one direction on the 27x27 adjoint
    workload (the oracle's reference for the adjoint); one step of every
    eighth scenario of the 64-scenario batch (DOF-updates over the summed
    times)."""
    import numpy as np
    from paper_1905_05524_amd import inputs as I
    out = {}
    w = I.mms_small(N=2, nx=9)
    Q = O.ic(w["phys"], w["mesh"], "mms")
    dt = O.dt(w["phys"], w["mesh"], Q)
    sec = _timed(lambda: O.run(w["phys"], w["mesh"], Q, 0.0, 10, dt))
    out["mms9x9_N2"] = {"dof_updates_per_s": model.dofs(81, 2) * 10 / sec, "sample": f"10 steps, {sec:.3f} s"}
    w = I.bubble27()
    Q = O.ic(w["phys"], w["mesh"], "bubbles", w["bubbles"])
    dt = O.dt(w["phys"], w["mesh"], Q)
    v = np.random.default_rng(4).standard_normal(Q.shape)
    sec = _timed(lambda: O.step_jvp(w["phys"], w["mesh"], Q, v, 0.0, dt))
    out["bubble27_N6_step_and_jvp"] = {"s_per_step_and_direction": sec,
                                       "sample": f"one step with one tangent direction, {sec:.3f} s"}
    ws = I.batch_scenarios(64)
    dofs, tot = 0, 0.0
    for k in range(0, 64, 8):
        wk = ws[k]
        Qk = O.ic(wk["phys"], wk["mesh"], "bubbles", wk["bubbles"])
        dk = O.dt(wk["phys"], wk["mesh"], Qk)
        tot += _timed(lambda: O.step(wk["phys"], wk["mesh"], Qk, 0.0, dk))
        dofs += model.dofs(wk["mesh"]["nx"] * wk["mesh"]["nz"], wk["phys"]["N"])
    out["batch64_every_8th"] = {"dof_updates_per_s": dofs / tot, "sample": f"8 scenarios, one step each, {tot:.2f} s"}
    return out


def cpu_baseline(w, budget_s=15.0, one_thread_budget_s=4.0):
    """Oracle (as it stands) on the same workload: whole steps of the 81x81
    grid on all host threads until about budget_s seconds of CPU work, and a
    shorter sample on one thread."""
    from oracle import oracle as O
    from paper_1905_05524_amd import model
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    rate, steps, total, used = _oracle_rate(O, model, w, threads, budget_s)
    r1, s1, t1, _ = _oracle_rate(O, model, w, 1, one_thread_budget_s)
    O.set_threads(threads)
    others = cpu_other_workloads(O, model)
    return {"value": rate, "unit": "DOF-updates/s", "cores": used, "kind": "oracle",
            "other_workloads": others,
            "sample": f"{steps} full step(s) of the 81x81 N=6 bubble workload, {total:.1f} s, "
                      f"OpenMP threads={used}",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "one_thread": {"value": r1, "unit": "DOF-updates/s",
                           "sample": f"{s1} full step(s), {t1:.1f} s, one thread"}}


def batched_leg(steps=20, warmup=3):
    """64 independent bubble scenarios (grids 9..81, N in 3..6): one HIP-graph
    launch per step of the whole batch (autotuned launch shapes), against the
    same 64 scenarios run one after another with plain adg_step calls; and
    the same graph step with the persistent work-counter predictor."""
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
    # the persistent work-counter predictor (one resident grid per order,
    # items from a device counter), same graph step otherwise
    bp = adg.Batch(ws)
    for s_, w in enumerate(ws):
        bp.init_state(s_, "bubbles", w["bubbles"])
    bp.compute_dt()
    bp.set_mode(adg.ADG_BATCH_PERSISTENT)
    with torch.cuda.stream(st):
        for _ in range(warmup):
            bp.step_graph(st)
        e0.record(st)
        for _ in range(steps):
            bp.step_graph(st)
        e1.record(st)
    torch.cuda.synchronize()
    t_pers = e0.elapsed_time(e1) / 1e3
    del bp
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
                        "N in 3..6, walls, mu=1e-3, Courant factor 0.4, each with its own clock",
            "cells": sum(w["mesh"]["nx"] * w["mesh"]["nz"] for w in ws), "dof": dof, "steps": steps,
            "batched_graph_s_per_step": t_batch / steps, "sequential_s_per_step": t_seq / steps,
            "speedup_batched_vs_sequential": t_seq / t_batch,
            "batched_dof_updates_per_s": dof * steps / t_batch,
            "batched_fp64_frac": flops * steps / t_batch / 1e12 / FP64_PEAK_TFLOPS,
            "autotuned_cells_per_wave": cpw, "autotuned_waves_per_block": wpb,
            "persistent_graph_s_per_step": t_pers / steps,
            "persistent_fp64_frac": flops * steps / t_pers / 1e12 / FP64_PEAK_TFLOPS,
            "kept": "per-order launches (faster than the persistent work-counter predictor)"
                    if t_batch <= t_pers else "persistent"}


def amr_leg(workload="amr27", steps=200, repeats=3):
    """Adaptive workloads, timed end to end (including the host-side regrid
    plan and the device-to-host flag copy):
      amr27: 27x27 coarse cells, one 3-way level, N=6, warm and cold bubbles;
      amr9:  the paper's colliding bubbles on 9x9 coarse cells, two levels.
    Initial refinement from the analytic state; TV indicator, flags and
    regrid every 10 steps.  The run is repeated from the initial state
    `repeats` times and the median time is reported (the host part makes a
    single run noisy)."""
    import numpy as np
    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I
    w = {"amr27": I.amr27, "amr9": I.amr9}[workload]()
    N = w["phys"]["N"]

    def run():
        m = adg.Mesh(w["phys"], w["mesh"])
        m.init_state("bubbles", w["bubbles"])

        def indicator():
            tv = torch.zeros(m.C, dtype=torch.float64, device="cuda")
            fl = torch.zeros(m.C, dtype=torch.int8, device="cuda")
            st = torch.zeros(3, dtype=torch.float64, device="cuda")
            m.tv_indicator(adg.ADG_VAR_THETA, w["T_refine"], w["T_coarsen"], tv, fl, st)
            return fl

        for _ in range(w.get("initial_passes", 1)):
            m.regrid(indicator())
            m.init_state("bubbles", w["bubbles"])
        m.compute_dt()
        c0 = m.C
        torch.cuda.synchronize()
        dof_updates, cells = 0, []
        t0 = time.perf_counter()
        for k in range(steps):
            m.step()
            dof_updates += model.dofs(m.C, N)
            if (k + 1) % w["regrid_every"] == 0 and k + 1 < steps:
                m.regrid(indicator())
                cells.append(m.C)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        m.check_health()
        return m, c0, cells, dof_updates, t

    runs = [run() for _ in range(repeats)]
    ts = sorted(r[4] for r in runs)
    m, c0, cells, dof_updates, _ = runs[0]
    t = ts[len(ts) // 2]
    levels = np.bincount([int(r[0]) for r in m.leaves()], minlength=w["mesh"]["max_level"] + 1)
    names = {"amr27": "amr27x27_L1_N6: 27x27 coarse cells of 37.04 m, one 3-way level, warm cosine + cold "
                      "Gaussian bubble, regrid every 10 steps (TV of theta, T_refine 0, T_coarsen -0.4)",
             "amr9": "amr9x9_L2_N6: colliding bubbles, 9x9 coarse cells of 111.1 m, two 3-way levels "
                     "(37.04 m, 12.35 m), 3 initial refinement passes, regrid every 10 steps "
                     "(TV of theta, T_refine 2.5, T_coarsen -0.5)"}
    return {"workload": names[workload],
            "steps": steps, "initial_leaves": c0, "leaves_min": min(cells + [c0]), "leaves_max": max(cells + [c0]),
            "leaves_final": m.C, "leaves_per_level_final": levels.tolist(),
            "s_per_step_incl_regrid": t / steps, "s_per_step_runs": [x / steps for x in ts],
            "dof_updates_per_s": dof_updates / t, "sim_time_s": m.t}


def paper_grid_leg(steps=20, warmup=2):
    """The grid of the paper's performance runs (the colliding bubbles on a
    uniform 729x729 grid, N=6, 104 M DOF, 20 steps) on this one GPU: the
    same step as the headline workload, 81 times as many cells."""
    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I
    w = I.paper_grid()
    N = w["phys"]["N"]
    m = adg.Mesh(w["phys"], w["mesh"])
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        m.step(s)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for k in range(steps):
        ev[k][0].record(s)
        m.predictor(s)
        ev[k][1].record(s)
        m.corrector(s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    pred_ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    m.check_health(s)
    # the TV indicator (TV of theta per cell, statistics, flags) on this grid
    tv = torch.zeros(m.C, dtype=torch.float64, device="cuda")
    fl = torch.zeros(m.C, dtype=torch.int8, device="cuda")
    st = torch.zeros(3, dtype=torch.float64, device="cuda")
    m.tv_indicator(adg.ADG_VAR_THETA, 1.5, -0.5, tv, fl, st, s)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(s)
    for _ in range(5):
        m.tv_indicator(adg.ADG_VAR_THETA, 1.5, -0.5, tv, fl, st, s)
    t1.record(s)
    torch.cuda.synchronize()
    tv_ms = t0.elapsed_time(t1) / 5
    dof = model.dofs(m.C, N)
    pt = model.predictor_flops(N) * m.C / (pred_ms / 1e3) / 1e12
    return {"workload": "colliding729x729_N6: warm plateau and cold bubble, 729x729 cells of 1.37 m, N=6, "
                        "no-slip walls, mu=1e-3, Courant factor 0.4 (the grid of the paper's performance runs)",
            "cells": m.C, "dof": dof, "steps": steps, "ms_per_step": ms,
            "dof_updates_per_s": dof / (ms / 1e3), "predictor_ms": pred_ms, "predictor_tflops": pt,
            "predictor_fp64_frac": pt / FP64_PEAK_TFLOPS, "tv_indicator_ms": tv_ms,
            "paper_context": "the paper reports 20.2 MDOF/s on half a CPU node and 137.3 MDOF/s on five nodes "
                             "for this grid (other hardware: context, not a target)"}


def adjoint_leg(steps=50):
    """Forward + hand-written adjoint: 27x27 cells, N=6, 50 steps with a
    checkpoint every step, gradient of the final theta' L2 norm with respect
    to the initial nodal theta'.  Timed twice: keeping every step's Picard
    iterates and face data in HBM (2.8 GB) so the backward pass skips the
    predictor recompute, and recomputing them from the checkpoints."""
    import numpy as np
    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I
    from paper_1905_05524_amd.autodiff import theta_rollout
    w = I.bubble27()
    N = w["phys"]["N"]
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    dt = m.dt
    C, n = m.C, N + 1
    out = {"workload": "bubble27x27_N6 forward + adjoint, 50 steps, frozen dt, checkpoint every step", "cells": C,
           "steps": steps}
    grads = {}
    for keep in (True, False):
        th = torch.zeros((C, n, n), dtype=torch.float64, device="cuda")
        th[:, :, :] = 0.1
        th.requires_grad_(True)
        # warm-up at the timed length, so that the kept iterates' 2.8 GB come
        # from the allocator's cache in the timed run, as in any repeated use
        L = theta_rollout(th, m, steps, dt, keep=keep)
        L.backward()
        torch.cuda.synchronize()
        th.grad = None
        t0 = time.perf_counter()
        L = theta_rollout(th, m, steps, dt, keep=keep)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd, bwd = (t1 - t0) / steps, (t2 - t1) / steps
        grads[keep] = th.grad.detach().clone()
        if keep:
            # the backward pass without the recompute: the reverse sweeps only
            aflops = (model.adjoint_flops(N) - model.predictor_flops(N)) * C
            out.update({"forward_ms_per_step": fwd * 1e3, "adjoint_ms_per_step": bwd * 1e3,
                        "fwd_plus_adj_ms_per_step": (fwd + bwd) * 1e3,
                        "adjoint_fp64_frac": aflops / bwd / 1e12 / FP64_PEAK_TFLOPS,
                        "grad_norm": float(th.grad.norm())})
        else:
            aflops = model.adjoint_flops(N) * C
            out["recompute"] = {"forward_ms_per_step": fwd * 1e3, "adjoint_ms_per_step": bwd * 1e3,
                                "fwd_plus_adj_ms_per_step": (fwd + bwd) * 1e3,
                                "adjoint_fp64_frac": aflops / bwd / 1e12 / FP64_PEAK_TFLOPS}
    out["kept_equals_recompute"] = bool(torch.equal(grads[True], grads[False]))
    return out


def _l2_rho_error(m, exact_kind, T, nx, L):
    import torch
    from paper_1905_05524_amd import adg
    ex = adg.Mesh(m.phys, m.mesh_desc)
    ex.init_state(exact_kind, t0=T)
    wq = torch.as_tensor(m.basis()["w"], dtype=torch.float64, device="cuda")
    W = torch.outer(wq, wq) * (L / nx) ** 2
    return float(torch.sqrt(torch.sum(W[None] * (m.Q[:, 0] - ex.Q[:, 0]) ** 2)))


def _run_to(w, kind, T):
    import math
    from paper_1905_05524_amd import adg
    m = adg.Mesh(w["phys"], w["mesh"], fixed_dt=True)
    m.init_state(kind)
    m.compute_dt()
    ns = int(math.ceil(T / m.dt))
    m.set_state(m.Q.clone(), t=0.0, dt=T / ns)
    for _ in range(ns):
        m.step()
    return m, ns


def convergence_leg(orders=(1, 2, 3, 4, 5, 6)):
    """Convergence studies on the GPU path: the paper's manufactured solution
    (CFD scenarios: periodic [0,10]^2, mu = 0.1, to t = 0.5, L2 error of rho
    on three or four grids per order), and the advected density wave
    (periodic unit square, mu = 0.01, Courant factor 0.4, to t = 0.05, grids
    9, 18, 36), with the experimental orders between successive grids; plus
    the step throughput of the 9x9, N=2 density-wave workload."""
    import math
    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I
    out = {"paper_mms": {"workload": "the paper's manufactured solution: periodic [0,10]^2, CFD constants, "
                                     "mu = 0.1, Courant factor 0.5, L2 error of rho at t = 0.5",
                         "orders": {}},
           "density_wave": {"workload": "periodic [0,1]^2, rho = 1 + 0.1 sin 2pi x sin 2pi z, u = w = 0.5, p = 1, "
                                        "mu = 0.01, Courant factor 0.4; L2 error of rho at t = 0.05",
                            "orders": {}}}
    for N in orders:
        errs = []
        for nx in I.PAPER_MMS_GRIDS[N]:
            w = I.paper_mms(N, nx)
            m, ns = _run_to(w, "paper_mms", w["t_end"])
            errs.append({"nx": nx, "steps": ns, "l2_rho": _l2_rho_error(m, "paper_mms", w["t_end"], nx, 10.0)})
        eoc = [math.log2(errs[k]["l2_rho"] / errs[k + 1]["l2_rho"]) for k in range(len(errs) - 1)]
        out["paper_mms"]["orders"][str(N)] = {"errors": errs, "eoc": eoc}
    for N in orders:
        errs = []
        for nx in (9, 18, 36):
            w = I.mms_small(N=N, nx=nx)
            w["phys"]["cfl"] = 0.4
            m, ns = _run_to(w, "mms", 0.05)
            errs.append({"nx": nx, "steps": ns, "l2_rho": _l2_rho_error(m, "mms", 0.05, nx, 1.0)})
        eoc = [math.log2(errs[k]["l2_rho"] / errs[k + 1]["l2_rho"]) for k in range(len(errs) - 1)]
        out["density_wave"]["orders"][str(N)] = {"errors": errs, "eoc": eoc}
    # throughput of the small workload: 9x9 cells, N = 2, 10 steps
    w = I.mms_small(N=2, nx=9)
    m = adg.Mesh(w["phys"], w["mesh"])
    m.init_state("mms")
    m.compute_dt()
    s = torch.cuda.current_stream()
    for _ in range(10):
        m.step(s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(10):
        m.step(s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    # the N = 2 workload sits at the ridge of the roofline: both fractions (81
    # cells are far too few to load the chip, so both are small)
    flops = model.step_flops(2) * 81
    bytes_ = (model.predictor_bytes(2) + model.corrector_bytes(2)) * 81
    out["mms9x9_N2"] = {"ms_per_step": ms, "dof_updates_per_s": model.dofs(81, 2) / (ms / 1e3),
                        "fp64_frac": flops / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                        "hbm_frac": bytes_ / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                        "flops_per_step": flops, "bytes_per_step": bytes_}
    return out


def three_d_leg(steps=50, warmup=5, abc=True):
    """The 3D cosine bubble at the paper's resolution (the 1000 m cube on 25^3
    cells of 40 m, N = 3, mu = 0.005, no-slip walls): DOF-updates/s of the
    whole step, predictor and corrector times from HIP events on the launch
    stream, the predictor against the FP64 peak; then the ABC flow (27^3
    cells, N = 3) run to t = 0.1 with the relative L2 error of the velocity
    against the analytic field, the paper's comparison time."""
    import math
    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I
    w = I.bubble3d()
    N = w["phys"]["N"]
    m = adg.Mesh3(w["phys"], w["mesh"])
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        m.step(s)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b, c in ev:
        a.record(s)
        m.predictor(s)
        b.record(s)
        m.corrector(s)
        c.record(s)
    torch.cuda.synchronize()
    m.check_health(s)
    total_ms = ev[0][0].elapsed_time(ev[-1][2])
    pred_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    corr_ms = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    C = m.C
    pflops = model.predictor3_flops(N) * C
    out = {"workload": "bubble3d_25^3_N3: cosine warm bubble in the 1000 m cube, 25^3 cells of 40 m, N=3, "
                       "mu=0.005, no-slip walls, Courant factor 0.4",
           "cells": C, "dof": model.dofs3(C, N), "steps": steps,
           "ms_per_step": total_ms / steps,
           "dof_updates_per_s": model.dofs3(C, N) * steps / (total_ms / 1e3),
           "predictor_ms": pred_ms, "corrector_ms": corr_ms,
           "predictor_tflops": pflops / (pred_ms / 1e3) / 1e12,
           "predictor_frac_fp64_peak": pflops / (pred_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
           "corrector_GBps": model.corrector3_bytes(N) * C / (corr_ms / 1e3) / 1e9,
           "sim_time_s": m.t}
    if not abc:
        return out
    # ABC flow to t = 0.1 against the analytic velocity (qualitative in the paper)
    wa = I.abc3d()
    a = adg.Mesh3(wa["phys"], wa["mesh"], fixed_dt=True)
    a.init_state("abc")
    a.compute_dt()
    ns = int(math.ceil(wa["t_end"] / a.dt))
    a.set_state(a.Q.clone(), t=0.0, dt=wa["t_end"] / ns)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(ns):
        a.step(s)
    e1.record(s)
    torch.cuda.synchronize()
    a.check_health(s)
    ex = adg.Mesh3(wa["phys"], wa["mesh"])
    ex.init_state("abc", t0=wa["t_end"])
    torch.cuda.synchronize()
    vel = a.Q[:, 1:4] / a.Q[:, 0:1]
    err = float(torch.sqrt(torch.sum((vel - ex.Q[:, 1:4]) ** 2) / torch.sum(ex.Q[:, 1:4] ** 2)))
    out["abc"] = {"workload": "ABC flow, periodic [-pi,pi]^3, 27^3 cells, N=3, mu=0.01, to t=0.1",
                  "steps": ns, "ms_per_step": e0.elapsed_time(e1) / ns,
                  "dof_updates_per_s": model.dofs3(a.C, wa["phys"]["N"]) * ns / (e0.elapsed_time(e1) / 1e3),
                  "rel_l2_velocity_error_vs_analytic": err}
    return out


def fv_leg(steps=200, warmup=10):
    """The colliding bubbles with the MUSCL-Hancock scheme (7^2 patches of
    90^2 cells: 630x630 cells of 1.59 m, inviscid, Courant factor 0.9):
    cell updates per second of the fused step (adg_fv_step: one tile kernel
    with the face values in LDS, a copy-back kernel that also reduces the
    time-step bound, the clock), its rate against the step's minimum HBM
    traffic (the state read and written once); then the split path
    (predictor and corrector through the workspace) with its kernel times."""
    import torch
    from paper_1905_05524_amd import adg, model
    from paper_1905_05524_amd import inputs as I
    w = I.fv_bubbles()
    m = adg.FV(w["phys"], w["mesh"])
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        m.step(s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        m.step(s)
    e1.record(s)
    torch.cuda.synchronize()
    m.check_health(s)
    ms = e0.elapsed_time(e1) / steps
    C = m.C
    out = {"workload": "fv630x630: colliding bubbles, MUSCL-Hancock with van Albada, 630x630 cells of 1.59 m, "
                       "inviscid, no-slip walls, Courant factor 0.9",
           "cells": C, "steps": steps, "ms_per_step": ms,
           "cell_updates_per_s": C / (ms / 1e3), "dof_updates_per_s": 4 * C / (ms / 1e3),
           "min_traffic_bytes": model.fv_min_bytes() * C,
           "GBps_vs_min_traffic": model.fv_min_bytes() * C / (ms / 1e3) / 1e9,
           "sim_time_s": m.t}
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b, c in ev:
        a.record(s)
        m.predictor(s)
        b.record(s)
        m.corrector(s)
        c.record(s)
    torch.cuda.synchronize()
    m.check_health(s)
    p_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    c_ms = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    out["split"] = {"ms_per_step": ev[0][0].elapsed_time(ev[-1][2]) / steps, "predict_ms": p_ms,
                    "correct_ms": c_ms,
                    "predict_GBps": model.fv_predict_bytes() * C / (p_ms / 1e3) / 1e9,
                    "correct_GBps": model.fv_correct_bytes() * C / (c_ms / 1e3) / 1e9}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU reaches its sustained clock only after about 0.1 s of work: a
    # warm-up of 10 steps measured the predictor 7 % slower than one of 400
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 10 device-to-device copies of MIB MiB (counter calibration)")
    ap.add_argument("--leg", choices=["batched", "adaptive", "adaptive2", "adjoint", "convergence", "three_d", "paper_grid",
                                      "bubble3d", "fv"],
                    default=None,
                    help="only run this leg and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.leg:
        fn = {"batched": batched_leg, "adaptive": amr_leg, "adaptive2": lambda: amr_leg("amr9"),
              "paper_grid": paper_grid_leg,
              "adjoint": adjoint_leg, "convergence": convergence_leg, "three_d": three_d_leg,
              "bubble3d": lambda: three_d_leg(abc=False), "fv": fv_leg}[args.leg]
        print(json.dumps({args.leg: fn()}), flush=True)
        return
    if args.copy_calibration:
        import torch
        nb = args.copy_calibration << 20
        a = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "copies": 10}), flush=True)
        return
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
    # kernel durations from events around the launches of every SAMPLE_EVERY-th
    # step of the timed region, from the middle of the first block of steps
    # on (away from the start of the region): an event on the stream costs
    # about 3 us, so events in every step would add about 5 % to the measured
    # step time
    sampled = [k for k in range(K) if k % SAMPLE_EVERY == SAMPLE_EVERY // 2]
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
              torch.cuda.Event(enable_timing=True)) for k in sampled}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(s)
    for k in range(K):
        if k in ev:
            a, b, c = ev[k]
            a.record(s)
            m.predictor(s)
            b.record(s)
            m.corrector(s)
            c.record(s)
        else:
            m.predictor(s)
            m.corrector(s)
        if k % TV_EVERY == TV_EVERY - 1:
            m.tv_indicator(adg.ADG_VAR_THETA, 1.5, -0.5, tv, fl, st, s)
    stop.record(s)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    pred_ms = sum(a.elapsed_time(b) for a, b, _ in ev.values()) / len(ev)
    corr_ms = sum(b.elapsed_time(c) for _, b, c in ev.values()) / len(ev)
    m.check_health(s)
    # the TV indicator alone (HBM-bound read of Q, theta per node): 10 calls
    t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0e.record(s)
    for _ in range(10):
        m.tv_indicator(adg.ADG_VAR_THETA, 1.5, -0.5, tv, fl, st, s)
    t1e.record(s)
    torch.cuda.synchronize()
    tv_ms = t0e.elapsed_time(t1e) / 10
    tv_bytes = C * (4 * (N + 1) ** 2 * 8 + 8 + 1)

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
                               "no-slip walls, mu=1e-3, Courant factor 0.4; TV indicator every 10 steps",
                   "cells": C, "order": N, "dof": dof, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(f"k_predictor<{N + 1}"),
                     "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
                     "kernel": f"k_predictor<{N + 1}>", "kernel_ms": pred_ms, "kernel_launches_timed": len(ev),
                     "flops_per_launch": pflops},
        "extra": {"corrector_ms": corr_ms,
                  "corrector_GBps": cbytes / (corr_ms / 1e3) / 1e9,
                  "tv_indicator_ms": tv_ms, "tv_indicator_GBps": tv_bytes / (tv_ms / 1e3) / 1e9,
                  "wall_s_timed_region": t_wall,
                  "sim_time_s": m.t, "dt_s": m.dt},
    }
    if not args.no_batch:
        out["extra"]["peaks"] = adg.measure_peaks(copy_mib=1024)
        out["extra"]["peaks"]["predictor_frac_of_measured_fp64"] = achieved / out["extra"]["peaks"]["fp64_vector_tflops"]
        out["extra"]["batched"] = batched_leg()
        out["extra"]["adaptive"] = amr_leg("amr27")
        out["extra"]["adaptive_two_levels"] = amr_leg("amr9")
        out["extra"]["adjoint"] = adjoint_leg()
        out["extra"]["convergence"] = convergence_leg()
        out["extra"]["three_d"] = three_d_leg()
        out["extra"]["finite_volume"] = fv_leg()
        out["extra"]["paper_grid"] = paper_grid_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
