#!/usr/bin/env python3
"""Throughput of the ENO-AO hot path on one MI355X.

Default workload: 2D Euler, 2048 x 2048 nodes, periodic, four seeded quadrant
states (rho, p ~ LogUniform[0.1, 10], u, v ~ U[-2, 2], generator seed
workloads.QUADRANT_BENCH_SEED), fifth-order ENO-AO with
Roe characteristic decomposition, SSP-RK3 with the device-side CFL step
(CFL 0.3); K timed steps after W warm-up steps, inputs resident in HBM.

Prints one JSON line: cell-updates/s of the whole job, the roofline of the
dominant kernel (HIP events on the stream the kernels run on) on the
algorithmic bytes of its Runge-Kutta stage (64/96/96 B per cell in 2D), the
step-level rooflines (256 B per cell-update against HBM, executed FP64 flops
from the committed counters against the FP64 peak), and the CPU oracle timed on
a bounded sample of the same workload on the host's cores.  Extra legs: the
smooth advection workload's latency (N = 200, 400 steps), the 1D Euler
workload (N = 2000 to t = 0.2), the batched and served workloads against their
plain per-solve launches, order 7, and the paper's discontinuous workloads.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "cell-updates/s + % HBM/FP64 roofline; batched vs plain; p50/p99 latency"
# y-sweep strip width the library takes by default for each order (the same
# launch as enoao_plan_set_tiles with 0)
DEFAULT_STRIP_COLUMNS = {5: 8, 7: 4}


def kernel_symbol(kind, order, y_strip_columns):
    """Kernel symbol as rocprofv3 prints it for a profile kind ("sweep_x_s2", ...) of a
    2D plan without selection record."""
    stage = int(kind[-1])
    if kind.startswith("sweep_x"):
        return f"enoao::sweep_x<2, {order}, {stage}, false, true>"
    return f"enoao::sweep_y<{order}, {stage}, false, {y_strip_columns}, true>"


def kernel_sources_hash():
    from paper_2108_12742_amd.counters import kernel_sources_hash as h
    return h()


def timed_solve(E, plan, u, u0, K, Wu, cfl=0.3):
    """K CFL steps of a plan from u0, timed twice.  The first pass is the value: the
    library's own path (one graph replay of K steps; the library captures that graph
    on its first replay of that length, so an untimed run of the same K steps comes
    first, after the Wu warm-up steps).  The second pass runs the same
    K steps with a HIP event pair around every launch, on the stream the kernels run
    on, for the per-kernel durations; the events cost a few microseconds per launch,
    which is why that pass is not the value.  Returns (seconds, instrumented seconds,
    per-kernel (mean ms, launches))."""
    import torch
    if Wu > 0:
        E.enoao_solve(plan, u, 1e30, cfl=cfl, max_steps=Wu)
    u.copy_(u0)
    E.enoao_solve(plan, u, 1e30, cfl=cfl, max_steps=K)
    u.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, steps = E.enoao_solve(plan, u, 1e30, cfl=cfl, max_steps=K)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert steps == K, (steps, K)
    E.enoao_plan_check(plan)
    u.copy_(u0)
    torch.cuda.synchronize()
    E.enoao_profile(plan, True)
    t0 = time.perf_counter()
    _, steps = E.enoao_solve(plan, u, 1e30, cfl=cfl, max_steps=K)
    torch.cuda.synchronize()
    el_inst = time.perf_counter() - t0
    prof = E.enoao_profile_read(plan)
    E.enoao_profile(plan, False)
    assert steps == K, (steps, K)
    E.enoao_plan_check(plan)
    return el, el_inst, prof


def _counters(workload):
    """The committed rocprofv3 counters of a workload (profiles/counters.json), or {}
    when the kernels changed since they were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "counters.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return {}
    if t.get("source_hash") != kernel_sources_hash():
        return {}
    return t.get("workloads", {}).get(workload, {})


def measured_traffic(symbol, workload):
    """HBM bytes per launch of `symbol` (FETCH_SIZE + WRITE_SIZE, scaled by a copy of
    known size), or None when the kernels changed since the counters were taken."""
    v = _counters(workload).get("bytes_per_launch", {}).get(symbol)
    return None if v is None else round(v)


def measured_fp64_flops(symbol, workload):
    """Executed FP64 flops per launch of `symbol` (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes),
    or None."""
    v = _counters(workload).get("fp64_flops_per_launch", {}).get(symbol)
    return None if v is None else float(v)


def kernel_roofline(R, equation, kind, stage, cells, ms, symbol, workload, order):
    """Roofline of one kernel kind: against HBM on the algorithmic bytes of its stage
    when it completes a stage, else against the FP64 peak on the essential flops of
    its faces; with the measured traffic (and its ratio to the algorithmic bytes)
    and the executed FP64 rate where the committed counters cover the kernel."""
    kern = kind[6] if kind.startswith("sweep") else "s"
    nbytes = cells * R.algorithmic_bytes(equation, kern, stage)
    if nbytes > 0:
        e = R.hbm_entry(nbytes, ms * 1e-3, measured_traffic(symbol, workload))
        e["algorithmic_bytes_per_cell"] = R.algorithmic_bytes(equation, kern, stage)
        if e["traffic"] is not None:
            e["traffic_ratio"] = round(e["traffic"] / nbytes, 3)
    else:
        e = R.alu_entry(cells * R.sweep_flops(equation, order, kern, stage), ms * 1e-3)
        e["flops"] = "essential (top form) flops per face"
    hw = measured_fp64_flops(symbol, workload)
    if hw is not None:
        e["fp64_executed_tflops"] = round(hw / (ms * 1e-3) / 1e12, 3)
        e["fp64_executed_frac"] = round(hw / (ms * 1e-3) / 1e12 / R.PEAK_FP64_TFLOPS, 4)
    e["kernel"] = symbol
    return e


def host_cpu():
    """(logical CPUs, CPU model string) of this host"""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(n_sample=2048, max_threads=16):
    """The oracle (plain C, FP64, single-threaded calls, unchanged) on a bounded sample
    of the workload, on the host's cores: one thread per core (at most max_threads,
    the host share of one GPU) each runs the first SSP-RK3 step of its own copy of
    the seeded quadrant problem at full size; the oracle's calls release the Python
    interpreter lock, so the threads run in parallel.  value = threads x cells / wall."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_2108_12742_amd import workloads as W
    nproc, model = host_cpu()
    threads = max(1, min(max_threads, nproc))
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, n_sample)
    p = O.Problem(O.EULER2D, nx=n_sample, ny=n_sample, order=5)

    def one(_):
        t0 = time.perf_counter()
        O.step(p, inst.u0, O.cfl_dt(p, inst.u0, 0.3))
        return time.perf_counter() - t0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        per = list(ex.map(one, range(threads)))
    el = time.perf_counter() - t0
    cells = n_sample * n_sample
    return {"value": threads * cells / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} concurrent copies of the first SSP-RK3 step of the 2D Euler quadrant workload "
                      f"(seed {W.QUADRANT_BENCH_SEED}) at {n_sample}x{n_sample}, one per thread, {el:.1f} s wall",
            "per_thread_value": cells / (sum(per) / len(per)), "nproc": nproc, "cpu_model": model}


def kernel_table(R, prof, cells, order, y_strip_columns, workload, equation="euler2d"):
    """Per kernel kind: mean duration, launches, symbol and roofline; and the kind with
    the largest total time (the dominant kernel)."""
    kernels, best = {}, None
    for kind, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        entry = {"mean_ms": round(ms, 4), "launches": cnt}
        if kind.startswith("sweep"):
            stage = int(kind[-1])
            entry["symbol"] = kernel_symbol(kind, order, y_strip_columns)
            entry["roofline"] = kernel_roofline(R, equation, kind, stage, cells, ms, entry["symbol"], workload, order)
            if best is None or ms * cnt > best[1]:
                best = (kind, ms * cnt)
        kernels[kind] = entry
    return kernels, best[0]


def step_roofline(R, equation, value, kernels, cells, steps, workload):
    """Whole-step rooflines: algorithmic bytes per cell-update x cell-updates/s against
    HBM; the executed FP64 flops of the sweeps (committed counters) per step time
    against the FP64 peak; measured traffic per cell-update against the algorithmic
    bytes."""
    bpc = R.cell_update_bytes(equation)
    gbs = bpc * value / 1e9
    out = {"bytes_per_cell_update": bpc, "achieved_gbs": round(gbs, 1), "frac_hbm": round(gbs / R.PEAK_HBM_GBS, 4)}
    sweeps = [e for k, e in kernels.items() if k.startswith("sweep")]
    hw = [measured_fp64_flops(e["symbol"], workload) for e in sweeps]
    tr = [measured_traffic(e["symbol"], workload) for e in sweeps]
    if sweeps and all(v is not None for v in hw):
        fl = sum(v * e["launches"] for v, e in zip(hw, sweeps)) / steps  # per step
        out["fp64_flops_per_cell_update"] = round(fl / cells, 1)
        tf = fl / cells * value / 1e12
        out["fp64_executed_tflops"] = round(tf, 3)
        out["frac_fp64"] = round(tf / R.PEAK_FP64_TFLOPS, 4)
    if sweeps and all(v is not None for v in tr):
        b = sum(v * e["launches"] for v, e in zip(tr, sweeps)) / steps / cells
        out["traffic_bytes_per_cell_update"] = round(b, 1)
        out["traffic_ratio"] = round(b / bpc, 3)
    return out


def bench_c0(solves=20, seed=0):
    """The smooth advection workload (N = 200, periodic, fifth order, CFL 0.5, t = 2:
    400 steps) as one plain solve: latency per whole solve (enoao_solve, state resident
    on the device; the call runs its steps in one LDS-resident launch and synchronises
    at its end), median and best of `solves` after a warm-up."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import workloads as W
    inst = W.advection(seed, 200)
    plan = E.enoao_plan_create(E.problem_from_instance(inst))
    u0 = torch.from_numpy(inst.u0).cuda()
    u = u0.clone()
    E.enoao_solve(plan, u, 2.0, cfl=0.5)  # warm-up
    lat = []
    for _ in range(solves):
        u.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t, n = E.enoao_solve(plan, u, 2.0, cfl=0.5)
        lat.append(time.perf_counter() - t0)
        assert (t, n) == (2.0, 400)
    lat = np.array(lat)
    err = float(np.abs(u.cpu().numpy() - inst.u0).max())
    return {"workload": "advection-200-ao5-cfl0.5-t2", "steps": 400, "solves": solves,
            "latency_ms_p50": float(np.median(lat) * 1e3), "latency_ms_min": float(lat.min() * 1e3),
            "us_per_step_p50": float(np.median(lat) * 1e6 / 400),
            "cell_updates_per_s": 200 * 400 / float(np.median(lat)), "max_error_after_one_period": err}


def bench_c1(seeds=(0, 1, 2, 3), repeats=3, streaming=True):
    """The 1D Euler workload: N = 2000, seeded Riemann data with the density
    perturbation, transmissive ends, CFL 0.3, to t = 0.2, one plain solve per seed;
    best of `repeats`.  N = 2000 is above the LDS-resident solver's limit, so the
    cooperative solver runs (one cooperative launch of up to 1024 controlled steps per
    enoao_solve call); with streaming=True the same solves on the streaming kernels
    (device-side CFL loop over captured graphs of 64 steps) are timed beside it."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import workloads as W

    def leg():
        runs = []
        for seed in seeds:
            inst = W.riemann_1d(seed, 2000)
            plan = E.enoao_plan_create(E.problem_from_instance(inst))
            u0 = torch.from_numpy(inst.u0).cuda()
            u = u0.clone()
            E.enoao_solve(plan, u, 0.2, cfl=0.3)  # warm-up (graph capture)
            best = None
            for _ in range(repeats):
                u.copy_(u0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t, n = E.enoao_solve(plan, u, 0.2, cfl=0.3)
                el = time.perf_counter() - t0
                best = el if best is None else min(best, el)
            runs.append({"seed": seed, "steps": n, "t_final": t, "seconds": best, "us_per_step": best * 1e6 / n,
                         "cell_updates_per_s": 2000 * n / best})
        return runs, sum(r["steps"] for r in runs) * 2000 / sum(r["seconds"] for r in runs)

    runs, rate = leg()
    out = {"workload": "euler1d-riemann-2000-ao5-cfl0.3-t0.2", "solver": "cooperative", "runs": runs,
           "cell_updates_per_s": rate}
    if streaming:
        E.enoao_set_coop(False)
        try:
            sruns, srate = leg()
        finally:
            E.enoao_set_coop(True)
        out["streaming"] = {"cell_updates_per_s": srate, "us_per_step": [round(r["us_per_step"], 2) for r in sruns]}
    return out


def bench_batched(steps=100, warmup=2, count=512, tune=True, plain=True, wg=0):
    """Batched workload: `count` 1D Euler Riemann instances, N ~ LogUniform[128, 16384],
    `steps` CFL steps each (own dt per member), in one persistent launch per stage
    (graph-captured), against the same solves launched one plan at a time (skipped
    with plain=False; tune=False keeps the default launch shape)."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import roofline as R
    from paper_2108_12742_amd import tune as T
    from paper_2108_12742_amd import workloads as W
    insts = W.batch_1d(0, count)
    probs = [E.problem_from_instance(i) for i in insts]
    u0 = [torch.from_numpy(i.u0).cuda() for i in insts]
    states = [u.clone() for u in u0]
    (best, yw), timing = T.tune_batch(probs, states, steps=3) if tune else ((wg, 8), {})
    kinds, kinds_info = T.tune_kinds(probs, states, best, yw) if tune else (None, None)
    batch = E.enoao_batch_create(probs)
    E.enoao_batch_set_launch(batch, best)
    if kinds:
        E.enoao_batch_set_launch_kinds(batch, kinds)

    def restart():
        E.enoao_batch_reset(batch)
        for u, v in zip(states, u0):
            u.copy_(v)
        torch.cuda.synchronize()

    E.enoao_batch_step(batch, states, warmup, 0.3)
    # the graph of `steps` steps is captured on its first replay: an untimed run
    restart()
    E.enoao_batch_step(batch, states, steps, 0.3)
    restart()
    t0 = time.perf_counter()
    E.enoao_batch_step(batch, states, steps, 0.3)
    _, nst, status = E.enoao_batch_query(batch)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the same steps with a HIP event pair around every launch: per-kernel durations
    restart()
    E.enoao_batch_profile(batch, True)
    t0 = time.perf_counter()
    E.enoao_batch_step(batch, states, steps, 0.3)
    _, nst2, status2 = E.enoao_batch_query(batch)
    torch.cuda.synchronize()
    el_inst = time.perf_counter() - t0
    prof = E.enoao_batch_profile_read(batch)
    E.enoao_batch_profile(batch, False)
    assert (nst == steps).all() and (nst2 == steps).all()
    cells = sum(int(p.nx) for p in probs)
    workload = f"euler1d-riemann-batch{count}-{cells}cells-ao5"
    ms, kind = max(((prof[k][0], k) for k in ("sweep_x_s1", "sweep_x_s2", "sweep_x_s3")), key=lambda x: x[0])
    stage = int(kind[-1])
    roof = kernel_roofline(R, "euler1d", kind, stage, cells, ms, f"enoao::sweep_x<1, 5, {stage}, false, true>",
                           workload, 5)
    value = cells * steps / el
    out = {"workload": workload, "members": count, "cells": cells, "steps": steps,
           "value": value, "unit": "cell-updates/s", "ms_per_step": el * 1e3 / steps,
           "instrumented_ms_per_step": round(el_inst * 1e3 / steps, 4),
           "members_ok": int((status == 0).sum()), "workgroups_per_cu": best,
           "workgroups_per_cu_by_kernel": list(kinds) if kinds else None,
           "tuner_ms_per_step": {str(k): round(v, 4) for k, v in timing.items()}, "tuner_by_kernel": kinds_info,
           "roofline": roof,
           "step_roofline_hbm": round(R.cell_update_bytes("euler1d") * value / 1e9 / R.PEAK_HBM_GBS, 4)}
    if not plain:
        return out
    # plain: one plan per instance, each solve a call of its own (a solve synchronises
    # its stream at the end), one after another on one stream (spread over 8 streams:
    # plain_8streams, in a process of its own)
    plans = [E.enoao_plan_create(p) for p in probs]
    plain = [u.clone() for u in u0]
    # graph capture and first touch, untimed, for both solvers of a lone 1D member
    # (the streaming graphs are captured on first use)
    for coop in (False, True):
        E.enoao_set_coop(coop)
        for pl, u, v in zip(plans, plain, u0):
            E.enoao_solve(pl, u, 1e300, cfl=0.3, max_steps=steps)
            u.copy_(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, u in zip(plans, plain):
        E.enoao_solve(pl, u, 1e300, cfl=0.3, max_steps=steps)
    torch.cuda.synchronize()
    el_plain = time.perf_counter() - t0
    identical = all(torch.equal(a, b) for a, b in zip(states, plain))
    out.update({"plain_value": cells * steps / el_plain, "speedup_vs_plain": el_plain / el,
                "identical_to_plain": identical})
    return out


def plain_8streams(steps=100, count=512, sets=4):
    """The plain baseline of the batched workload spread over 8 streams driven by 8
    host threads, so that solves overlap on the device.  Lone-member plans that
    would take the cooperative solver run faster here on the streaming kernels
    (cooperative launches do not overlap one another), so both are timed.  The rate
    depends on how HIP has spread the streams over its few hardware queues, so the
    streaming solves are timed on `sets` sets of 8 streams (torch's pool holds 32
    per device) and the fastest counts.  Returns cell-updates/s per solver, the
    streaming rate of each set, and whether all results are identical."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import workloads as W
    insts = W.batch_1d(0, count)
    probs = [E.problem_from_instance(i) for i in insts]
    u0 = [torch.from_numpy(i.u0).cuda() for i in insts]
    cells = sum(int(p.nx) for p in probs)
    plans = [E.enoao_plan_create(p) for p in probs]
    plain = [u.clone() for u in u0]
    for coop in (False, True):  # graph capture and first touch, untimed, for both solvers
        E.enoao_set_coop(coop)
        for pl, u, v in zip(plans, plain, u0):
            E.enoao_solve(pl, u, 1e300, cfl=0.3, max_steps=steps)
            u.copy_(v)
    E.enoao_set_coop(True)
    nstreams = 8
    stream_sets = [[torch.cuda.Stream() for _ in range(nstreams)] for _ in range(sets)]

    def timed(coop, streams):
        def lane(k):
            for i in range(k, len(plans), nstreams):
                E.enoao_solve(plans[i], plain[i], 1e300, cfl=0.3, max_steps=steps, stream=streams[k])

        E.enoao_set_coop(coop)
        try:
            for u, v in zip(plain, u0):
                u.copy_(v)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with ThreadPoolExecutor(nstreams) as ex:
                list(ex.map(lane, range(nstreams)))
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        finally:
            E.enoao_set_coop(True)
        return cells * steps / el, [u.clone() for u in plain]

    coop_rate, first = timed(True, stream_sets[0])
    by_set, same = [], True
    for streams in stream_sets:
        rate, res = timed(False, streams)
        by_set.append(rate)
        same = same and all(torch.equal(a, b) for a, b in zip(first, res))
    return {"values": {"cooperative": coop_rate, "streaming": max(by_set)}, "streaming_by_stream_set": by_set,
            "identical": same}


def run_plain_8streams(steps=100):
    """The 8-stream plain baseline in a child process of its own, started before
    this process touches the GPU.  How HIP spreads torch's pool of streams over its
    few hardware queues depends on the streams a process made before (late in the
    benchmark's process the same solves measured 2.3e8 cell-updates/s against 6.2e8
    in a process of their own); and beside a process that has made cooperative
    launches, the runtime turns a second process's cooperative launches down."""
    import subprocess
    r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--only-leg", "plain8", "--steps", str(steps)],
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"8-stream plain baseline failed (exit {r.returncode}):\n{r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])["plain8"]


def add_plain_8streams(batched, res):
    """The `batched` entry against the 8-stream plain baseline (the faster solver)."""
    if "error" in res or "error" in batched:
        batched["plain_8streams_error"] = res.get("error", "the batched leg failed")
        return
    best8 = max(res["values"], key=res["values"].get)
    batched.update({"identical_8streams": res["identical"], "plain_8streams_value": res["values"][best8],
                    "speedup_vs_plain_8streams": batched["value"] / res["values"][best8],
                    "plain_8streams_solver": best8, "plain_8streams_values": res["values"],
                    "plain_8streams_streaming_by_stream_set": res["streaming_by_stream_set"],
                    "plain_8streams_process": "a child process of its own, before the benchmark's"})


def run_leg(out, key, fn, *args, **kwargs):
    """One extra leg into out[key].  An exception is printed and recorded there as
    {"error": ...}, so that a failing extra leg cannot take the main workload's
    line with it."""
    import traceback
    try:
        out[key] = fn(*args, **kwargs)
    except Exception as e:  # every failure of a leg, reported in its entry
        traceback.print_exc()
        out[key] = {"error": f"{type(e).__name__}: {e}"}


def bench_resident(steps=100, count=512, n_hi=1700):
    """Small 1D members: `count` Euler Riemann instances with N ~ LogUniform[128, n_hi]
    (each fits one workgroup's LDS), `steps` CFL steps, as one batch: the LDS-resident
    solver (one launch for all steps) against the streaming persistent sweeps.  Each
    mode is warmed up with a run of the timed length (the streaming graph is captured
    there); the resident kernel's duration, from a second pass with HIP events, gives
    its roofline (FP64 VALU: the state stays in LDS for the whole call)."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import roofline as R
    from paper_2108_12742_amd import workloads as W
    insts = W.batch_1d(1, count, n_hi=n_hi)
    probs = [E.problem_from_instance(i) for i in insts]
    cells = sum(int(p.nx) for p in probs)
    res = {"workload": f"euler1d-riemann-batch{count}-N128..{n_hi}-{cells}cells-ao5", "members": count,
           "cells": cells, "steps": steps}
    finals = []
    for mode in ("resident", "streaming"):
        E.enoao_set_resident(mode == "resident")
        try:
            b = E.enoao_batch_create(probs)
            us = [torch.from_numpy(i.u0).cuda() for i in insts]

            def restart():
                E.enoao_batch_reset(b)
                for u, i in zip(us, insts):
                    u.copy_(torch.from_numpy(i.u0))
                torch.cuda.synchronize()

            E.enoao_batch_step(b, us, steps, 0.3)  # warm-up of the timed length
            restart()
            t0 = time.perf_counter()
            E.enoao_batch_step(b, us, steps, 0.3)
            _, nst, status = E.enoao_batch_query(b)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            entry = {"value": cells * steps / el, "unit": "cell-updates/s", "ms_per_step": el * 1e3 / steps,
                     "members_ok": int((status == 0).sum())}
            if mode == "resident":
                final = [u.clone() for u in us]
                restart()
                E.enoao_batch_profile(b, True)
                E.enoao_batch_step(b, us, steps, 0.3)
                prof = E.enoao_batch_profile_read(b)
                E.enoao_batch_profile(b, False)
                ms, n = prof["resident"]
                entry["kernel_ms"] = round(ms, 4)
                roof = R.alu_entry(cells * steps * R.cell_update_flops("euler1d", 5), ms * 1e-3)
                roof["flops"] = "essential (top form) flops per cell-update"
                roof["kernel"] = "enoao::resident_1d<1, 5, true>"
                entry["roofline"] = roof
                us = final
        finally:
            E.enoao_set_resident(True)
        finals.append(us)
        res[mode] = entry
    res["identical"] = all(torch.equal(a, b) for a, b in zip(*finals))
    res["speedup_resident"] = res["resident"]["value"] / res["streaming"]["value"]
    return res


def bench_order7(n=2048, steps=30, warmup=2, tune=True):
    """The main 2D workload at order 7 (ENO-AO7, Section 3.3's nine candidates), at the
    autotuner's launch shape (the order's default with tune=False): throughput, per-kernel
    mean times and each sweep's roofline."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import roofline as R
    from paper_2108_12742_amd import tune as T
    from paper_2108_12742_amd import workloads as W
    workload = f"euler2d-quadrants-{n}x{n}-ao7"
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, n)
    ep = E.problem_from_instance(inst, order=7)
    u0 = torch.from_numpy(inst.u0).cuda()
    u = u0.clone()
    (wg, yw), kinds = (0, DEFAULT_STRIP_COLUMNS[7]), None
    if tune:
        (wg, yw), _ = T.tune_batch([ep], [u], steps=3)
        kinds, _ = T.tune_kinds([ep], [u], wg, yw)
    plan = E.enoao_plan_create(ep)
    E.enoao_plan_set_launch(plan, wg)
    E.enoao_plan_set_tiles(plan, yw)
    if kinds:
        E.enoao_plan_set_launch_kinds(plan, kinds)
    el, el_inst, prof = timed_solve(E, plan, u, u0, steps, warmup)
    cells = n * n
    kernels, best = kernel_table(R, prof, cells, 7, yw, workload)
    value = cells * steps / el
    return {"workload": workload, "steps": steps, "value": value,
            "unit": "cell-updates/s", "ms_per_step": el * 1e3 / steps,
            "workgroups_per_cu": wg, "y_strip_columns": yw,
            "workgroups_per_cu_by_kernel": list(kinds) if kinds else None,
            "instrumented_ms_per_step": round(el_inst * 1e3 / steps, 4), "roofline": kernels[best]["roofline"],
            "step_roofline": step_roofline(R, "euler2d", value, kernels, cells, steps, workload), "kernels": kernels}


def bench_discontinuous(order=5):
    """Discontinuous workloads of the paper at its meshes: the combination profile
    (advection, N = 400, t = 20) and the Lax tube (1D Euler, N = 200, t = 0.26), each a
    whole CFL-0.3 solve on the GPU; error against the exact solution."""
    import numpy as np
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import workloads as W
    from paper_2108_12742_amd import exact_riemann as RX
    out = {}
    for name, inst, tf in (("combination_wave", W.combination_wave(400), 20.0), ("lax_tube", W.lax_tube(200), 0.26)):
        entry = {"n": inst.nx, "order": order}
        for mode in ("resident", "streaming"):
            E.enoao_set_resident(mode == "resident")
            E.enoao_set_coop(False)  # lines this short take the resident solver; "streaming": the kernels
            try:
                plan = E.enoao_plan_create(E.problem_from_instance(inst, order=order))
                u = torch.from_numpy(inst.u0).cuda()
                E.enoao_solve(plan, u, tf, cfl=0.3)  # warm-up (graph capture)
                u.copy_(torch.from_numpy(inst.u0))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t, n = E.enoao_solve(plan, u, tf, cfl=0.3)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
            finally:
                E.enoao_set_resident(True)
                E.enoao_set_coop(True)
            g = u.cpu().numpy()
            if name == "lax_tube":
                ex = RX.sample((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), W.nodes(0.0, 2.0, inst.nx), 1.0, tf)[0]
            else:
                ex = inst.u0[0, 0]
            entry.update({"t_final": t, "steps": n})
            entry[mode] = {"seconds": el, "us_per_step": el * 1e6 / n, "cell_updates_per_s": inst.nx * n / el,
                           "l1_error_vs_exact": float(np.abs(g[0, 0] - ex).mean())}
        out[name] = entry
    return out


def bench_served(requests=200, nsteps=50, rates=(0.25, 0.5, 0.75, 0.9, 1.0, 1.2), arena_gib=4.0, plain=True):
    """Served workload: Poisson arrivals of 2D Euler quadrant solves, N x N with
    N ~ U{128..1024}, each request its own seeded draw of the quadrant generator,
    `nsteps` CFL steps each, admitted into a device pool by arena footprint (requests
    queue when the arena is full); rounds of several steps end when the active
    request closest to its end finishes.  Saturated throughput (all requests submitted
    at once) against the plain per-solve path (each request alone: plan, upload,
    solve, download, one after another), and p50/p99 latency per arrival rate
    (fractions of the saturated rate).  Host arrays in and out, so PCIe is included.
    A draw that the scheme drives to a non-physical state stops there (in the pool and
    alone alike: the request reports the failure); the work counted is the steps each
    request actually took."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import serve as S
    from paper_2108_12742_amd import workloads as W
    t_arr, sizes, seeds = W.arrivals(1, requests, 1.0)
    data = [W.quadrants(int(sd), int(n)) for sd, n in zip(seeds, sizes)]
    probs = [E.problem_from_instance(d) for d in data]
    like = probs[0]
    arena = int(arena_gib * (1 << 30))

    def server():
        return S.Server(S.GpuPoolBackend(like, max_members=256, arena_bytes=arena))

    # an untimed pass of the same requests first: the first server of a process ran
    # about 4% slower than the ones after it (one-time set-up of the pool, the
    # staging buffers and streams)
    srv = server()
    for p, d in zip(probs, data):
        srv.submit(p, d.u0, nsteps)
    srv.drain()
    srv.backend.close()
    # saturated: every request submitted at once
    srv = server()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, d in zip(probs, data):
        srv.submit(p, d.u0, nsteps)
    done = srv.drain()
    sat_s = time.perf_counter() - t0
    by_id = {r.rid: r for r in done}
    taken = [by_id[i].steps_done for i in range(requests)]
    work = sum(int(p.nx) * int(p.ny) * k for p, k in zip(probs, taken))
    failed = [i for i in range(requests) if by_id[i].status != 0]
    out = {"workload": f"euler2d-served-{requests}req-{nsteps}steps-N128..1024-ao5", "requests": requests,
           "request_data": "quadrant draws, one seed per request",
           "saturated": {"requests_per_s": requests / sat_s, "cell_updates_per_s": work / sat_s,
                         "failed_nonphysical": len(failed), "rounds": srv.rounds},
           "rates": []}
    if not plain:
        return out
    # plain: each request alone, one after another (plan creation included, as a
    # per-request caller of the plain path would do it)
    plain_res = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (p, d) in enumerate(zip(probs, data)):
        plan = E.enoao_plan_create(p)
        u = torch.from_numpy(d.u0).cuda()
        try:
            E.enoao_solve(plan, u, 1e300, cfl=0.3, max_steps=nsteps)
            plain_res[i] = u.cpu().numpy()
        except E.EnoaoError:
            plain_res[i] = None
        del plan
    plain_s = time.perf_counter() - t0
    same = all((by_id[i].status != 0) == (plain_res[i] is None) and
               (plain_res[i] is None or np.array_equal(by_id[i].result, plain_res[i])) for i in range(requests))
    out["saturated"].update({"plain_cell_updates_per_s": work / plain_s, "speedup_vs_plain": plain_s / sat_s,
                             "identical_to_plain": same})
    sat_rate = requests / sat_s
    for f in rates:
        rate = f * sat_rate
        arr = t_arr / t_arr[-1] * (requests - 1) / rate if requests > 1 else t_arr
        srv = server()
        reqs, wall = S.run_arrivals(srv, arr, lambda i: (probs[i], data[i].u0, nsteps))
        st = S.latency_stats(reqs)
        st.update({"rate_fraction": f, "requests_per_s": rate,
                   "cell_updates_per_s": sum(int(r.problem.nx) * int(r.problem.ny) * r.steps_done for r in reqs) / wall,
                   "failed": sum(r.status != 0 for r in reqs), "rounds": srv.rounds})
        out["rates"].append(st)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2048, help="nodes per direction")
    ap.add_argument("--order", type=int, default=5, choices=(5, 7))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (512 1D members, batched vs plain) and served (Poisson arrivals) legs")
    ap.add_argument("--served-requests", type=int, default=200)
    ap.add_argument("--no-tune", action="store_true",
                    help="main workload at the default launch shape (occupancy; y strips of the "
                         "order's default width, or --y-strip-columns)")
    ap.add_argument("--y-strip-columns", type=int, default=0, choices=(0, 4, 8),
                    help="with --no-tune: y-sweep strip width (0 = the order's default)")
    ap.add_argument("--workgroups-per-cu", type=int, default=0,
                    help="with --no-tune: resident workgroups per CU of the persistent sweeps (0 = occupancy)")
    ap.add_argument("--only-leg", choices=("batched", "batched_small", "served", "c1", "plain8"), default=None,
                    help="run only this extra leg (with --steps, --warmup and --no-tune; no comparison "
                         "against one plan per member) and print its JSON: a short run to profile")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the run, one device-to-device copy of this many MiB (a known-size "
                         "reference for the HBM byte counters of a profiler pass)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the kernels are measured on a single GPU "
              "(sharding across GPUs is described in the design notes, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    plain8 = None
    if not args.no_extras and args.only_leg is None:
        print("[bench] batched workload's plain solves over 8 streams, in a process of their own ...",
              file=sys.stderr, flush=True)
        box = {}
        run_leg(box, "plain8", run_plain_8streams)
        plain8 = box["plain8"]

    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import roofline as R
    from paper_2108_12742_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only_leg == "batched":
        print(json.dumps({"batched": bench_batched(steps=args.steps, warmup=args.warmup, tune=not args.no_tune,
                                                   plain=False, wg=args.workgroups_per_cu)}), flush=True)
        return
    if args.only_leg == "batched_small":
        print(json.dumps({"batched_small": bench_resident(steps=args.steps)}), flush=True)
        return
    if args.only_leg == "served":  # saturated throughput only (no plain path, no arrival rates)
        print(json.dumps({"served": bench_served(requests=args.served_requests, plain=False)}), flush=True)
        return
    if args.only_leg == "plain8":  # the batched workload's plain solves over 8 streams
        print(json.dumps({"plain8": plain_8streams(steps=args.steps)}), flush=True)
        return
    if args.only_leg == "c1":  # the 1D Euler N = 2000 solves, cooperative solver only
        print(json.dumps({"euler1d_c1": bench_c1(repeats=1, streaming=False)}), flush=True)
        return
    n, K, Wu = args.n, args.steps, args.warmup
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, n)
    ep = E.problem_from_instance(inst, order=args.order)
    u0 = torch.from_numpy(inst.u0).cuda()
    u = u0.clone()
    launch, tuner = (args.workgroups_per_cu, args.y_strip_columns or DEFAULT_STRIP_COLUMNS[args.order]), None
    kinds, kinds_info = None, None
    if not args.no_tune:  # launch shape (workgroups per CU, y strip columns) from the autotuner
        from paper_2108_12742_amd import tune as T
        launch, tuner = T.tune_batch([ep], [u], steps=3)
        kinds, kinds_info = T.tune_kinds([ep], [u], launch[0], launch[1])
    plan = E.enoao_plan_create(ep)
    E.enoao_plan_set_launch(plan, launch[0])
    E.enoao_plan_set_tiles(plan, launch[1])
    if kinds:
        E.enoao_plan_set_launch_kinds(plan, kinds)
    el, el_inst, prof = timed_solve(E, plan, u, u0, K, Wu)

    cells = n * n
    value = cells * K / el
    workload = f"euler2d-quadrants-{n}x{n}-ao{args.order}"
    kernels, best = kernel_table(R, prof, cells, args.order, launch[1], workload)
    roof = dict(kernels[best]["roofline"])
    roof["step"] = step_roofline(R, "euler2d", value, kernels, cells, K, workload)
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": Wu,
        "ms_per_step": el * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "kernel_timing": {"pass": "the same K steps again with a HIP event pair around every launch",
                          "ms_per_step": round(el_inst * 1e3 / K, 4)},
        "config": {"workload": workload, "nx": n, "ny": n, "order": args.order,
                   "bc": "periodic", "cfl": 0.3, "seed": W.QUADRANT_BENCH_SEED, "parallelism": "single-gpu",
                   "workgroups_per_cu": launch[0], "y_strip_columns": launch[1],
                   "workgroups_per_cu_by_kernel": list(kinds) if kinds else None},
        "tuner_ms_per_step": tuner,
        "tuner_by_kernel": kinds_info,
        "roofline": roof,
        "cpu_baseline": None,
        "kernels": kernels,
        "essential_flops_per_cell_update": R.cell_update_flops("euler2d", args.order),
    }
    # stencil choices on the state the timed steps reached (the metric depends on them:
    # waves whose faces all take the top candidate skip the rest of the selection)
    rec = E.enoao_plan_create(E.problem_from_instance(inst, order=args.order, record_selection=True))
    Lh = torch.empty_like(u)
    E.enoao_rhs(rec, u, Lh)
    sel = E.enoao_get_selection(rec)
    nxs = 4 * 2 * n * (n + 1)
    K = 6 if args.order == 5 else 9
    out["selection_histogram"] = {
        "candidates": "increasing priority; index K-1 is the full stencil",
        "x": [round(float(v), 5) for v in np.bincount(sel[:nxs], minlength=K) / nxs],
        "y": [round(float(v), 5) for v in np.bincount(sel[nxs:], minlength=K) / (sel.size - nxs)]}
    del plan, u, u0, rec, Lh
    if not args.no_cpu_baseline:
        print("[bench] oracle baseline on the host ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    if not args.no_extras:
        print(f"[bench] main workload: {value:.4g} cell-updates/s; smooth advection latency ...", file=sys.stderr,
              flush=True)
        run_leg(out, "advection_c0", bench_c0)
        print("[bench] 1D Euler N = 2000 to t = 0.2 ...", file=sys.stderr, flush=True)
        run_leg(out, "euler1d_c1", bench_c1)
        print("[bench] batched leg ...", file=sys.stderr, flush=True)
        run_leg(out, "batched", bench_batched)
        print("[bench] batched leg done; LDS-resident small members ...", file=sys.stderr, flush=True)
        run_leg(out, "batched_small", bench_resident)
        print("[bench] order 7 ...", file=sys.stderr, flush=True)
        run_leg(out, "order7", bench_order7, n=n)
        print("[bench] discontinuous workloads ...", file=sys.stderr, flush=True)
        run_leg(out, "discontinuous", bench_discontinuous)
        print("[bench] served leg ...", file=sys.stderr, flush=True)
        run_leg(out, "served", bench_served, requests=args.served_requests)
        add_plain_8streams(out["batched"], plain8)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
