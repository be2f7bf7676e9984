#!/usr/bin/env python3
"""Throughput of the ENO-AO hot path on one MI355X.

Default workload: 2D Euler, 2048 x 2048 nodes, periodic, four seeded quadrant
states (rho, p ~ LogUniform[0.1, 10], u, v ~ U[-2, 2], generator seed
workloads.QUADRANT_BENCH_SEED), fifth-order ENO-AO with
Roe characteristic decomposition, SSP-RK3 with the device-side CFL step
(CFL 0.3); K timed steps after W warm-up steps, inputs resident in HBM.

Prints one JSON line: cell-updates/s of the whole job, the roofline of the
dominant kernel (HIP events on the stream the kernels run on), and the CPU
oracle timed on a bounded sample of the same workload.
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
        return f"enoao::sweep_x<2, {order}, {stage}, false>"
    return f"enoao::sweep_y<{order}, {stage}, false, {y_strip_columns}>"


def kernel_sources_hash():
    """sha256 (first 16 hex) of the HIP sources and of the build script that holds the
    compiler flags: a change to either invalidates the recorded byte counters."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(here, "paper_2108_12742_amd", "csrc", "*.hip"))
                   + glob.glob(os.path.join(here, "paper_2108_12742_amd", "csrc", "*.hpp")))
    files.append(os.path.join(here, "paper_2108_12742_amd", "build.py"))
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def measured_traffic(symbol, workload):
    """HBM bytes per launch of `symbol` from the committed rocprofv3 byte counters
    (profiles/traffic.json, per workload), or None when the kernels changed since
    they were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_sources_hash():
        return None
    v = t.get("workloads", {}).get(workload, {}).get("bytes_per_launch", {}).get(symbol)
    return None if v is None else round(v)


def cpu_baseline(n_sample=2048, steps=1):
    """The oracle (single-threaded C, FP64) on a bounded sample of the workload: the
    first `steps` of its SSP-RK3 steps (same seeded quadrant problem, same size)."""
    from oracle import oracle as O
    from paper_2108_12742_amd import workloads as W
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, n_sample)
    p = O.Problem(O.EULER2D, nx=n_sample, ny=n_sample, order=5)
    u = inst.u0
    t0 = time.perf_counter()
    for _ in range(steps):
        dt = O.cfl_dt(p, u, 0.3)
        u = O.step(p, u, dt)
    el = time.perf_counter() - t0
    return {"value": n_sample * n_sample * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of the 2D Euler quadrant workload (seed {W.QUADRANT_BENCH_SEED}) at {n_sample}x{n_sample}, "
                      f"{el:.1f} s on one host core"}


def bench_batched(steps=100, warmup=2, count=512, tune=True, plain=True):
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
    (best, yw), timing = T.tune_batch(probs, states, steps=3) if tune else ((0, 8), {})
    batch = E.enoao_batch_create(probs)
    E.enoao_batch_set_launch(batch, best)

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
    roof = R.roofline_entry(cells * R.sweep_flops("euler1d", 5, "x", stage), cells * R.sweep_bytes("euler1d", "x", stage),
                            ms * 1e-3)
    roof["kernel"] = f"enoao::sweep_x<1, 5, {stage}, false>"
    roof["traffic"] = measured_traffic(roof["kernel"], workload)
    out = {"workload": workload, "members": count, "cells": cells, "steps": steps,
           "value": cells * steps / el, "unit": "cell-updates/s", "ms_per_step": el * 1e3 / steps,
           "instrumented_ms_per_step": round(el_inst * 1e3 / steps, 4),
           "members_ok": int((status == 0).sum()), "workgroups_per_cu": best,
           "tuner_ms_per_step": {str(k): round(v, 4) for k, v in timing.items()}, "roofline": roof}
    if not plain:
        return out
    # plain: one plan per instance, solved one after another on the same stream
    plans = [E.enoao_plan_create(p) for p in probs]
    plain = [u.clone() for u in u0]
    for pl, u, v in zip(plans, plain, u0):  # graph capture and first touch, untimed
        E.enoao_solve(pl, u, 1e300, cfl=0.3, max_steps=warmup)
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
                roof = R.roofline_entry(cells * steps * R.cell_update_flops("euler1d", 5),
                                        cells * steps * R.resident_bytes("euler1d", steps), ms * 1e-3)
                roof["kernel"] = "enoao::resident_1d<1, 5>"
                entry["roofline"] = roof
                us = final
        finally:
            E.enoao_set_resident(True)
        finals.append(us)
        res[mode] = entry
    res["identical"] = all(torch.equal(a, b) for a, b in zip(*finals))
    res["speedup_resident"] = res["resident"]["value"] / res["streaming"]["value"]
    return res


def bench_order7(n=2048, steps=30, warmup=2):
    """The main 2D workload at order 7 (ENO-AO7, Section 3.3's nine candidates), with the
    default launch shape: throughput, per-kernel mean times and each sweep's roofline."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import roofline as R
    from paper_2108_12742_amd import workloads as W
    workload = f"euler2d-quadrants-{n}x{n}-ao7"
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, n)
    plan = E.enoao_plan_create(E.problem_from_instance(inst, order=7))
    u0 = torch.from_numpy(inst.u0).cuda()
    u = u0.clone()
    el, el_inst, prof = timed_solve(E, plan, u, u0, steps, warmup)
    cells = n * n
    kernels = {}
    for kind, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        entry = {"mean_ms": round(ms, 4), "launches": cnt}
        if kind.startswith("sweep"):
            kern, stage = kind[6], int(kind[-1])
            entry["symbol"] = kernel_symbol(kind, 7, DEFAULT_STRIP_COLUMNS[7])
            entry["roofline"] = R.roofline_entry(cells * R.sweep_flops("euler2d", 7, kern, stage),
                                                 cells * R.sweep_bytes("euler2d", kern, stage), ms * 1e-3)
            entry["roofline"]["traffic"] = measured_traffic(entry["symbol"], workload)
        kernels[kind] = entry
    return {"workload": workload, "steps": steps, "value": cells * steps / el,
            "unit": "cell-updates/s", "ms_per_step": el * 1e3 / steps,
            "instrumented_ms_per_step": round(el_inst * 1e3 / steps, 4), "kernels": kernels}


def bench_discontinuous(order=5):
    """Discontinuous workloads of the paper at its meshes: the combination profile
    (advection, N = 400, t = 20) and the Lax tube (1D Euler, N = 200, t = 0.26), each a
    whole CFL-0.3 solve on the GPU; error against the exact solution."""
    import numpy as np
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import workloads as W
    from tests import riemann_exact as RX
    out = {}
    for name, inst, tf in (("combination_wave", W.combination_wave(400), 20.0), ("lax_tube", W.lax_tube(200), 0.26)):
        entry = {"n": inst.nx, "order": order}
        for mode in ("resident", "streaming"):
            E.enoao_set_resident(mode == "resident")
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


def bench_served(requests=200, nsteps=50, rates=(0.25, 0.5, 0.75, 0.9, 1.0, 1.2), arena_gib=4.0):
    """Served workload: Poisson arrivals of 2D Euler quadrant solves, N x N with
    N ~ U{128..1024}, `nsteps` steps each, admitted into a device pool by arena
    footprint; p50/p99 latency per arrival rate (fractions of the saturated rate)."""
    import torch
    from paper_2108_12742_amd import enoao as E
    from paper_2108_12742_amd import serve as S
    from paper_2108_12742_amd import workloads as W
    t_arr, sizes, _ = W.arrivals(1, requests, 1.0)
    # every request is the four-quadrant problem of the main workload at its own size
    data = [W.quadrants(W.QUADRANT_BENCH_SEED, int(n)) for n in sizes]
    probs = [E.problem_from_instance(d) for d in data]
    like = probs[0]
    arena = int(arena_gib * (1 << 30))

    def server():
        return S.Server(S.GpuPoolBackend(like, max_members=256, arena_bytes=arena), steps_per_round=1)

    # saturated: every request submitted at once
    srv = server()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, d in zip(probs, data):
        srv.submit(p, d.u0, nsteps)
    done = srv.drain()
    sat_s = time.perf_counter() - t0
    sat_rate = requests / sat_s
    total_cu = sum(int(p.nx) * int(p.ny) for p in probs) * nsteps
    out = {"workload": f"euler2d-served-{requests}req-{nsteps}steps-N128..1024-ao5", "requests": requests,
           "saturated": {"requests_per_s": sat_rate, "cell_updates_per_s": total_cu / sat_s,
                         "failed": sum(r.status != 0 for r in done)}, "rates": []}
    for f in rates:
        rate = f * sat_rate
        arr = t_arr / t_arr[-1] * (requests - 1) / rate if requests > 1 else t_arr
        srv = server()
        reqs, wall = S.run_arrivals(srv, arr, lambda i: (probs[i], data[i].u0, nsteps))
        st = S.latency_stats(reqs)
        st.update({"rate_fraction": f, "requests_per_s": rate, "cell_updates_per_s": total_cu / wall,
                   "failed": sum(r.status != 0 for r in reqs)})
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
    ap.add_argument("--only-leg", choices=("batched",), default=None,
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
                                                   plain=False)}), flush=True)
        return
    n, K, Wu = args.n, args.steps, args.warmup
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, n)
    ep = E.problem_from_instance(inst, order=args.order)
    u0 = torch.from_numpy(inst.u0).cuda()
    u = u0.clone()
    launch, tuner = (0, args.y_strip_columns or DEFAULT_STRIP_COLUMNS[args.order]), None
    if not args.no_tune:  # launch shape (workgroups per CU, y strip columns) from the autotuner
        from paper_2108_12742_amd import tune as T
        launch, tuner = T.tune_batch([ep], [u], steps=3)
    plan = E.enoao_plan_create(ep)
    E.enoao_plan_set_launch(plan, launch[0])
    E.enoao_plan_set_tiles(plan, launch[1])
    el, el_inst, prof = timed_solve(E, plan, u, u0, K, Wu)

    cells = n * n
    value = cells * K / el
    kernels = {}
    best = None
    for kind, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        entry = {"mean_ms": round(ms, 4), "launches": cnt}
        if kind.startswith("sweep"):
            kern = kind[6]
            stage = int(kind[-1])
            fl = cells * R.sweep_flops("euler2d", args.order, kern, stage)
            by = cells * R.sweep_bytes("euler2d", kern, stage)
            entry["roofline"] = R.roofline_entry(fl, by, ms * 1e-3)
            entry["symbol"] = kernel_symbol(kind, args.order, launch[1])
            if best is None or ms * cnt > best[1]:
                best = (kind, ms * cnt)
        kernels[kind] = entry
    roof = dict(kernels[best[0]]["roofline"])
    roof["kernel"] = kernels[best[0]]["symbol"]
    workload = f"euler2d-quadrants-{n}x{n}-ao{args.order}"
    roof["traffic"] = measured_traffic(roof["kernel"], workload)
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": Wu,
        "ms_per_step": el * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "kernel_timing": {"pass": "the same K steps again with a HIP event pair around every launch",
                          "ms_per_step": round(el_inst * 1e3 / K, 4)},
        "config": {"workload": workload, "nx": n, "ny": n, "order": args.order,
                   "bc": "periodic", "cfl": 0.3, "seed": W.QUADRANT_BENCH_SEED, "parallelism": "single-gpu",
                   "workgroups_per_cu": launch[0], "y_strip_columns": launch[1]},
        "tuner_ms_per_step": tuner,
        "roofline": roof,
        "cpu_baseline": None,
        "kernels": kernels,
        "flops_per_cell_update": R.cell_update_flops("euler2d", args.order),
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
        print(f"[bench] main workload: {value:.4g} cell-updates/s; batched leg ...", file=sys.stderr, flush=True)
        out["batched"] = bench_batched()
        print("[bench] batched leg done; LDS-resident small members ...", file=sys.stderr, flush=True)
        out["batched_small"] = bench_resident()
        print("[bench] order 7 ...", file=sys.stderr, flush=True)
        out["order7"] = bench_order7(n=n)
        print("[bench] discontinuous workloads ...", file=sys.stderr, flush=True)
        out["discontinuous"] = bench_discontinuous()
        print("[bench] served leg ...", file=sys.stderr, flush=True)
        out["served"] = bench_served(requests=args.served_requests)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
