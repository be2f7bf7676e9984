"""Autotuner of the persistent launches.

The sweeps run as persistent grids of (CUs x W) workgroups; W (workgroups of 4
waves resident per CU) trades latency hiding against the tail of the last
tiles.  In 2D the y-sweep tile width is a second knob: wave strips of 4 or 8
columns (longer row segments per load against fewer staged halo rows).  The
tuner times a few steps of the caller's batch for each candidate (W, width)
and keeps the fastest per (equation, order, size bucket) in a JSON cache
(ENOAO_TUNE_CACHE, default ~/.cache/enoao_tune.json).  tune_kinds then lets
each stage kernel take its own W (coordinate descent on whole timed steps),
kept when a whole step beats the uniform shape.  Results do not depend on any
of these knobs, so tuning never changes answers.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATES = (0, 1, 2, 3, 4, 6, 8, 12, 16)  # W; 0 = the occupancy the kernels' resources allow
Y_WIDTHS = (8, 4)                    # columns per wave strip of the y tiles (2D only)


def cache_path():
    return os.environ.get("ENOAO_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "enoao_tune.json"))


def build_id() -> str:
    """First 12 hex digits of the sha256 of the built library: a rebuilt library does
    not reuse launch shapes tuned for the previous kernels."""
    import hashlib
    from . import enoao as E
    try:
        with open(E.LIB_PATH, "rb") as fh:
            return hashlib.sha256(fh.read()).hexdigest()[:12]
    except OSError:
        return "nolib"


def bucket_key(problems) -> str:
    """(equation, order, log2 of the total cell count, log2 of the member count, library build)."""
    cells = sum(int(p.nx) * int(p.ny) for p in problems)
    return (f"eq{problems[0].equation}-o{problems[0].order}-c{int(math.log2(max(cells, 1)))}"
            f"-m{int(math.log2(len(problems)))}-b{build_id()}")


def load_cache():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def store(key, value):
    c = load_cache()
    c[key] = value
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(c, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_batch(problems, states, steps=4, candidates=CANDIDATES, cfl=0.3, use_cache=True, rounds=2):
    """Best launch shape for advancing `problems` (GPU tensors `states`, restored
    afterwards): ((workgroups per CU, y strip columns), {"W/width": ms per step}).
    Each candidate's time is the best of `rounds` timings of `steps` steps, after
    an untimed warm-up of several times that work (clocks ramp up on the first
    launches, which would otherwise penalise the first candidate)."""
    import torch
    from . import enoao as E
    key = bucket_key(problems)
    if use_cache:
        hit = load_cache().get(key)
        if hit is not None and "y_strip_columns" in hit:
            return (hit["workgroups_per_cu"], hit["y_strip_columns"]), hit["ms_per_step"]
    widths = Y_WIDTHS if problems[0].equation == E.EULER2D else (Y_WIDTHS[0],)
    saved = [u.clone() for u in states]
    timing = {}

    def run(w, yw, n):
        batch = E.enoao_batch_create(problems)
        E.enoao_batch_set_launch(batch, w)
        E.enoao_batch_set_tiles(batch, yw)
        # warm-up of the same length: the graph of n steps is captured on its first
        # replay, which then stays out of the timing
        E.enoao_batch_step(batch, states, n, cfl)
        E.enoao_batch_reset(batch)
        for u, s in zip(states, saved):
            u.copy_(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E.enoao_batch_step(batch, states, n, cfl)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) * 1e3 / max(n, 1)
        E.enoao_batch_destroy(batch)
        for u, s in zip(states, saved):
            u.copy_(s)
        return el

    run(candidates[0], widths[0], 4 * steps)  # untimed: module loads, first touches, clock ramp
    for _ in range(max(rounds, 1)):
        for yw in widths:
            for w in candidates:
                k = f"{w}/{yw}"
                t = run(w, yw, steps)
                timing[k] = min(timing.get(k, t), t)
    best = min(timing, key=timing.get)
    w, yw = (int(x) for x in best.split("/"))
    store(key, {"workgroups_per_cu": w, "y_strip_columns": yw, "ms_per_step": timing})
    return (w, yw), timing


KINDS = ("sweep_x_s1", "sweep_x_s2", "sweep_x_s3", "sweep_y_s1", "sweep_y_s2", "sweep_y_s3")


def tune_kinds(problems, states, w, yw, steps=30, candidates=(2, 3, 4, 6), cfl=0.3, use_cache=True, rounds=3):
    """Per-kernel launch shapes on top of the uniform (w, yw) from tune_batch, by
    coordinate descent on whole steps: kernel kind by kind (x-sweep stages 1..3,
    then in 2D y-sweep stages 1..3), each candidate W for that kind is compared
    with the current shapes on whole captured steps, the two timed in turn (best
    of `rounds` timings of `steps` steps each: long enough that the launch and the
    synchronisation around a timing stay below the differences sought, and taken
    in turn so that drifts of the clock affect both), and kept when it gains more
    than 0.3%.  The result is kept if it beats the uniform shape by more than
    0.5% in a last comparison of the same kind.  (The kernels' durations in a
    profiled run, with events between the launches, did not rank the shapes of the
    later y-sweeps as a graph replay does.)  Returns (shapes, info): shapes is a
    tuple of workgroups per CU per kind (0: the uniform w) or None; info has the
    trials (ms per step, current and candidate) and the last comparison."""
    import torch
    from . import enoao as E
    key = bucket_key(problems) + f"-kinds-w{w}-y{yw}"
    if use_cache:
        hit = load_cache().get(key)
        if hit is not None and "shapes" in hit:
            return (tuple(hit["shapes"]) if hit["shapes"] else None), hit["info"]
    nk = 6 if problems[0].equation == E.EULER2D else 3
    saved = [u.clone() for u in states]

    def restore():
        for u, s in zip(states, saved):
            u.copy_(s)

    def make(shape):
        batch = E.enoao_batch_create(problems)
        E.enoao_batch_set_launch(batch, w)
        E.enoao_batch_set_tiles(batch, yw)
        if shape is not None:
            E.enoao_batch_set_launch_kinds(batch, shape)
        E.enoao_batch_step(batch, states, steps, cfl)  # graph capture outside the timings
        restore()
        return batch

    def one(batch):
        E.enoao_batch_reset(batch)
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E.enoao_batch_step(batch, states, steps, cfl)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / max(steps, 1)

    def compare(sa, sb, n):
        a, b = make(sa), make(sb)
        ta = tb = math.inf
        for _ in range(max(n, 1)):
            ta = min(ta, one(a))
            tb = min(tb, one(b))
        E.enoao_batch_destroy(a)
        E.enoao_batch_destroy(b)
        restore()
        return ta, tb

    shape = [0] * nk
    trials = {}
    for k in range(nk):
        for c in candidates:
            if c == w or c == shape[k]:
                continue
            trial = list(shape)
            trial[k] = c
            t_cur, t_new = compare(shape, trial, rounds)
            trials[f"{KINDS[k]}={c}"] = [round(t_cur, 4), round(t_new, 4)]
            if t_new < 0.997 * t_cur:
                shape = trial
    shape = tuple(shape)
    if any(shape):
        uniform_ms, kinds_ms = compare(None, shape, rounds + 2)
    else:
        uniform_ms = kinds_ms = compare(None, None, 1)[0]
    keep = any(shape) and kinds_ms < 0.995 * uniform_ms
    info = {"trials_ms_per_step": trials, "uniform_ms_per_step": round(uniform_ms, 4),
            "kinds_ms_per_step": round(kinds_ms, 4), "shapes": list(shape)}
    store(key, {"shapes": list(shape) if keep else None, "info": info})
    return (shape if keep else None), info
