"""Continuous-batching service for ENO-AO solves.

Requests (an initial state and a number of SSP-RK3 steps) arrive over time.
The server admits them into a device pool as arena memory frees up (FIFO by
arrival; a request that can never fit is rejected), advances every admitted
request together with the batched kernels, and retires each one when its
last step is done.  Request states stay in HBM between steps; admissions and
retirements happen between step rounds, while other requests are on the GPU.
A backend may move states between host and device asynchronously: `stage`
starts a queued request's upload while a round computes, and `retire` may hand
back a pending result whose download overlaps later rounds; the server finishes
a request when its result has arrived.

A round is several steps of the pool when nothing would be gained by stopping
earlier: with steps_per_round = 0 (the default) a round runs as many steps as
the active request closest to its end still needs (at most max_round_steps), so
that request retires, and its memory frees up for the queue, exactly when the
round ends; every request stops at its own step count on the device either way.

A pipelined backend (retire_async and fence) lets the host run ahead of the
device: every member takes exactly the steps it is given, so the server knows
which requests end with a round without reading the device, retires them right
after enqueuing that round (their copies follow it on the stream), and admits
the next ones into the freed memory while the round computes.  A request that
stopped early (a non-physical state) is found from the progress its retirement
returns.  fence() keeps at most a few rounds in flight.  Otherwise the host
reads the pool's state once per round (poll) and retires what it reports done.

The scheduling is independent of the device: `Server` drives any backend with
the `Backend` methods below.  `GpuPoolBackend` is the HIP pool of the C ABI.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    problem: object            # enoao.Problem
    u0: np.ndarray
    nsteps: int
    cfl: float
    arrival: float
    admitted: float | None = None
    finished: float | None = None
    slot: int | None = None
    steps_done: int = 0        # steps taken, as of the last poll
    staged: object = None      # backend handle of an upload started before admission
    result: np.ndarray | None = None
    status: int = 0            # 0 ok, non-zero: non-physical state or rejected
    error: str | None = None

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival

    @property
    def cell_updates(self):
        return int(self.problem.nx) * int(self.problem.ny) * self.nsteps


class Backend:
    """What the server needs from a device pool."""
    max_members: int
    arena_bytes: int
    pipelined = False   # True: retire_async and fence below are available

    def member_bytes(self, problem) -> int: ...
    def admit(self, problem, u0, nsteps, cfl): ...  # slot, or None when there is no room now
    def step(self, nsteps: int): ...
    def poll(self): ...                            # (done, status, steps) per slot
    def retire(self, slot: int, shape): ...        # final state: numpy, or a Pending

    def stage(self, problem, u0):
        """Start moving u0 towards the device; the result is passed to admit in place
        of u0.  The default keeps u0 (admit copies it)."""
        return u0

    def retire_async(self, slot: int, shape):  # a Pending whose info() gives (status, steps)
        raise NotImplementedError

    def ready(self, staged) -> bool:
        """Whether a staged state has arrived (admitting it would not wait)."""
        return True

    def fence(self):
        """Called after each round is enqueued: waits while too many are in flight."""


class Pending:
    """A result on its way to the host."""

    def ready(self) -> bool: ...
    def result(self) -> np.ndarray: ...

    def info(self):
        """(status, steps) of the member when it was retired, or None if unknown."""
        return None


class _Download(Pending):
    def __init__(self, host, event, host_info=None):
        self.host, self.event, self.host_info = host, event, host_info

    def ready(self):
        return self.event.query()

    def result(self):
        # a view of the pinned buffer: the caller holds it until it drops the
        # result (copying it out instead cost 20-40% of the saturated rate)
        self.event.synchronize()
        return self.host.numpy()

    def info(self):
        if self.host_info is None:
            return None
        self.event.synchronize()
        i = self.host_info.numpy()
        return int(i[1]), int(i[2])


class GpuPoolBackend(Backend):
    """The HIP pool.  With overlap=True, host states move through pinned memory on a
    copy stream of their own: inputs are copied into pinned memory and uploaded by a
    staging thread while rounds compute, and admitted from the device; results are
    copied out of the arena on the device and downloaded while later rounds compute.
    (Uploading at admission instead, from pageable memory, held the host about 1 ms per
    request while the device idled at the boundary between two generations of
    requests.)"""

    def __init__(self, like, max_members=256, arena_bytes=8 << 30, stream=None, workgroups_per_cu=0,
                 overlap=True, depth=2):
        import torch
        from . import enoao as E
        self.E, self.torch = E, torch
        self.stream = stream
        self.pipelined = overlap
        self.depth = depth      # rounds in flight at most (pipelined)
        self.inflight = deque()
        self.pool = E.enoao_pool_create(like, max_members, arena_bytes, stream)
        if workgroups_per_cu:
            E.enoao_pool_set_launch(self.pool, workgroups_per_cu)
        self.max_members = max_members
        self.arena_bytes = E.enoao_pool_usage(self.pool)[1]
        self.device = torch.cuda.current_device()
        self.copy = torch.cuda.Stream() if overlap else None
        self.stager = ThreadPoolExecutor(1) if overlap else None

    def _compute(self):
        return self.stream if self.stream is not None else self.torch.cuda.current_stream()

    def member_bytes(self, problem):
        return self.E.enoao_pool_member_bytes(problem)

    def stage(self, problem, u0):
        if self.copy is None or not isinstance(u0, np.ndarray):
            return u0
        return self.stager.submit(self._upload, u0)

    def _upload(self, u0):
        # staging thread: pinned copy, then the upload on the copy stream
        torch = self.torch
        host = torch.empty(u0.shape, dtype=torch.float64, pin_memory=True)
        host.numpy()[...] = u0
        with torch.cuda.device(self.device), torch.cuda.stream(self.copy):
            dev = torch.empty(u0.shape, dtype=torch.float64, device="cuda")
            dev.copy_(host, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy)
        return (dev, ev, host)

    def ready(self, staged):
        if isinstance(staged, Future):
            return staged.done() and staged.result()[1].query()
        return True

    def admit(self, problem, u0, nsteps, cfl):
        if isinstance(u0, Future):
            u0 = u0.result()
        if isinstance(u0, tuple):
            dev, ev, _ = u0
            comp = self._compute()
            comp.wait_event(ev)
            dev.record_stream(comp)
            u0 = dev
        return self.E.enoao_pool_admit(self.pool, problem, u0, max_steps=nsteps, cfl=cfl, stream=self.stream)

    def step(self, nsteps):
        self.E.enoao_pool_step(self.pool, nsteps, self.stream)

    def poll(self):
        d, f, s, _ = self.E.enoao_pool_poll(self.pool, self.stream)
        return d, f, s

    def retire(self, slot, shape):
        if self.copy is None:
            return self.E.enoao_pool_retire(self.pool, slot, shape=shape, stream=self.stream)
        torch = self.torch
        comp = self._compute()
        dev = torch.empty(shape, dtype=torch.float64, device="cuda")
        self.E.enoao_pool_retire(self.pool, slot, out=dev, stream=self.stream)
        host = torch.empty(shape, dtype=torch.float64, pin_memory=True)
        self.copy.wait_stream(comp)
        with torch.cuda.stream(self.copy):
            host.copy_(dev, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy)
        dev.record_stream(self.copy)
        return _Download(host, ev)

    def retire_async(self, slot, shape):
        torch = self.torch
        comp = self._compute()
        dev = torch.empty(shape, dtype=torch.float64, device="cuda")
        info = torch.empty(4, dtype=torch.float64, device="cuda")
        self.E.enoao_pool_retire_async(self.pool, slot, out=dev, info=info, stream=self.stream)
        host = torch.empty(shape, dtype=torch.float64, pin_memory=True)
        host_info = torch.empty(4, dtype=torch.float64, pin_memory=True)
        self.copy.wait_stream(comp)
        with torch.cuda.stream(self.copy):
            host.copy_(dev, non_blocking=True)
            host_info.copy_(info, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy)
        dev.record_stream(self.copy)
        info.record_stream(self.copy)
        return _Download(host, ev, host_info)

    def fence(self):
        ev = self.torch.cuda.Event()
        ev.record(self._compute())
        self.inflight.append(ev)
        while len(self.inflight) > self.depth:
            self.inflight.popleft().synchronize()

    def close(self):
        if self.stager is not None:
            self.stager.shutdown(wait=True)
        self.E.enoao_pool_destroy(self.pool)


@dataclass
class Server:
    backend: Backend
    steps_per_round: int = 0   # 0: adaptive (the fewest steps an active request still needs)
    max_round_steps: int = 8   # bound on an adaptive round (latency of newly arrived requests)
    clock: object = time.perf_counter
    stage_ahead: int = 64      # queued requests whose upload may start while rounds compute
    stage_bytes: int = 1 << 30  # ... as long as their states total at most this many bytes
    queue: deque = field(default_factory=deque)
    active: dict = field(default_factory=dict)   # slot -> Request
    pending: list = field(default_factory=list)  # (Request, Pending) results on their way
    done: list = field(default_factory=list)
    rounds: int = 0
    _next_id: int = 0

    def submit(self, problem, u0, nsteps, cfl=0.3, arrival=None) -> Request:
        r = Request(self._next_id, problem, np.ascontiguousarray(u0, np.float64), int(nsteps), float(cfl),
                    self.clock() if arrival is None else arrival)
        self._next_id += 1
        if self.backend.member_bytes(problem) > self.backend.arena_bytes or nsteps < 1:
            r.status, r.error, r.finished = -1, "request can never fit the device pool", r.arrival
            self.done.append(r)
        else:
            self.queue.append(r)
        return r

    def admit(self):
        """FIFO admission while slots and arena memory allow.  While other requests
        compute, a request whose staged upload has not arrived yet waits for the next
        round instead of holding the host."""
        n = 0
        while self.queue and len(self.active) < self.backend.max_members:
            r = self.queue[0]
            if self.active and r.staged is not None and not self.backend.ready(r.staged):
                break
            slot = self.backend.admit(r.problem, r.u0 if r.staged is None else r.staged, r.nsteps, r.cfl)
            if slot is None:
                break
            self.queue.popleft()
            r.slot, r.admitted, r.staged, r.steps_done = slot, self.clock(), None, 0
            self.active[slot] = r
            n += 1
        return n

    def _stage(self):
        staged = sum(r.u0.nbytes for r in self.queue if r.staged is not None)
        for i, r in enumerate(self.queue):
            if i >= self.stage_ahead:
                break
            if r.staged is None:
                if staged > 0 and staged + r.u0.nbytes > self.stage_bytes:
                    break
                r.staged = self.backend.stage(r.problem, r.u0)
                staged += r.u0.nbytes

    def _finish(self, r, result):
        r.result = result
        r.finished = self.clock()
        self.done.append(r)

    def collect(self, wait=False):
        """Finish the requests whose results have arrived (all of them with wait)."""
        left = []
        for r, p in self.pending:
            if wait or p.ready():
                res = p.result()
                info = p.info()
                if info is not None:  # retired on the prediction: check what the device did
                    status, steps = info
                    r.steps_done = steps
                    if status:
                        r.status, r.error = status, "non-physical state"
                    elif steps != r.nsteps:
                        r.status, r.error = -2, f"stopped after {steps} of {r.nsteps} steps"
                self._finish(r, res)
            else:
                left.append((r, p))
        self.pending = left

    def round_steps(self):
        """Steps of the next round: fixed, or the fewest an active request still needs."""
        if self.steps_per_round > 0:
            return self.steps_per_round
        need = min(max(r.nsteps - r.steps_done, 1) for r in self.active.values())
        return max(1, min(need, self.max_round_steps))

    def round(self):
        """Admit, advance every admitted request, retire the finished ones.  While the
        round computes, the next queued requests are staged and arrived results are
        collected."""
        self.admit()
        if not self.active:
            self.collect(wait=not self.queue)
            return 0
        k = self.round_steps()
        self.backend.step(k)
        self.rounds += 1
        if self.backend.pipelined:
            finished = 0
            for slot in list(self.active):
                r = self.active[slot]
                r.steps_done = min(r.nsteps, r.steps_done + k)
                if r.steps_done >= r.nsteps:
                    del self.active[slot]
                    self.pending.append((r, self.backend.retire_async(slot, r.problem.shape)))
                    finished += 1
            self.backend.fence()
            self._stage()
            self.collect()
            return finished
        self._stage()
        self.collect()
        done, status, steps = self.backend.poll()
        finished = 0
        for slot, r in self.active.items():
            r.steps_done = int(steps[slot])
        for slot in list(self.active):
            if done[slot] == 1 or status[slot] != 0:
                r = self.active.pop(slot)
                r.status = int(status[slot])
                if r.status:
                    r.error = "non-physical state"
                elif steps[slot] != r.nsteps:
                    r.status, r.error = -2, f"stopped after {steps[slot]} of {r.nsteps} steps"
                res = self.backend.retire(slot, r.problem.shape)
                if isinstance(res, Pending):
                    self.pending.append((r, res))
                else:
                    self._finish(r, res)
                finished += 1
        return finished

    def idle(self):
        return not self.queue and not self.active and not self.pending

    def drain(self):
        while not self.idle():
            self.round()
        return self.done


def latency_stats(requests):
    lat = np.array([r.latency for r in requests if r.status == 0])
    if lat.size == 0:
        return {"count": 0}
    return {"count": int(lat.size), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}


def run_arrivals(server: Server, arrivals, make_request):
    """Drive a server with a timed request stream.

    arrivals: increasing arrival offsets (s) from the start; make_request(i) ->
    (problem, u0, nsteps).  Requests are submitted when the wall clock passes
    their arrival time; the server runs rounds meanwhile and sleeps only when it
    has nothing to do.  Returns (requests, wall seconds from first arrival to
    last completion)."""
    t0 = server.clock()
    pending = deque(range(len(arrivals)))
    reqs = []
    while pending or not server.idle():
        now = server.clock() - t0
        while pending and arrivals[pending[0]] <= now:
            i = pending.popleft()
            p, u0, ns = make_request(i)
            reqs.append(server.submit(p, u0, ns, arrival=t0 + arrivals[i]))
        if server.idle():
            if pending:
                time.sleep(max(0.0, arrivals[pending[0]] - (server.clock() - t0)))
            continue
        server.round()
    end = max(r.finished for r in reqs)
    return reqs, end - t0
