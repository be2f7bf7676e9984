"""Scheduling logic of the continuous-batching server, on the CPU: a fake pool that
steps its members with the oracle, a virtual clock, and the real Server."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12742_amd import serve as S
from paper_2108_12742_amd import workloads as W


class FakeProblem:
    def __init__(self, inst):
        self.inst = inst
        self.nx, self.ny = inst.nx, inst.ny
        self.shape = inst.u0.shape

    def oracle(self):
        return O.Problem(O.EULER1D, nx=self.nx, x_lo=self.inst.x_lo, x_hi=self.inst.x_hi, bc_x=O.TRANSMISSIVE)


class FakePool(S.Backend):
    """Same contract as the HIP pool: slots, an arena budget in bytes, members that stop at
    their own step count; steps with the oracle."""

    def __init__(self, max_members, arena_bytes, clock):
        self.max_members, self.arena_bytes, self.clock = max_members, arena_bytes, clock
        self.used = 0
        self.members = {}
        self.stepped = []

    def member_bytes(self, problem):
        return 3 * 8 * problem.nx * problem.ny * 3

    def admit(self, problem, u0, nsteps, cfl):
        b = self.member_bytes(problem)
        free = [k for k in range(self.max_members) if k not in self.members]
        if not free or self.used + b > self.arena_bytes:
            return None
        self.used += b
        self.members[free[0]] = [problem, u0.copy(), 0, nsteps, cfl, b]
        return free[0]

    def step(self, nsteps):
        self.stepped.append(sorted(self.members))
        for m in self.members.values():
            p, u, k, n, cfl, _ = m
            for _ in range(min(nsteps, n - k)):
                op = p.oracle()
                u = O.step(op, u, O.cfl_dt(op, u, cfl))
                k += 1
            m[1], m[2] = u, k
        self.clock.t += 1.0

    def poll(self):
        done = np.full(self.max_members, -1)
        steps = np.zeros(self.max_members, int)
        for s, m in self.members.items():
            done[s] = int(m[2] >= m[3])
            steps[s] = m[2]
        return done, np.zeros(self.max_members, int), steps

    def retire(self, slot, shape):
        m = self.members.pop(slot)
        self.used -= m[5]
        return m[1]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def _request(seed, n):
    inst = W.riemann_1d(seed, n)
    return FakeProblem(inst), inst.u0


def test_footprint_admission_fifo_and_results():
    clock = Clock()
    small, big = _request(1, 32), _request(2, 64)
    budget = 3 * 8 * 3 * (32 + 64)  # room for one small and one big request at a time
    pool = FakePool(max_members=8, arena_bytes=budget, clock=clock)
    srv = S.Server(pool, steps_per_round=2, clock=clock)
    reqs = [srv.submit(*small, nsteps=4), srv.submit(*big, nsteps=4), srv.submit(*big, nsteps=2),
            srv.submit(*small, nsteps=6)]
    srv.admit()
    assert [r.slot is not None for r in reqs] == [True, True, False, False]  # arena full: FIFO waits
    srv.drain()
    assert all(r.status == 0 for r in reqs)
    # every member of every round fitted the arena; requests 3 and 4 joined while others ran
    assert max(len(s) for s in pool.stepped) == 2
    assert reqs[2].admitted > reqs[1].admitted and reqs[3].admitted >= reqs[2].admitted
    # results do not depend on the mix: each equals its solve alone
    for r, (prob, u0) in zip(reqs, [small, big, big, small]):
        op = prob.oracle()
        u = u0
        for _ in range(r.nsteps):
            u = O.step(op, u, O.cfl_dt(op, u, 0.3))
        np.testing.assert_array_equal(r.result, u)
    st = S.latency_stats(reqs)
    assert st["count"] == 4 and st["p99_s"] >= st["p50_s"] > 0


def test_never_fitting_request_rejected():
    clock = Clock()
    pool = FakePool(max_members=4, arena_bytes=1000, clock=clock)
    srv = S.Server(pool, clock=clock)
    r = srv.submit(*_request(3, 64), nsteps=3)
    assert r.status != 0 and "never fit" in r.error
    assert srv.idle()


def test_slot_limit():
    clock = Clock()
    pool = FakePool(max_members=2, arena_bytes=1 << 30, clock=clock)
    srv = S.Server(pool, clock=clock)
    reqs = [srv.submit(*_request(k, 16), nsteps=1 + k) for k in range(5)]
    srv.admit()
    assert sum(r.slot is not None for r in reqs) == 2
    srv.drain()
    assert all(r.status == 0 and r.finished is not None for r in reqs)
    assert max(len(s) for s in pool.stepped) == 2


class _LateResult(S.Pending):
    def __init__(self, value, clock, at):
        self.value, self.clock, self.at = value, clock, at

    def ready(self):
        return self.clock.t >= self.at

    def result(self):
        return self.value


class AsyncFakePool(FakePool):
    """Stages inputs (a marker the admit checks) and hands back results that arrive two
    rounds after retirement, as the GPU backend's overlapped transfers do."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.staged = 0

    def stage(self, problem, u0):
        self.staged += 1
        return ("staged", u0)

    def admit(self, problem, u0, nsteps, cfl):
        if isinstance(u0, tuple):
            u0 = u0[1]
        return super().admit(problem, u0, nsteps, cfl)

    def retire(self, slot, shape):
        return _LateResult(super().retire(slot, shape), self.clock, self.clock.t + 2.0)


def test_overlapped_transfers():
    """Staged uploads are admitted in FIFO order; a request finishes when its result has
    arrived, and drain waits for the last ones."""
    clock = Clock()
    pool = AsyncFakePool(max_members=2, arena_bytes=1 << 30, clock=clock)
    srv = S.Server(pool, steps_per_round=1, clock=clock, stage_ahead=2)
    reqs = [srv.submit(*_request(10 + k, 16), nsteps=1 + k % 3) for k in range(6)]
    srv.drain()
    assert srv.idle() and not srv.pending
    assert pool.staged >= 4  # requests beyond the first two waited in the queue, staged
    assert [r.admitted for r in reqs] == sorted(r.admitted for r in reqs)
    for r in reqs:
        assert r.status == 0 and r.finished is not None and r.finished >= r.admitted
        op = r.problem.oracle()
        u = r.u0
        for _ in range(r.nsteps):
            u = O.step(op, u, O.cfl_dt(op, u, 0.3))
        np.testing.assert_array_equal(r.result, u)


def test_adaptive_rounds_stop_when_the_first_request_finishes():
    """steps_per_round = 0: each round runs the fewest steps an active request still needs
    (bounded by max_round_steps), so a request retires exactly at the end of a round and
    the queue is admitted then; results equal each request's solve alone."""
    clock = Clock()
    reqs_in = [(_request(11, 24), 7), (_request(12, 24), 3), (_request(13, 24), 12), (_request(14, 24), 5)]
    budget = 3 * 8 * 3 * 24 * 2  # two members at a time
    pool = FakePool(max_members=8, arena_bytes=budget, clock=clock)
    rounds = []
    srv = S.Server(pool, clock=clock, max_round_steps=4)
    orig = pool.step

    def step(n):
        rounds.append(n)
        orig(n)

    pool.step = step
    reqs = [srv.submit(*rq, nsteps=n) for rq, n in reqs_in]
    srv.drain()
    assert all(r.status == 0 for r in reqs)
    # members 7 and 3 start: 3 steps; then 7 (4 left) with 12: 4 steps; 12 (8 left) with 5:
    # 4 (bound), 1 ... every round ends where the closest request ends or at the bound
    assert rounds[0] == 3 and rounds[1] == 4 and max(rounds) <= 4
    assert len(rounds) < sum(rounds)  # fewer host polls than pool steps
    for r, ((prob, u0), n) in zip(reqs, reqs_in):
        op = prob.oracle()
        u = u0
        for _ in range(n):
            u = O.step(op, u, O.cfl_dt(op, u, 0.3))
        np.testing.assert_array_equal(r.result, u)


class _Retired(S.Pending):
    def __init__(self, value, status, steps, clock, at):
        self.value, self.status, self.steps, self.clock, self.at = value, status, steps, clock, at

    def ready(self):
        return self.clock.t >= self.at

    def result(self):
        return self.value

    def info(self):
        return self.status, self.steps


class PipelinedFakePool(FakePool):
    """A pipelined backend: the server never polls; it retires on its own step count and
    learns from the retirement what the member did.  Members whose initial state is
    marked fail after `fail_after` steps (they stop there with a non-zero status, as the
    device does on a non-physical state)."""
    pipelined = True

    def __init__(self, *a, fail_after=None, **k):
        super().__init__(*a, **k)
        self.fail_after = fail_after or {}
        self.fences = 0
        self.status = {}

    def admit(self, problem, u0, nsteps, cfl):
        slot = super().admit(problem, u0, nsteps, cfl)
        if slot is not None:
            self.status[slot] = 0
            key = np.ascontiguousarray(u0).tobytes()
            if key in self.fail_after:
                self.members[slot][3] = self.fail_after[key]   # the device stops it there
                self.status[slot] = 1
        return slot

    def poll(self):
        raise AssertionError("a pipelined server does not poll")

    def retire_async(self, slot, shape):
        steps = self.members[slot][2]
        status = self.status.pop(slot)
        return _Retired(super().retire(slot, shape), status, steps, self.clock, self.clock.t + 1.0)

    def fence(self):
        self.fences += 1


def test_pipelined_rounds_retire_on_the_step_count():
    """Pipelined backend: requests retire right after the round that gives them their last
    step, without polling; a request whose member stopped early on the device reports
    the failure from its retirement; every other result equals its solve alone."""
    clock = Clock()
    reqs_in = [(_request(21, 24), 7), (_request(22, 24), 3), (_request(23, 24), 12), (_request(24, 24), 5),
               (_request(25, 24), 4)]
    bad = reqs_in[2][0][1]
    budget = 3 * 8 * 3 * 24 * 2  # two members at a time
    pool = PipelinedFakePool(max_members=8, arena_bytes=budget, clock=clock,
                             fail_after={np.ascontiguousarray(bad).tobytes(): 2})
    srv = S.Server(pool, clock=clock, max_round_steps=4)
    reqs = [srv.submit(*rq, nsteps=n) for rq, n in reqs_in]
    srv.drain()
    assert srv.idle() and pool.fences == srv.rounds and pool.used == 0
    assert reqs[2].status != 0 and reqs[2].error == "non-physical state" and reqs[2].steps_done == 2
    for k, (r, ((prob, u0), n)) in enumerate(zip(reqs, reqs_in)):
        if k == 2:
            continue
        assert r.status == 0 and r.steps_done == n and r.finished >= r.admitted
        op = prob.oracle()
        u = u0
        for _ in range(n):
            u = O.step(op, u, O.cfl_dt(op, u, 0.3))
        np.testing.assert_array_equal(r.result, u)
    assert [r.admitted for r in reqs] == sorted(r.admitted for r in reqs)


def test_staging_stays_within_its_byte_budget():
    """Queued requests are staged in FIFO order while their states total at most
    stage_bytes (at least one is staged), and admission takes staged uploads only once
    they have arrived, in order."""
    clock = Clock()

    class Staging(FakePool):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.staged_bytes = []
            self.arrived = set()

        def stage(self, problem, u0):
            self.staged_bytes.append(u0.nbytes)
            return ("staged", id(u0), u0)

        def ready(self, staged):
            return staged[1] in self.arrived

        def admit(self, problem, u0, nsteps, cfl):
            if isinstance(u0, tuple):
                u0 = u0[2]
            return super().admit(problem, u0, nsteps, cfl)

    pool = Staging(max_members=2, arena_bytes=1 << 30, clock=clock)
    reqs_in = [_request(30 + k, 32) for k in range(6)]
    one = reqs_in[0][1].nbytes
    srv = S.Server(pool, steps_per_round=1, clock=clock, stage_ahead=64, stage_bytes=2 * one)
    reqs = [srv.submit(*rq, nsteps=2) for rq in reqs_in]
    srv._stage()
    assert pool.staged_bytes == [one, one]          # the budget holds two states
    srv._stage()
    assert len(pool.staged_bytes) == 2              # nothing new while both wait
    srv.admit()
    # an empty pool takes the first even before its upload arrives; with it running,
    # the second waits for its own
    assert reqs[0].slot is not None and reqs[1].slot is None
    pool.arrived.add(reqs[1].staged[1])
    srv.admit()
    assert reqs[1].slot is not None and reqs[2].slot is None  # two slots: full
    srv._stage()
    assert len(pool.staged_bytes) == 4              # the admitted ones left the budget
    srv.drain()
    assert all(r.status == 0 and r.finished is not None for r in reqs)
    assert [r.admitted for r in reqs] == sorted(r.admitted for r in reqs)
