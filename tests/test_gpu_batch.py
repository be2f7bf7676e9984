"""Batched and pooled launches on the GPU: every member's result equals its solve alone
(bitwise: same kernels, same per-member arithmetic), and matches the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12742_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _alone(torch, E, inst, nsteps, cfl=0.3, t_final=1e300):
    plan = E.enoao_plan_create(E.problem_from_instance(inst))
    u = PT.to_dev(torch, inst.u0)
    t, n = E.enoao_solve(plan, u, t_final, cfl=cfl, max_steps=nsteps)
    return u.cpu().numpy(), t, n


def test_batch_1d_members_match_alone_and_oracle():
    torch = PT.torch_cuda()
    E = _E()
    sizes = [128, 5, 63, 64, 300, 1031, 2000, 77]
    insts = [W.riemann_1d(100 + k, n) for k, n in enumerate(sizes)]
    probs = [E.problem_from_instance(i) for i in insts]
    batch = E.enoao_batch_create(probs)
    us = [PT.to_dev(torch, i.u0) for i in insts]
    E.enoao_batch_step(batch, us, 10, 0.3)
    t, steps, status = E.enoao_batch_query(batch)
    assert (steps == 10).all() and (status == 0).all()
    for k, inst in enumerate(insts):
        ref, ta, na = _alone(torch, E, inst, 10)
        assert torch.equal(us[k].cpu(), torch.from_numpy(ref)), f"member {k} (N={sizes[k]}) differs from alone"
        assert t[k] == ta
    for k in (0, 4):
        ur, _, _, _, _ = PT.lockstep_solve(torch, E, probs[k], insts[k].u0, 1e300, cfl=0.3, max_steps=10,
                                           what=f"member {k}")
        assert np.array_equal(us[k].cpu().numpy(), ur)


def test_batch_continues_across_calls_and_stops_at_t_final():
    torch = PT.torch_cuda()
    E = _E()
    insts = [W.riemann_1d(7, 200), W.riemann_1d(8, 500), W.advection(3, 150)]
    insts = insts[:2]
    probs = [E.problem_from_instance(i) for i in insts]
    batch = E.enoao_batch_create(probs)
    us = [PT.to_dev(torch, i.u0) for i in insts]
    tf = [0.002, 0.05]
    E.enoao_batch_step(batch, us, 6, 0.3, t_final=tf)
    E.enoao_batch_step(batch, us, 6, 0.3, t_final=tf)
    t, steps, status = E.enoao_batch_query(batch)
    for k, inst in enumerate(insts):
        ref, ta, na = _alone(torch, E, inst, 12, t_final=tf[k])
        assert steps[k] == na and t[k] == ta
        assert torch.equal(us[k].cpu(), torch.from_numpy(ref))
    assert t[0] == tf[0] and steps[0] < 12   # the first member reached its end time early


def test_batch_2d_members_and_launch_shape():
    torch = PT.torch_cuda()
    E = _E()
    insts = [W.quadrants(1, 40, 37), W.quadrants(3, 16, 15), W.quadrants(5, 70, 31), W.quadrants(6, 5, 9)]
    probs = [E.problem_from_instance(i) for i in insts]
    outs = []
    # uniform shapes, then a shape per kernel kind (x stages 1..3, y stages 1..3)
    for wg, kinds in ((0, None), (1, None), (3, (6, 1, 16, 2, 4, 3))):
        batch = E.enoao_batch_create(probs)
        E.enoao_batch_set_launch(batch, wg)
        if kinds:
            E.enoao_batch_set_launch_kinds(batch, kinds)
        us = [PT.to_dev(torch, i.u0) for i in insts]
        E.enoao_batch_step(batch, us, 4, 0.3)
        outs.append([u.cpu() for u in us])
    for k, inst in enumerate(insts):
        ref, _, _ = _alone(torch, E, inst, 4)
        assert torch.equal(outs[0][k], torch.from_numpy(ref))
        assert torch.equal(outs[1][k], outs[0][k])
        assert torch.equal(outs[2][k], outs[0][k])
    for bad in ((1,) * 7, (-1,), (65, 2)):
        with pytest.raises(E.EnoaoError):
            E.enoao_batch_set_launch_kinds(batch, bad)


def test_pool_members_join_and_leave():
    """Members admitted at different rounds, retired when done: each equals its solve alone."""
    torch = PT.torch_cuda()
    E = _E()
    insts = [W.quadrants(s, n, n) for s, n in ((1, 48), (2, 33), (3, 64), (5, 20), (1, 40))]
    nsteps = [5, 3, 4, 6, 2]
    like = E.problem_from_instance(insts[0])
    bytes_per = [E.enoao_pool_member_bytes(E.problem_from_instance(i)) for i in insts]
    pool = E.enoao_pool_create(like, 3, sum(sorted(bytes_per)[-2:]) + 4096)
    results, slots, pending = {}, {}, list(range(len(insts)))
    rounds = 0
    while pending or slots:
        while pending:  # FIFO admission while there is room
            k = pending[0]
            s = E.enoao_pool_admit(pool, E.problem_from_instance(insts[k]), insts[k].u0, max_steps=nsteps[k])
            if s is None:
                break
            slots[s] = k
            pending.pop(0)
        E.enoao_pool_step(pool, 1)
        rounds += 1
        done, status, steps, _ = E.enoao_pool_poll(pool)
        for s in list(slots):
            assert status[s] == 0
            if done[s] == 1:
                k = slots.pop(s)
                assert steps[s] == nsteps[k]
                results[k] = E.enoao_pool_retire(pool, s, shape=insts[k].u0.shape)
        assert rounds < 100
    for k, inst in enumerate(insts):
        ref, _, _ = _alone(torch, E, inst, nsteps[k])
        np.testing.assert_array_equal(results[k], ref)
    assert E.enoao_pool_usage(pool)[0] == 0


def test_pool_launch_shape_and_short_chunks():
    """A pool's grid covers the machine 24 times (workgroups per CU) and each launch
    shares its tiles among as many workgroups as give 16 tiles each, at least the
    occupancy.  24 members of about 512^2 hold more tiles than 16 per resident
    workgroup in both sweeps, so the short-chunk path runs; at the occupancy
    (enoao_pool_set_launch 0) every launch shares its tiles among the resident
    workgroups only.  Both give every member bitwise its solve alone."""
    torch = PT.torch_cuda()
    E = _E()
    sizes = [(512, 512)] * 20 + [(509, 515), (497, 520), (530, 480), (512, 500)]
    insts = [W.quadrants(k + 1, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    probs = [E.problem_from_instance(i) for i in insts]
    arena = sum(E.enoao_pool_member_bytes(p) for p in probs) + (1 << 20)
    nsteps = 3
    results = {}
    for wg in (None, 0):
        pool = E.enoao_pool_create(probs[0], len(insts), arena)
        if wg is not None:
            E.enoao_pool_set_launch(pool, wg)
        slots = [E.enoao_pool_admit(pool, p, PT.to_dev(torch, i.u0), max_steps=nsteps) for p, i in zip(probs, insts)]
        assert None not in slots
        E.enoao_pool_step(pool, nsteps)
        done, status, steps, _ = E.enoao_pool_poll(pool)
        for s in slots:
            assert status[s] == 0 and steps[s] == nsteps
        results[wg] = [E.enoao_pool_retire(pool, s, shape=i.u0.shape) for s, i in zip(slots, insts)]
        E.enoao_pool_destroy(pool)
    for a, b in zip(results[None], results[0]):
        np.testing.assert_array_equal(a, b)
    for k in (0, 20, 21, 23):
        ref, _, _ = _alone(torch, E, insts[k], nsteps)
        np.testing.assert_array_equal(results[None][k], ref)


def test_pool_retire_async_reuses_space_in_stream_order():
    """enoao_pool_retire_async: no host synchronisation between rounds.  Members are
    retired on their own step count right after the step call that finished them, the
    next member is admitted into the freed arena space at once (its copy follows the
    retirement's on the stream), and the host reads nothing until the end: every result
    equals its solve alone and every progress record says status 0 and its step count."""
    torch = PT.torch_cuda()
    E = _E()
    insts = [W.quadrants(s, n, n + 3) for s, n in ((1, 45), (2, 33), (3, 61), (5, 20), (1, 40), (4, 52))]
    nsteps = [5, 3, 4, 6, 2, 3]
    like = E.problem_from_instance(insts[0])
    bytes_per = [E.enoao_pool_member_bytes(E.problem_from_instance(i)) for i in insts]
    pool = E.enoao_pool_create(like, 2, sum(sorted(bytes_per)[-2:]) + 4096)
    outs = {k: torch.empty(i.u0.shape, dtype=torch.float64, device="cuda") for k, i in enumerate(insts)}
    infos = {k: torch.empty(4, dtype=torch.float64, device="cuda") for k in range(len(insts))}
    slots, left, pending, rounds = {}, {}, list(range(len(insts))), 0
    while pending or slots:
        while pending:
            k = pending[0]
            s = E.enoao_pool_admit(pool, E.problem_from_instance(insts[k]), PT.to_dev(torch, insts[k].u0),
                                   max_steps=nsteps[k])
            if s is None:
                break
            slots[s], left[s] = k, nsteps[k]
            pending.pop(0)
        n = min(left.values())
        E.enoao_pool_step(pool, n)
        rounds += 1
        for s in list(slots):
            left[s] -= n
            if left[s] == 0:
                k = slots.pop(s)
                del left[s]
                E.enoao_pool_retire_async(pool, s, out=outs[k], info=infos[k])
        assert rounds < 100
    torch.cuda.synchronize()
    for k, inst in enumerate(insts):
        ref, _, _ = _alone(torch, E, inst, nsteps[k])
        np.testing.assert_array_equal(outs[k].cpu().numpy(), ref)
        done, status, steps, t = infos[k].cpu().numpy()
        # (done is set by the step control of the step after the last one)
        assert done in (0, 1) and status == 0 and steps == nsteps[k] and t > 0
    assert E.enoao_pool_usage(pool)[0] == 0


def test_server_on_gpu_pool():
    PT.torch_cuda()
    E = _E()
    from paper_2108_12742_amd import serve as S
    insts = [W.quadrants(s % 3 + 1, n, n) for s, n in enumerate((32, 48, 40, 24, 56, 32))]
    like = E.problem_from_instance(insts[0])
    arena = 2 * E.enoao_pool_member_bytes(E.problem_from_instance(insts[4])) + 4096
    srv = S.Server(S.GpuPoolBackend(like, max_members=4, arena_bytes=arena), steps_per_round=2)
    reqs = [srv.submit(E.problem_from_instance(i), i.u0, nsteps=3 + k % 3) for k, i in enumerate(insts)]
    srv.drain()
    torch = PT.torch_cuda()
    for r, inst in zip(reqs, insts):
        assert r.status == 0, r.error
        ref, _, _ = _alone(torch, E, inst, r.nsteps)
        np.testing.assert_array_equal(r.result, ref)
    st = S.latency_stats(reqs)
    assert st["count"] == len(insts)


def test_autotuner_restores_states_and_picks_a_candidate(tmp_path, monkeypatch):
    """The tuner times every (workgroups per CU, y strip width) candidate on the caller's
    batch, leaves the states as they were, and its choice gives the same results."""
    torch = PT.torch_cuda()
    E = _E()
    from paper_2108_12742_amd import tune as T
    monkeypatch.setenv("ENOAO_TUNE_CACHE", str(tmp_path / "tune.json"))
    insts = [W.quadrants(1, 80, 70), W.quadrants(3, 50, 90)]
    probs = [E.problem_from_instance(i) for i in insts]
    us = [PT.to_dev(torch, i.u0) for i in insts]
    (w, yw), timing = T.tune_batch(probs, us, steps=2, candidates=(0, 2))
    assert set(timing) == {"0/8", "2/8", "0/4", "2/4"} and (w, yw) in {(0, 8), (2, 8), (0, 4), (2, 4)}
    for u, i in zip(us, insts):
        assert torch.equal(u.cpu(), torch.from_numpy(i.u0))
    assert T.tune_batch(probs, us, steps=2, candidates=(0, 2))[0] == (w, yw)  # cached
    outs = []
    for shape in ((w, yw), (0, 8)):
        b = E.enoao_batch_create(probs)
        E.enoao_batch_set_launch(b, shape[0])
        E.enoao_batch_set_tiles(b, shape[1])
        vs = [PT.to_dev(torch, i.u0) for i in insts]
        E.enoao_batch_step(b, vs, 3, 0.3)
        outs.append([v.cpu() for v in vs])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    # a shape per kernel kind on top of the uniform one: states restored, and the
    # shapes (if kept) give the same results
    kinds, info = T.tune_kinds(probs, us, w, yw, steps=2, candidates=(2, 4), rounds=1)
    tried = {k.split("=")[0] for k in info["trials_ms_per_step"]}
    assert tried == set(T.KINDS)
    assert kinds is None or (len(kinds) == 6 and set(kinds) <= {0, 2, 4})
    for u, i in zip(us, insts):
        assert torch.equal(u.cpu(), torch.from_numpy(i.u0))
    b = E.enoao_batch_create(probs)
    E.enoao_batch_set_launch(b, w)
    E.enoao_batch_set_tiles(b, yw)
    E.enoao_batch_set_launch_kinds(b, info["shapes"])
    vs = [PT.to_dev(torch, i.u0) for i in insts]
    E.enoao_batch_step(b, vs, 3, 0.3)
    for v, a in zip(vs, outs[0]):
        assert torch.equal(v.cpu(), a)


@pytest.mark.slow
def test_c3_full_batch_sampled_members():
    """The batched workload at its full size (512 seeded 1D Euler members, N from 128 to
    16384, sum of N about 1.9M) in one batch at the default launch shape: every member
    takes its 5 CFL steps without a non-physical state, and sampled members (the
    smallest, the largest and six more) equal their solve alone, whose every step
    matches the oracle (tests/parity.py lockstep_solve)."""
    torch = PT.torch_cuda()
    E = _E()
    insts = W.batch_1d(0, 512)
    probs = [E.problem_from_instance(i) for i in insts]
    batch = E.enoao_batch_create(probs)
    us = [PT.to_dev(torch, i.u0) for i in insts]
    E.enoao_batch_step(batch, us, 5, 0.3)
    t, steps, status = E.enoao_batch_query(batch)
    assert (steps == 5).all() and (status == 0).all()
    sizes = np.array([i.nx for i in insts])
    rng = np.random.default_rng(5)
    pick = sorted({int(sizes.argmin()), int(sizes.argmax())} | {int(k) for k in rng.choice(512, 6, replace=False)})
    for k in pick:
        ur, nr, tr, _, _ = PT.lockstep_solve(torch, E, probs[k], insts[k].u0, 1e300, cfl=0.3, max_steps=5,
                                             what=f"member {k} (N={sizes[k]})")
        assert nr == 5 and t[k] == tr
        assert np.array_equal(us[k].cpu().numpy(), ur), f"member {k} differs from its solve alone"


@pytest.mark.slow
def test_c4_served_workload_sampled_requests():
    """The served workload at its full size (200 seeded requests, N x N with N from 128 to
    1024, 50 steps each) submitted at once to the server with the benchmark's pool: every
    request succeeds; sampled requests equal their solve alone bitwise, and every step
    of the smallest matches the oracle (tests/parity.py lockstep_solve)."""
    torch = PT.torch_cuda()
    E = _E()
    from paper_2108_12742_amd import serve as S
    _, sizes, _ = W.arrivals(1, 200, 1.0)
    data = [W.quadrants(W.QUADRANT_BENCH_SEED, int(n)) for n in sizes]
    probs = [E.problem_from_instance(d) for d in data]
    srv = S.Server(S.GpuPoolBackend(probs[0], max_members=256, arena_bytes=4 << 30), steps_per_round=1)
    reqs = [srv.submit(p, d.u0, 50) for p, d in zip(probs, data)]
    srv.drain()
    assert all(r.status == 0 for r in reqs), [r.error for r in reqs if r.status]
    small = int(np.argmin(sizes))
    rng = np.random.default_rng(9)
    for k in sorted({small, int(np.argmax(sizes))} | {int(k) for k in rng.choice(200, 3, replace=False)}):
        ref, _, n = _alone(torch, E, data[k], 50)
        assert n == 50
        np.testing.assert_array_equal(reqs[k].result, ref)
    ur, nr, _, _, _ = PT.lockstep_solve(torch, E, probs[small], data[small].u0, 1e300, cfl=0.3, max_steps=50,
                                        what=f"request {small} (N={sizes[small]})")
    assert nr == 50
    np.testing.assert_array_equal(reqs[small].result, ur)


def test_pool_1d_order7_members():
    """A pool of 1D Euler members at order 7 (sizes from 7 to 2000 nodes) admitted as
    room frees up: each equals its solve alone bitwise."""
    torch = PT.torch_cuda()
    E = _E()
    sizes = [2000, 7, 333, 64, 1031, 150]
    insts = [W.riemann_1d(200 + k, n) for k, n in enumerate(sizes)]
    probs = [E.problem_from_instance(i, order=7) for i in insts]
    nsteps = [4, 6, 3, 5, 2, 4]
    bytes_per = [E.enoao_pool_member_bytes(p) for p in probs]
    pool = E.enoao_pool_create(probs[0], 3, sum(sorted(bytes_per)[-2:]) + 4096)
    results, slots, pending = {}, {}, list(range(len(insts)))
    rounds = 0
    while pending or slots:
        while pending:
            k = pending[0]
            s = E.enoao_pool_admit(pool, probs[k], insts[k].u0, max_steps=nsteps[k])
            if s is None:
                break
            slots[s] = k
            pending.pop(0)
        E.enoao_pool_step(pool, 1)
        rounds += 1
        done, status, steps, _ = E.enoao_pool_poll(pool)
        for s in list(slots):
            assert status[s] == 0
            if done[s] == 1:
                k = slots.pop(s)
                assert steps[s] == nsteps[k]
                results[k] = E.enoao_pool_retire(pool, s, shape=insts[k].u0.shape)
        assert rounds < 100
    for k, inst in enumerate(insts):
        plan = E.enoao_plan_create(probs[k])
        u = PT.to_dev(torch, inst.u0)
        E.enoao_solve(plan, u, 1e300, cfl=0.3, max_steps=nsteps[k])
        np.testing.assert_array_equal(results[k], u.cpu().numpy())


def _poisoned(inst, k=40):
    """the instance with a negative pressure at one node (E below the kinetic energy)"""
    u0 = inst.u0.copy()
    nc = u0.shape[0]
    flat = u0.reshape(nc, -1)
    j = min(k, flat.shape[1] - 1)
    kin = 0.5 * sum(flat[c, j] ** 2 for c in range(1, nc - 1)) / flat[0, j]
    flat[nc - 1, j] = 0.5 * kin
    return u0


def test_failure_isolation():
    """One member with a non-physical state (p < 0 at one node) in a batch, a pool and the
    server: only that member or request reports the non-physical status; every other
    member equals its solve alone bitwise."""
    torch = PT.torch_cuda()
    E = _E()
    from paper_2108_12742_amd import serve as S
    insts = [W.riemann_1d(300 + k, n) for k, n in enumerate([300, 1200, 77, 1600])]
    bad = 1
    u0s = [i.u0 if k != bad else _poisoned(i) for k, i in enumerate(insts)]
    probs = [E.problem_from_instance(i) for i in insts]
    alone = [_alone(torch, E, i, 8)[0] for i in insts]
    # batch (streaming kernels and, for members that fit, the LDS-resident solver)
    for resident in (True, False):
        E.enoao_set_resident(resident)
        try:
            batch = E.enoao_batch_create(probs)
            us = [PT.to_dev(torch, u) for u in u0s]
            E.enoao_batch_step(batch, us, 8, 0.3)
            t, steps, status = E.enoao_batch_query(batch)
        finally:
            E.enoao_set_resident(True)
        assert status[bad] != 0 and all(status[k] == 0 for k in range(4) if k != bad)
        for k in range(4):
            if k != bad:
                assert steps[k] == 8 and np.array_equal(us[k].cpu().numpy(), alone[k]), (resident, k)
    # pool
    pool = E.enoao_pool_create(probs[0], 8, 64 << 20)
    slots = [E.enoao_pool_admit(pool, p, u, max_steps=8) for p, u in zip(probs, u0s)]
    for _ in range(10):
        E.enoao_pool_step(pool, 1)
    done, status, steps, _ = E.enoao_pool_poll(pool)
    for k, s in enumerate(slots):
        res = E.enoao_pool_retire(pool, s, shape=insts[k].u0.shape)
        if k == bad:
            assert status[s] != 0
        else:
            assert status[s] == 0 and steps[s] == 8 and np.array_equal(res, alone[k])
    # server on a 2D pool: the poisoned request fails, the others are served
    q = [W.quadrants(1, 70, 60), W.quadrants(3, 96, 96), W.quadrants(5, 40, 33)]
    qp = [E.problem_from_instance(d) for d in q]
    srv = S.Server(S.GpuPoolBackend(qp[0], max_members=4, arena_bytes=64 << 20))
    reqs = [srv.submit(p, d.u0 if k != 1 else _poisoned(d), 6) for k, (p, d) in enumerate(zip(qp, q))]
    srv.drain()
    assert reqs[1].status != 0 and reqs[1].error
    for k in (0, 2):
        assert reqs[k].status == 0
        np.testing.assert_array_equal(reqs[k].result, _alone(torch, E, q[k], 6)[0])


def test_pool_retire_checks_the_member_shape():
    """The binding refuses an output whose shape is not the admitted member's (the
    library copies the whole state)."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.riemann_1d(7, 200)
    p = E.problem_from_instance(inst)
    pool = E.enoao_pool_create(p, 2, 16 << 20)
    s = E.enoao_pool_admit(pool, p, inst.u0, max_steps=1)
    with pytest.raises(ValueError):
        E.enoao_pool_retire(pool, s, shape=(3, 1, 100))
    with pytest.raises(ValueError):
        E.enoao_pool_retire(pool, s, out=torch.empty((3, 1, 100), dtype=torch.float64, device="cuda"))
    out = E.enoao_pool_retire(pool, s, shape=(3, 1, 200))
    np.testing.assert_array_equal(out, inst.u0)
    with pytest.raises(ValueError):
        E.enoao_pool_retire(pool, s, shape=(3, 1, 200))
