"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs, at every cell (tests/parity.py: the oracle replays the GPU's stencil
choices at near ties, and any choice outside the oracle's tie set fails).  Sizes span
several tiles and ragged tails (x segments hold 63 cells, y tiles 32 x 8 cells), plus
the degenerate sizes below one tile; both reconstruction variables of the Euler
systems."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12742_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _adv_case(n, order=5, jumps=False, a=1.0):
    inst = W.advection(n % 7, n)
    u = inst.u0.copy()
    if jumps:
        x = W.nodes(-1.0, 1.0, n)
        u[0, 0] += np.where((x > -0.45) & (x < 0.1), 0.8, 0.0) - np.where(x > 0.6, 0.3, 0.0)
    inst.u0 = u
    inst.adv_speed = a
    return inst, order


def _euler1d_case(n, order=5, bc="transmissive", seed=None, recon="characteristic"):
    inst = W.riemann_1d(n if seed is None else seed, n)
    inst.bc_x = bc
    inst.meta["recon"] = recon
    return inst, order


def _euler2d_case(nx, ny, order=5, bc="periodic", seed=None, recon="characteristic"):
    inst = W.quadrants(nx + 3 * ny if seed is None else seed, nx, ny)
    inst.bc_x = inst.bc_y = bc
    inst.meta["recon"] = recon
    return inst, order


CASES = (
    [("adv", _adv_case, (n,), {}) for n in (1, 5, 63, 64, 127, 200)]
    + [("adv-jumps", _adv_case, (n,), {"jumps": True}) for n in (131, 257)]
    + [("adv-left", _adv_case, (150,), {"jumps": True, "a": -0.7})]
    + [("adv7", _adv_case, (190,), {"order": 7, "jumps": True})]
    + [("e1", _euler1d_case, (n,), {}) for n in (3, 8, 63, 126, 300)]
    + [("e1-periodic", _euler1d_case, (n,), {"bc": "periodic"}) for n in (64, 255)]
    + [("e1-o7", _euler1d_case, (211,), {"order": 7})]
    + [("e2", _euler2d_case, (40, 37), {}), ("e2", _euler2d_case, (16, 15), {}),
       ("e2-tr", _euler2d_case, (70, 31), {"bc": "transmissive"}), ("e2", _euler2d_case, (5, 9), {}),
       ("e2-o7", _euler2d_case, (33, 29), {"order": 7})]
    + [("e1-comp", _euler1d_case, (n,), {"recon": "component"}) for n in (63, 300)]
    + [("e1-comp-o7", _euler1d_case, (211,), {"recon": "component", "order": 7})]
    + [("e2-comp", _euler2d_case, (40, 37), {"recon": "component"}),
       ("e2-comp-tr", _euler2d_case, (70, 31), {"recon": "component", "bc": "transmissive"}),
       ("e2-comp-o7", _euler2d_case, (33, 29), {"recon": "component", "order": 7})]
)
IDS = [f"{c[0]}-{'x'.join(map(str, c[2]))}" for c in CASES]


def _setup(case, record=True):
    _, fn, args, kw = case
    inst, order = fn(*args, **kw)
    E = _E()
    ep = E.problem_from_instance(inst, order=order, record_selection=record,
                                 recon_vars=inst.meta.get("recon", "characteristic"))
    return inst, ep, PT.oracle_problem(ep)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_rhs_matches_oracle(case):
    torch = PT.torch_cuda()
    E = _E()
    inst, ep, op = _setup(case)
    print(f"rhs case {IDS[CASES.index(case)]}", flush=True)
    plan = E.enoao_plan_create(ep)
    u = PT.to_dev(torch, inst.u0)
    L = torch.full_like(u, float("nan"))
    E.enoao_rhs(plan, u, L)
    sel = E.enoao_get_selection(plan)
    torch.cuda.synchronize()
    PT.check_rhs(op, inst.u0, L.cpu().numpy(), sel)
    assert torch.equal(u.cpu(), torch.from_numpy(inst.u0)), "rhs must not modify u"


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_step_matches_oracle(case):
    torch = PT.torch_cuda()
    E = _E()
    inst, ep, op = _setup(case, record=False)
    _, ep_rec, _ = _setup(case, record=True)
    print(f"step case {IDS[CASES.index(case)]}", flush=True)
    plan = E.enoao_plan_create(ep)
    dt = 0.5 * O.cfl_dt(op, inst.u0, 0.3)
    u = PT.to_dev(torch, inst.u0)
    E.enoao_step(plan, u, dt)
    torch.cuda.synchronize()
    E.enoao_plan_check(plan)
    # the recording kernels give bitwise the same step, with the three stage records
    got, recs = PT.gpu_step_recorded(torch, E, E.enoao_plan_create(ep_rec), inst.u0, dt)
    assert np.array_equal(got, u.cpu().numpy())
    PT.check_step(op, inst.u0, dt, got, recs)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c0_solve_matches_oracle(seed):
    """The smooth advection workload end to end: N = 200, CFL 0.5, 400 steps to t = 2,
    every step against the oracle; the oracle's own run takes the same 400 steps."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.advection(seed, 200)
    ep = E.problem_from_instance(inst)
    _, n, t, _, _ = PT.lockstep_solve(torch, E, ep, inst.u0, 2.0, cfl=0.5, what=f"C0 seed {seed}")
    _, tr, nr = O.solve(PT.oracle_problem(ep), inst.u0, 2.0, cfl=0.5)
    assert (t, n) == (tr, nr) == (2.0, 400)


@pytest.mark.parametrize("order", [5, 7])
def test_convergence_row_on_gpu(order):
    """The paper's convergence test at dx = 1/20 and 1/30 with the GPU solver (fixed dt)."""
    torch = PT.torch_cuda()
    E = _E()
    printed = {(5, 20): (2.47e-5, 6.23e-5), (5, 30): (1.30e-6, 3.04e-6),
               (7, 20): (3.68e-8, 5.89e-8), (7, 30): (2.17e-9, 3.46e-9)}
    for inv in (20, 30):
        n = 2 * inv
        x = W.nodes(-1.0, 1.0, n)
        u0 = np.sin(np.pi * x).reshape(1, 1, n)
        ep = E.make_problem("advection", n, order=order)
        dtf = (1.0 / inv) ** (order / 3.0)
        g, steps, t, _, _ = PT.lockstep_solve(torch, E, ep, u0, 2.0, dt_fixed=dtf, what=f"1/{inv}")
        _, tr, nr = O.solve(PT.oracle_problem(ep), u0, 2.0, dt_fixed=dtf)
        assert (t, steps) == (tr, nr)
        e = np.abs(g[0, 0] - u0[0, 0])
        l1, li = np.append(e, e[0]).mean(), e.max()
        p1, pi = printed[(order, inv)]
        tol = 0.1 if (order, inv) == (5, 20) else 0.02
        assert abs(l1 / p1 - 1) < tol and abs(li / pi - 1) < tol, (l1, li)


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_c1_full_solve_matches_oracle():
    """The 1D Euler workload at its stated size and end time (N = 2000, seeded Riemann
    data with the density perturbation, transmissive ends, CFL 0.3, t = 0.2), four seeds:
    every one of the several thousand steps against the oracle (same dt, same clipping,
    every cell at 1e-12 with the GPU's picks replayed at near ties), and the one-call
    device loop bitwise equal to the stepped run."""
    torch = PT.torch_cuda()
    E = _E()
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(PT.workers()) as pool:
        for seed in range(4):
            inst = W.riemann_1d(seed, 2000)
            ep = E.problem_from_instance(inst)
            print(f"C1 seed {seed}: stepping N = 2000 to t = 0.2", flush=True)
            _, n, t, flagged, alt = PT.lockstep_solve(torch, E, ep, inst.u0, 0.2, cfl=0.3, what=f"C1 seed {seed}",
                                                      pool=pool)
            print(f"C1 seed {seed}: {n} steps, {flagged} flagged face sides, {alt} GPU picks of another "
                  f"tie candidate", flush=True)
            assert t == 0.2 and n > 1000


def test_euler1d_solve_matches_oracle():
    """Device-side CFL step control and graph replay against the oracle's time loop."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.riemann_1d(1, 400)
    ep = E.problem_from_instance(inst)
    _, n, t, _, _ = PT.lockstep_solve(torch, E, ep, inst.u0, 0.004, cfl=0.3, what="riemann N = 400")
    _, tr, nr = O.solve(PT.oracle_problem(ep), inst.u0, 0.004, cfl=0.3)
    assert n == nr and t == tr == 0.004


@pytest.mark.parametrize("recon", ["characteristic", "component"])
def test_euler2d_solve_matches_oracle(recon):
    torch = PT.torch_cuda()
    E = _E()
    inst = W.quadrants(11, 48, 40)
    ep = E.problem_from_instance(inst, recon_vars=recon)
    _, n, t, _, _ = PT.lockstep_solve(torch, E, ep, inst.u0, 1.0, cfl=0.3, max_steps=6, what="quadrants 48 x 40")
    _, tr, nr = O.solve(PT.oracle_problem(ep), inst.u0, 1.0, cfl=0.3, max_steps=6)
    assert n == nr == 6 and abs(t / tr - 1) <= 1e-14


def test_launch_shape_invariance():
    """Results do not depend on the persistent grid size (catches LDS/halo races)."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.quadrants(3, 100, 90)
    ep = E.problem_from_instance(inst)
    outs = []
    try:
        for wg in (0, 1, 3):
            E.enoao_set_launch(wg)
            plan = E.enoao_plan_create(ep)
            u = PT.to_dev(torch, inst.u0)
            E.enoao_solve(plan, u, 1.0, cfl=0.3, max_steps=3)
            outs.append(u.cpu())
    finally:
        E.enoao_set_launch(0)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


@pytest.mark.parametrize("order", [5, 7])
def test_multi_tile_walks(order):
    """A grid large enough that every workgroup walks several tiles of a strip (x
    segments and y tiles), with walks that start mid-column and cross column groups:
    L with selections and one step match the oracle, for persistent launch shapes and
    y tile widths that cut the walks differently (bitwise equal to each other)."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.quadrants(7, 640, 403)
    print(f"multi-tile walks, order {order}, 640 x 403", flush=True)
    ep = E.problem_from_instance(inst, order=order, record_selection=True)
    op = PT.oracle_problem(ep)
    dt = 0.5 * O.cfl_dt(op, inst.u0, 0.3)
    steps = []
    try:
        for wg, yw in ((1, 8), (2, 8), (1, 4)):
            E.enoao_set_launch(wg)
            plan = E.enoao_plan_create(ep)
            E.enoao_plan_set_tiles(plan, yw)
            u = PT.to_dev(torch, inst.u0)
            L = torch.empty_like(u)
            E.enoao_rhs(plan, u, L)
            sel = E.enoao_get_selection(plan)
            PT.check_rhs(op, inst.u0, L.cpu().numpy(), sel, what=f"L (wg {wg}, y strips {yw})")
            E.enoao_step(plan, u, dt)
            recs = E.enoao_get_step_selection(plan)
            steps.append(u.cpu())
            PT.check_step(op, inst.u0, dt, steps[-1].numpy(), recs, what=f"u (wg {wg}, y strips {yw})")
    finally:
        E.enoao_set_launch(0)
    assert torch.equal(steps[0], steps[1]) and torch.equal(steps[0], steps[2])


def test_nonphysical_state_reported():
    torch = PT.torch_cuda()
    E = _E()
    inst = W.riemann_1d(2, 128)
    u0 = inst.u0.copy()
    u0[2, 0, 40] = 0.5 * u0[1, 0, 40] ** 2 / u0[0, 0, 40] * 0.5  # E below kinetic energy: p < 0
    plan = E.enoao_plan_create(E.problem_from_instance(inst))
    u = PT.to_dev(torch, u0)
    with pytest.raises(E.EnoaoError) as ei:
        E.enoao_solve(plan, u, 0.01, cfl=0.3)
    assert ei.value.status == E.ENONPHYSICAL
    # the device flag stays set until a check reports it once and clears it
    with pytest.raises(E.EnoaoError) as ei:
        E.enoao_plan_check(plan)
    assert ei.value.status == E.ENONPHYSICAL
    E.enoao_plan_check(plan)


def test_invalid_arguments():
    PT.torch_cuda()
    E = _E()
    bad = E.make_problem("euler1d", 10, order=6)
    with pytest.raises(E.EnoaoError):
        E.enoao_plan_create(bad)
    bad = E.make_problem("euler1d", 10, ny=3)
    with pytest.raises(E.EnoaoError):
        E.enoao_plan_create(bad)


@pytest.mark.slow
def test_c2_full_size_rhs():
    """The 2D Euler workload at its full size (2048^2, periodic, quadrant data): one
    evaluation of L against the oracle, with the launch configuration of the benchmark."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, 2048)
    ep = E.problem_from_instance(inst, record_selection=True)
    op = PT.oracle_problem(ep)
    plan = E.enoao_plan_create(ep)
    u = PT.to_dev(torch, inst.u0)
    L = torch.empty_like(u)
    E.enoao_rhs(plan, u, L)
    sel = E.enoao_get_selection(plan)
    print("oracle rhs at 2048^2 ...", flush=True)
    flagged, alt = PT.check_rhs(op, inst.u0, L.cpu().numpy(), sel)
    print(f"{flagged} flagged face sides, {alt} GPU picks of another tie candidate", flush=True)


@pytest.mark.slow
@pytest.mark.parametrize("order", [5, 7])
def test_c2_full_size_solve_step(order):
    """The 2D Euler workload at its full size (2048^2, quadrant data, the benchmark's seed):
    one CFL-controlled SSP-RK3 step through enoao_solve -- the captured graph of stage
    kernels without selection record that the benchmark times, at the default launch
    shape -- against the oracle's time loop; then the same step at other launch shapes
    (resident workgroups per CU and y strip width; 3 per CU at the order's default
    width, the benchmark's usual tuned shape; a shape per kernel kind) and through the
    recording kernels, bitwise equal; the oracle's step from the same state replays the
    recorded choices at near ties and matches every cell."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.quadrants(W.QUADRANT_BENCH_SEED, 2048)
    ep = E.problem_from_instance(inst, order=order)
    op = PT.oracle_problem(ep)
    plan = E.enoao_plan_create(ep)
    u = PT.to_dev(torch, inst.u0)
    t, n = E.enoao_solve(plan, u, 1e30, cfl=0.3, max_steps=1)
    E.enoao_plan_check(plan)
    # another launch shape, the one the benchmark's tuner usually picks (3 per CU), and
    # a shape per kernel kind as the tuner may add to it
    for wg, yw, kinds in ((2, 4 if order == 5 else 8, None), (3, 0, None), (3, 0, (6, 6, 6, 2, 3, 3))):
        other = E.enoao_plan_create(ep)
        E.enoao_plan_set_launch(other, wg)
        E.enoao_plan_set_tiles(other, yw)
        if kinds:
            E.enoao_plan_set_launch_kinds(other, kinds)
        u2 = PT.to_dev(torch, inst.u0)
        E.enoao_solve(other, u2, 1e30, cfl=0.3, max_steps=1)
        torch.cuda.synchronize()
        assert torch.equal(u, u2), f"launch shape {wg}/{yw} changed the result"
        del u2, other
    rec_ep = E.problem_from_instance(inst, order=order, record_selection=True)
    rec = E.enoao_plan_create(rec_ep)
    u3 = PT.to_dev(torch, inst.u0)
    t3, n3 = E.enoao_solve(rec, u3, 1e30, cfl=0.3, max_steps=1)
    assert (t3, n3) == (t, n) and torch.equal(u, u3), "the recording kernels changed the result"
    recs = E.enoao_get_step_selection(rec)
    del u3, rec
    print(f"oracle step at 2048^2, order {order} ...", flush=True)
    dto = O.cfl_dt(op, inst.u0, 0.3)
    assert n == 1 and abs(t / dto - 1) <= 1e-14
    PT.check_step(op, inst.u0, dto, u.cpu().numpy(), recs, what=f"u after one step (order {order})")


def _smooth_1d(n=126):
    """1D Euler data with no flat stretch (smooth profiles and one jump in density)."""
    x = W.nodes(-1.0, 1.0, n)
    rho = 1.0 + 0.3 * np.sin(np.pi * x) + 0.5 * (x > 0.2)
    return W.conserved_1d(rho, 0.4 * np.cos(2 * np.pi * x), 1.0 + 0.2 * np.sin(3 * np.pi * x + 0.4)).reshape(3, 1, n)


def _smooth_2d(nx=48, ny=40):
    """2D Euler data with no flat stretch: smooth fields plus a discontinuous block,
    periodic with period 24."""
    t = np.arange(24) * (2.0 * np.pi / 24)
    X, Y = np.meshgrid(t, t)
    block = ((np.arange(24)[None, :] < 11) & (np.arange(24)[:, None] < 15)).astype(float)
    rho = 1.0 + 0.3 * np.sin(X + 0.7) * np.cos(Y + 1.9) + 0.8 * block
    vx = 0.4 * np.sin(Y + 0.2) + 0.2 * block
    vy = 0.4 * np.cos(X + 2.5) - 0.3 * block
    p = 1.0 + 0.25 * np.cos(X + Y + 1.1) + 1.5 * block
    tab = W.conserved_2d(rho, vx, vy, p)
    return np.tile(tab, (1, ny // 24 + 1, nx // 24 + 1))[:, :ny, :nx].copy()


@pytest.mark.parametrize("delta", [0.0, 1.0, 1e30])
@pytest.mark.parametrize("kind,order", [("advection", 5), ("euler1d", 5), ("euler1d", 7), ("euler2d", 5),
                                        ("euler2d", 7)])
def test_threshold_extremes(kind, order, delta):
    """Selection threshold at its extremes (Section 3's two principles): delta = 0 leaves
    the first principle to indicators that are exactly zero, so most faces take the
    argmin of the second; delta = 1e30 always takes the top candidate (the linear
    scheme); delta = 1 mixes both.  L with selections and one step against the oracle at
    every cell, the GPU's choices replayed at near ties (they must lie in the oracle's
    tie sets).  The data have no flat stretch: there the oracle's row sums leave
    rounding residues that a difference table does not, and with delta = 0 every such
    face is a near tie."""
    torch = PT.torch_cuda()
    E = _E()
    if kind == "advection":
        inst, _ = _adv_case(131, jumps=True)
        u0 = inst.u0
        ep = E.problem_from_instance(inst, order=order, delta=delta, record_selection=True)
    elif kind == "euler1d":
        u0 = _smooth_1d()
        ep = E.make_problem(kind, u0.shape[2], order=order, bc_x="transmissive", delta=delta,
                            record_selection=True)
    else:
        u0 = _smooth_2d()
        ep = E.make_problem(kind, u0.shape[2], u0.shape[1], order=order, delta=delta, record_selection=True)
    op = PT.oracle_problem(ep)
    plan = E.enoao_plan_create(ep)
    u = PT.to_dev(torch, u0)
    L = torch.empty_like(u)
    E.enoao_rhs(plan, u, L)
    sel = E.enoao_get_selection(plan)
    PT.check_rhs(op, u0, L.cpu().numpy(), sel, what=f"L (delta {delta})")
    _, selr, _ = O.rhs(op, u0, with_selection=True)
    K = 6 if order == 5 else 9
    if delta == 1e30:
        assert (selr == K - 1).all() and (np.asarray(sel) == K - 1).all()
    if delta == 0.0:
        assert (selr != K - 1).mean() > 0.1  # the second principle decides many faces
    dt = 0.5 * O.cfl_dt(op, u0, 0.3)
    E.enoao_step(plan, u, dt)
    recs = E.enoao_get_step_selection(plan)
    PT.check_step(op, u0, dt, u.cpu().numpy(), recs, what=f"u (delta {delta})")


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("eq,shape", [("advection", (1, 1, 70)), ("euler1d", (3, 1, 70)),
                                      ("euler2d", (4, 37, 70))])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_constant_state(eq, shape, bc, order):
    """A uniform state (moving, for Euler) is steady: every face sees the same data and
    computes the same flux, so L is exactly zero; one step matches the oracle."""
    torch = PT.torch_cuda()
    E = _E()
    nc, ny, nx = shape
    if eq == "advection":
        u0 = np.full(shape, 0.7)
    elif eq == "euler1d":
        u0 = np.broadcast_to(W.conserved_1d(1.3, 0.4, 0.9).reshape(3, 1, 1), shape).copy()
    else:
        u0 = np.broadcast_to(W.conserved_2d(1.3, 0.4, -0.25, 0.9).reshape(4, 1, 1), shape).copy()
    ep = E.make_problem(eq, nx, ny, order=order, bc_x=bc, bc_y=bc)
    op = PT.oracle_problem(ep)
    plan = E.enoao_plan_create(ep)
    u = PT.to_dev(torch, u0)
    L = torch.full_like(u, float("nan"))
    E.enoao_rhs(plan, u, L)
    assert torch.equal(L, torch.zeros_like(L)), "L of a uniform state must vanish"
    dt = 0.5 * O.cfl_dt(op, u0, 0.3)
    E.enoao_step(plan, u, dt)
    torch.cuda.synchronize()
    PT.assert_close_by_component(u.cpu().numpy(), O.step(op, u0, dt), what="u")


def test_plans_on_two_streams_concurrently():
    """Two plans advanced at the same time from two host threads, each on a stream of
    its own (and a batch of both on a third stream), give bitwise the results of
    running them one after the other: every call is ordered on the stream it is given
    and the plans share no device state."""
    import threading
    torch = PT.torch_cuda()
    E = _E()
    insts = [W.quadrants(1, 300, 260), W.quadrants(3, 257, 301)]
    probs = [E.problem_from_instance(i) for i in insts]
    seq = []
    for p, i in zip(probs, insts):
        plan = E.enoao_plan_create(p)
        u = PT.to_dev(torch, i.u0)
        E.enoao_solve(plan, u, 1e30, cfl=0.3, max_steps=12)
        seq.append(u.cpu())
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    plans = [E.enoao_plan_create(p, stream=s) for p, s in zip(probs, streams)]
    for plan in plans:
        E.enoao_plan_set_launch(plan, 1)  # one workgroup per CU each: room for both at once
    us = [PT.to_dev(torch, i.u0) for i in insts]
    errors = []

    def run(k):
        try:
            E.enoao_solve(plans[k], us[k], 1e30, cfl=0.3, max_steps=12, stream=streams[k])
        except Exception as e:  # reported by the main thread
            errors.append((k, e))

    for rep in range(2):
        for k in range(2):
            us[k].copy_(torch.from_numpy(insts[k].u0))
        torch.cuda.synchronize()
        threads = [threading.Thread(target=run, args=(k,)) for k in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=60)
        assert not any(t.is_alive() for t in threads) and not errors, errors
        torch.cuda.synchronize()
        for k in range(2):
            assert torch.equal(us[k].cpu(), seq[k]), f"plan {k}, repetition {rep}"
    s3 = torch.cuda.Stream()
    batch = E.enoao_batch_create(probs, stream=s3)
    vs = [PT.to_dev(torch, i.u0) for i in insts]
    torch.cuda.synchronize()
    E.enoao_batch_step(batch, vs, 12, 0.3, stream=s3)
    torch.cuda.synchronize()
    for k in range(2):
        assert torch.equal(vs[k].cpu(), seq[k]), f"batch member {k}"
