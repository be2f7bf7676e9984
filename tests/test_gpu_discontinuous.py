"""GPU parity on the discontinuous workloads of Sections 4.1 and 4.2: the advected
Jiang-Shu combination profile (Gaussians, square wave, triangle, half ellipse) and the
Lax shock tube.  Near discontinuities the lower-order candidates are selected and the
wave-uniform top-candidate shortcut is rarely taken, so these runs exercise the full
selection path.

Per step: from the oracle's state, the GPU's L (with selections) and one GPU step match
the oracle at every cell, with the GPU's choices replayed by the oracle at near ties.
Whole runs: every step of the GPU's run is checked from the GPU's state before it (same
dt, every cell at 1e-12), the one-call device loop equals the stepped run bitwise, and
the oracle's own run takes as many steps to the same end time."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12742_amd import workloads as W
from tests import parity as PT
from paper_2108_12742_amd import exact_riemann as RX

pytestmark = pytest.mark.gpu

LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _trajectory_parity(torch, E, inst, order, nsteps, cfl=0.3):
    """Along the oracle's trajectory: per step, L with its selection record and the
    step with its three stage records against the oracle, which replays the GPU's picks
    at near ties (tests/parity.py); the streaming plan without a record takes bitwise
    the same step.  The trajectory continues from the replayed oracle state."""
    ep = E.problem_from_instance(inst, order=order, record_selection=True)
    op = PT.oracle_problem(ep)
    plan_rec = E.enoao_plan_create(ep)
    plan = E.enoao_plan_create(E.problem_from_instance(inst, order=order))
    ur = inst.u0.copy()
    low = 0
    for k in range(nsteps):
        u = PT.to_dev(torch, ur)
        L = torch.empty_like(u)
        E.enoao_rhs(plan_rec, u, L)
        sel = E.enoao_get_selection(plan_rec)
        PT.check_rhs(op, ur, L.cpu().numpy(), sel, what=f"L step {k}")
        low += int((np.asarray(sel) < O.num_candidates(order) - 1).sum())
        dt = O.cfl_dt(op, ur, cfl)
        got, recs = PT.gpu_step_recorded(torch, E, plan_rec, ur, dt)
        E.enoao_step(plan, u, dt)
        assert np.array_equal(u.cpu().numpy(), got)
        ur = PT.check_step(op, ur, dt, got, recs, what=f"u step {k}")
    return low


@pytest.mark.parametrize("order", [5, 7])
def test_combination_wave_steps(order):
    torch = PT.torch_cuda()
    E = _E()
    print(f"combination wave, order {order}, N = 400", flush=True)
    low = _trajectory_parity(torch, E, W.combination_wave(400), order, 25)
    assert low > 0  # lower-order candidates were taken and compared


@pytest.mark.timeout(900)
@pytest.mark.slow
@pytest.mark.parametrize("order", [5, 7])
def test_combination_wave_ten_periods(order):
    """N = 400 (dx = 1/200), t = 20 as in Section 4.1: all 13334 CFL steps checked one by
    one against the oracle (tests/parity.py lockstep_solve: same dt, every cell at 1e-12
    with the GPU's picks replayed at near ties), the one-call device loop bitwise equal
    to the stepped run, and the oracle's own run taking as many steps; the profile stays
    within its bounds."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.combination_wave(400)
    ep = E.problem_from_instance(inst, order=order)
    print(f"combination wave to t = 20, order {order}", flush=True)
    g, n, t, flagged, alt = PT.lockstep_solve(torch, E, ep, inst.u0, 20.0, cfl=0.3, what="combination")
    print(f"{n} steps, {flagged} flagged face sides, {alt} other tie picks", flush=True)
    _, tr, nr = O.solve(PT.oracle_problem(ep), inst.u0, 20.0, cfl=0.3)
    assert n == nr and t == tr == 20.0
    g = g[0, 0]
    assert g.max() <= 1.0 + 1e-3 and g.min() >= -1e-3


@pytest.mark.parametrize("order", [5, 7])
def test_lax_tube_steps(order):
    torch = PT.torch_cuda()
    E = _E()
    print(f"Lax tube, order {order}, N = 200", flush=True)
    low = _trajectory_parity(torch, E, W.lax_tube(200), order, 40)
    assert low > 0


@pytest.mark.parametrize("order", [5, 7])
def test_lax_tube_to_t026(order):
    """dx = 1/100, t = 0.26 as in Section 4.2; the GPU's density error against the exact
    Riemann solution equals the oracle's."""
    torch = PT.torch_cuda()
    E = _E()
    inst = W.lax_tube(200)
    ep = E.problem_from_instance(inst, order=order)
    g, n, t, _, _ = PT.lockstep_solve(torch, E, ep, inst.u0, 0.26, cfl=0.3, what="Lax tube")
    ur, tr, nr = O.solve(PT.oracle_problem(ep), inst.u0, 0.26, cfl=0.3)
    assert n == nr and t == tr == 0.26
    ex = RX.sample(*LAX, W.nodes(0.0, 2.0, 200), 1.0, 0.26)
    e_g = np.abs(g[0, 0] - ex[0]).mean()
    e_r = np.abs(ur[0, 0] - ex[0]).mean()
    assert abs(e_g / e_r - 1) < 1e-6 and e_g < 0.012, (e_g, e_r)
