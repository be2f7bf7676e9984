"""Invariants of the method checked on the GPU path at the benchmark's full size.

These hold at any size, so they cover the 2048^2 workload (seeded quadrant data, the
benchmark's launch path: enoao_solve with CFL time steps) for several steps, where the
oracle would take minutes per step:
  * x <-> y transposition (with the momentum components swapped) commutes with a step:
    a transposed problem sends the data through the other sweep kernel;
  * mirroring x -> -x (x momentum negated) commutes with a step: plus-side
    reconstructions become minus-side ones;
  * on a periodic grid the conservative difference keeps the sum of every conserved
    variable (the flux differences telescope).
"""
import numpy as np
import pytest

from tests import parity as PT

pytestmark = pytest.mark.gpu

STEPS = 3


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _instance(n=2048, ny=None):
    from paper_2108_12742_amd import workloads as W
    return W.quadrants(W.QUADRANT_BENCH_SEED, n, ny)


def _run(E, ep, u, order):
    plan = E.enoao_plan_create(ep)
    t, k = E.enoao_solve(plan, u, 1e30, cfl=0.3, max_steps=STEPS)
    E.enoao_plan_check(plan)
    assert k == STEPS
    return t


def _assert_close(torch, a, b, what):
    for q in range(a.shape[0]):
        scale = b[q].abs().max().item()
        d = (a[q] - b[q]).abs().max().item()
        assert d <= PT.RTOL * scale, f"{what}[{q}]: max |diff| {d:.3e} > {PT.RTOL:.0e} * {scale:.3e}"


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("shape", [(2048, 2048), (1000, 777)], ids=["2048x2048", "1000x777"])
def test_transpose_symmetry(shape, order):
    torch = PT.torch_cuda()
    E = _E()
    nx, ny = shape
    inst = _instance(nx, ny)
    ep = E.problem_from_instance(inst, order=order)
    epT = E.make_problem("euler2d", ny, nx, order=order, x_lo=ep.y_lo, x_hi=ep.y_hi, y_lo=ep.x_lo,
                         y_hi=ep.x_hi, bc_x=ep.bc_y, bc_y=ep.bc_x, gamma=ep.gamma)
    u = PT.to_dev(torch, inst.u0)
    uT = torch.stack([u[0].t(), u[2].t(), u[1].t(), u[3].t()]).contiguous()
    print(f"transpose {nx}x{ny} order {order}", flush=True)
    t = _run(E, ep, u, order)
    tT = _run(E, epT, uT, order)
    assert abs(t / tT - 1) <= 1e-14
    back = torch.stack([uT[0].t(), uT[2].t(), uT[1].t(), uT[3].t()])
    print(f"  bitwise equal: {torch.equal(back, u)}", flush=True)
    _assert_close(torch, back, u, "transposed solve")


@pytest.mark.parametrize("order", [5, 7])
def test_mirror_symmetry(order):
    torch = PT.torch_cuda()
    E = _E()
    inst = _instance()
    ep = E.problem_from_instance(inst, order=order)
    assert ep.x_lo == -ep.x_hi and ep.bc_x == E.BC_PERIODIC
    n = ep.nx
    u = PT.to_dev(torch, inst.u0)
    # node i sits at x_lo + i dx; -x maps it to node (n - i) mod n
    idx = (-torch.arange(n, device="cuda")) % n
    sign = torch.tensor([1.0, -1.0, 1.0, 1.0], dtype=torch.float64, device="cuda").view(4, 1, 1)
    um = (u[:, :, idx] * sign).contiguous()
    print(f"mirror order {order}", flush=True)
    t = _run(E, ep, u, order)
    tm = _run(E, ep, um, order)
    assert t == tm
    back = u.new_empty(u.shape)
    back[:, :, idx] = um * sign
    print(f"  bitwise equal: {torch.equal(back, u)}", flush=True)
    _assert_close(torch, back, u, "mirrored solve")


@pytest.mark.parametrize("order", [5, 7])
def test_periodic_conservation(order):
    """Sum of each conserved variable over the periodic grid, before and after the steps,
    to 1e-13 of the sum of magnitudes (the rounding of the updates and of the sums)."""
    torch = PT.torch_cuda()
    E = _E()
    inst = _instance()
    ep = E.problem_from_instance(inst, order=order)
    assert ep.bc_x == E.BC_PERIODIC and ep.bc_y == E.BC_PERIODIC
    u = PT.to_dev(torch, inst.u0)
    before = u.sum(dim=(1, 2))
    mag = u.abs().sum(dim=(1, 2))
    _run(E, ep, u, order)
    after = u.sum(dim=(1, 2))
    rel = ((after - before).abs() / mag).max().item()
    print(f"conservation order {order}: max relative change {rel:.2e}", flush=True)
    assert rel <= 1e-13


@pytest.mark.slow
def test_long_run_deterministic_and_conservative():
    """400 CFL steps of the 2048^2 workload, twice from the same state: the runs are
    bitwise identical (the per-stage maxima are combined with an order-independent
    atomic max, and every other result has one writer), the state stays physical, and
    the conserved sums drift only at rounding level."""
    torch = PT.torch_cuda()
    E = _E()
    inst = _instance()
    ep = E.problem_from_instance(inst)
    plan = E.enoao_plan_create(ep)
    runs = []
    for rep in range(2):
        u = PT.to_dev(torch, inst.u0)
        before = u.sum(dim=(1, 2))
        mag = u.abs().sum(dim=(1, 2))
        t, k = E.enoao_solve(plan, u, 1e30, cfl=0.3, max_steps=400)
        E.enoao_plan_check(plan)
        assert k == 400
        rel = ((u.sum(dim=(1, 2)) - before).abs() / mag).max().item()
        print(f"run {rep}: t = {t:.6g}, max relative drift of the sums {rel:.2e}", flush=True)
        assert rel <= 1e-11
        runs.append((t, u))
    assert runs[0][0] == runs[1][0] and torch.equal(runs[0][1], runs[1][1])


def _oblique_wave(n):
    from paper_2108_12742_amd import workloads as W
    x = W.nodes(-1.0, 1.0, n)
    X, Y = np.meshgrid(x, x)
    rho = 1 + 0.2 * np.sin(np.pi * (X + Y))
    one = np.ones_like(rho)
    return X, Y, W.conserved_2d(rho, one, 0.5 * one, one)


@pytest.mark.slow
def test_oblique_density_wave_against_exact_solution():
    """rho = 1 + 0.2 sin(pi (x + y)), (u, v) = (1, 0.5), p = 1 on [-1, 1]^2 periodic is the
    profile translated by (u t, v t): the GPU path at 40^2 and 80^2 (order above 4.5) and
    at 1024^2 (about 1640 steps), each against the closed form, with no oracle involved."""
    torch = PT.torch_cuda()
    E = _E()
    errs = {}
    for n, t_end in ((40, 0.4), (80, 0.4), (1024, 0.05)):
        X, Y, u0 = _oblique_wave(n)
        plan = E.enoao_plan_create(E.make_problem("euler2d", n, n))
        u = PT.to_dev(torch, u0)
        t, k = E.enoao_solve(plan, u, t_end, dt_fixed=(2.0 / n) ** (5 / 3))
        assert t == t_end
        exact = 1 + 0.2 * np.sin(np.pi * ((X - t_end) + (Y - 0.5 * t_end)))
        errs[n] = np.abs(u[0].cpu().numpy() - exact).max()
        print(f"n = {n}: {k} steps, max error {errs[n]:.3e}", flush=True)
    order = np.log2(errs[40] / errs[80])
    assert errs[80] < 1e-6 and order > 4.5, (errs, order)
    assert errs[1024] < 1e-10, errs


@pytest.mark.slow
def test_oblique_density_wave_order7():
    """The same wave at order 7 with dt = dx^(7/3) (so the RK3 time error stays at seventh
    order): the GPU error against the closed form falls at close to seventh order."""
    torch = PT.torch_cuda()
    E = _E()
    errs = {}
    for n in (40, 80):
        X, Y, u0 = _oblique_wave(n)
        plan = E.enoao_plan_create(E.make_problem("euler2d", n, n, order=7))
        u = PT.to_dev(torch, u0)
        t, k = E.enoao_solve(plan, u, 0.4, dt_fixed=(2.0 / n) ** (7 / 3))
        assert t == 0.4
        exact = 1 + 0.2 * np.sin(np.pi * ((X - 0.4) + (Y - 0.2)))
        errs[n] = np.abs(u[0].cpu().numpy() - exact).max()
        print(f"n = {n}: {k} steps, max error {errs[n]:.3e}", flush=True)
    order = np.log2(errs[40] / errs[80])
    assert errs[80] < 1e-8 and order > 6.5, (errs, order)
