"""The face kernels' wave-uniform shortcut (Section 3.2, first principle: a field whose
top candidate is within delta on every face of a wave takes that candidate's value
directly) must not change any result: with the shortcut switched off every face takes
the full selection, and states and selection records agree bit for bit, for the
x-sweep (top differences staged per node), the y-sweep and the LDS-resident solver
(formed per face) and batches."""
import numpy as np
import pytest

from paper_2108_12742_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _run(torch, inst, order, steps, cfl, shortcut, resident=True, record=True):
    E = _E()
    E.enoao_set_shortcut(shortcut)
    E.enoao_set_resident(resident)
    try:
        plan = E.enoao_plan_create(E.problem_from_instance(inst, order=order, record_selection=record))
        u = PT.to_dev(torch, inst.u0)
        t, n = E.enoao_solve(plan, u, 1e300, cfl=cfl, max_steps=steps)
        sel = E.enoao_get_selection(plan) if record else None
        torch.cuda.synchronize()
        return u.cpu().numpy(), sel, n
    finally:
        E.enoao_set_shortcut(True)
        E.enoao_set_resident(True)


CASES = [
    ("quadrants", lambda: W.quadrants(1, 96, 80), 25, 0.3),
    ("riemann", lambda: W.riemann_1d(5, 700), 120, 0.5),
    ("lax", lambda: W.lax_tube(200), 100, 0.3),
    ("combination", lambda: W.combination_wave(400), 200, 0.5),
]


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("name,make,steps,cfl", CASES, ids=[c[0] for c in CASES])
def test_shortcut_does_not_change_results(name, make, steps, cfl, order):
    torch = PT.torch_cuda()
    inst = make()
    print(f"[shortcut] {name} order {order}", flush=True)
    a, sa, na = _run(torch, inst, order, steps, cfl, True, resident=False)
    b, sb, nb = _run(torch, inst, order, steps, cfl, False, resident=False)
    assert na == nb == steps
    assert np.array_equal(a, b), f"{name}: max diff {np.abs(a - b).max():.3e}"
    assert np.array_equal(sa, sb)
    if inst.equation != "euler2d":
        # the LDS-resident solver, with and without the shortcut
        c, _, nc = _run(torch, inst, order, steps, cfl, True, resident=True, record=False)
        d, _, nd = _run(torch, inst, order, steps, cfl, False, resident=True, record=False)
        assert nc == nd == steps
        assert np.array_equal(c, d) and np.array_equal(a, c)


def test_shortcut_batch():
    torch = PT.torch_cuda()
    E = _E()
    insts = W.batch_1d(3, 12, n_lo=128, n_hi=3000)
    out = []
    for shortcut in (True, False):
        E.enoao_set_shortcut(shortcut)
        try:
            b = E.enoao_batch_create([E.problem_from_instance(i) for i in insts])
            states = [PT.to_dev(torch, i.u0) for i in insts]
            E.enoao_batch_step(b, states, 60, 0.5)
            torch.cuda.synchronize()
            out.append([s.cpu().numpy() for s in states])
            E.enoao_batch_destroy(b)
        finally:
            E.enoao_set_shortcut(True)
    for x, y in zip(*out):
        assert np.array_equal(x, y)


def test_shortcut_rejects_bad_values():
    E = _E()
    assert E.lib().enoao_set_shortcut(2) != 0
