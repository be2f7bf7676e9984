"""Cooperative solver of one mid-sized 1D problem: every controlled step of an
enoao_solve call in one cooperative launch with grid barriers between stages.
Results are bitwise those of the streaming kernels (same arithmetic), match the
oracle, and the cooperative path is the one that ran."""
import numpy as np
import pytest

from paper_2108_12742_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _solve(torch, E, inst, order, coop, t_final=1e300, max_steps=40, cfl=0.3, u0=None):
    # coop=False: the streaming kernels (the resident solver off as well)
    E.enoao_set_coop(coop)
    E.enoao_set_resident(False)
    try:
        plan = E.enoao_plan_create(E.problem_from_instance(inst, order=order,
                                                           recon_vars=inst.meta.get("recon", 0)))
        E.enoao_profile(plan, True)
        u = PT.to_dev(torch, inst.u0 if u0 is None else u0)
        t, n = E.enoao_solve(plan, u, t_final, cfl=cfl, max_steps=max_steps)
        prof = E.enoao_profile_read(plan)
    finally:
        E.enoao_set_coop(True)
        E.enoao_set_resident(True)
    return u.cpu(), t, n, prof


def _case(kind, n, seed):
    if kind == "adv":
        inst = W.advection(seed, n)
        x = W.nodes(-1.0, 1.0, n)
        inst.u0 = inst.u0 + np.where((x > -0.3) & (x < 0.25), 0.6, 0.0).reshape(1, 1, n)
        return inst
    inst = W.riemann_1d(seed, n)
    if kind == "e1-comp":
        inst.meta["recon"] = "component"
    if kind == "e1-periodic":
        inst.bc_x = "periodic"
    return inst


# sizes past the LDS-resident limit (about 1890 Euler nodes at order 5, 1880 at
# order 7, 6600 advection nodes) up to one 63-cell segment per wave of one
# workgroup per CU (1024 segments: 64512 nodes on 256 CUs)
CASES = [("e1", 2000, 5), ("e1", 1900, 7), ("e1-periodic", 4097, 5), ("e1-comp", 3001, 7), ("adv", 7000, 5),
         ("e1", 64512, 5)]


@pytest.mark.parametrize("kind,n,order", CASES, ids=[f"{k}-{n}-ao{o}" for k, n, o in CASES])
def test_coop_bitwise_equals_streaming(kind, n, order):
    torch = PT.torch_cuda()
    E = _E()
    inst = _case(kind, n, 5 + n % 7)
    print(f"cooperative case {kind} N={n} order {order}", flush=True)
    uc, tc, nc, prof_c = _solve(torch, E, inst, order, True)
    us, ts, ns, prof_s = _solve(torch, E, inst, order, False)
    assert prof_c["coop"][1] > 0 and prof_c["sweep_x_s1"][1] == 0, "the cooperative solver did not run"
    assert prof_s["coop"][1] == 0 and prof_s["resident"][1] == 0 and prof_s["sweep_x_s1"][1] > 0
    assert (tc, nc) == (ts, ns) and nc == 40
    assert torch.equal(uc, us), "cooperative and streaming results differ"


def test_coop_not_taken_past_its_size():
    """One segment per wave more than one workgroup per CU allows: the streaming kernels."""
    torch = PT.torch_cuda()
    E = _E()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = 63 * 4 * cus + 1
    inst = _case("e1", n, 3)
    _, _, nc, prof = _solve(torch, E, inst, 5, True, max_steps=3)
    assert nc == 3 and prof["coop"][1] == 0 and prof["sweep_x_s1"][1] > 0


def test_coop_matches_oracle_step_by_step():
    """The C1 size: the oracle's CFL loop checked step by step (recording streaming
    plan), and the same run as one enoao_solve call of the cooperative solver
    bitwise equal to it."""
    torch = PT.torch_cuda()
    E = _E()
    inst = _case("e1", 2000, 11)
    ep = E.problem_from_instance(inst)
    uo, no, to, _, _ = PT.lockstep_solve(torch, E, ep, inst.u0, 1e300, cfl=0.3, max_steps=30, what="coop N=2000")
    uc, tc, nc, prof = _solve(torch, E, inst, 5, True, max_steps=30)
    assert prof["coop"][1] > 0
    assert (nc, tc) == (no, to)
    assert np.array_equal(uc.numpy(), uo)


def test_coop_stops_at_t_final_and_resumes():
    torch = PT.torch_cuda()
    E = _E()
    inst = _case("e1", 2500, 4)
    outs = []
    for coop in (True, False):
        E.enoao_set_coop(coop)
        try:
            plan = E.enoao_plan_create(E.problem_from_instance(inst))
            u = PT.to_dev(torch, inst.u0)
            t1, n1 = E.enoao_solve(plan, u, 0.01, cfl=0.3)
            t2, n2 = E.enoao_solve(plan, u, 0.004, cfl=0.3, max_steps=7)
        finally:
            E.enoao_set_coop(True)
        outs.append((u.cpu(), t1, n1, t2, n2))
    (ua, *ra), (ub, *rb) = outs
    assert ra == rb and ra[0] == 0.01 and ra[3] <= 7
    assert torch.equal(ua, ub)


def test_coop_reports_nonphysical_state():
    torch = PT.torch_cuda()
    E = _E()
    inst = _case("e1", 3000, 2)
    u0 = inst.u0.copy()
    u0[2, 0, 1500] = 0.25 * u0[1, 0, 1500] ** 2 / u0[0, 0, 1500]  # E below the kinetic energy: p < 0
    inst.u0 = u0
    res = []
    for coop in (True, False):
        E.enoao_set_coop(coop)
        try:
            plan = E.enoao_plan_create(E.problem_from_instance(inst))
            E.enoao_profile(plan, True)
            u = PT.to_dev(torch, inst.u0)
            with pytest.raises(E.EnoaoError) as ei:
                E.enoao_solve(plan, u, 1.0, cfl=0.3, max_steps=200)
            assert ei.value.status == E.ENONPHYSICAL
            assert (E.enoao_profile_read(plan)["coop"][1] > 0) == coop
        finally:
            E.enoao_set_coop(True)
        res.append(u.cpu().numpy())
    assert np.array_equal(res[0], res[1], equal_nan=True)


@pytest.mark.parametrize("kind,n,solver", [("e1", 500, "resident"), ("e1", 700, "coop"), ("adv", 1200, "resident"),
                                           ("adv", 1400, "coop")])
def test_lone_member_solver_choice(kind, n, solver):
    """A lone member that fits the resident solver takes the cooperative one past 9
    segments (Euler; advection: 20), and without it the resident one: both bitwise
    equal to the streaming kernels."""
    torch = PT.torch_cuda()
    E = _E()
    inst = _case(kind, n, 2)
    outs = []
    for coop, resident in ((True, True), (False, True), (False, False)):
        E.enoao_set_coop(coop)
        E.enoao_set_resident(resident)
        try:
            plan = E.enoao_plan_create(E.problem_from_instance(inst))
            E.enoao_profile(plan, True)
            u = PT.to_dev(torch, inst.u0)
            E.enoao_solve(plan, u, 1e300, cfl=0.3, max_steps=25)
            prof = E.enoao_profile_read(plan)
        finally:
            E.enoao_set_coop(True)
            E.enoao_set_resident(True)
        ran = "coop" if prof["coop"][1] else "resident" if prof["resident"][1] else "stream"
        outs.append((ran, u.cpu()))
    assert [o[0] for o in outs] == [solver, "resident", "stream"]
    assert torch.equal(outs[0][1], outs[2][1]) and torch.equal(outs[1][1], outs[2][1])


_CHILD = r'''
import json, sys
import numpy as np
import torch
from paper_2108_12742_amd import enoao as E
from paper_2108_12742_amd import workloads as W
inst = W.riemann_1d(7, 2000)
out = {}
for coop in (1, 0):
    E.enoao_set_coop(coop)
    plan = E.enoao_plan_create(E.problem_from_instance(inst))
    E.enoao_profile(plan, True)
    u = torch.from_numpy(inst.u0).cuda()
    t, n = E.enoao_solve(plan, u, 1e300, cfl=0.3, max_steps=40)
    out[coop] = (u.cpu().numpy(), t, n, E.enoao_profile_read(plan)["coop"][1])
    # the same line as a one-member batch (its steps take the same path)
    b = E.enoao_batch_create([E.problem_from_instance(inst)])
    ub = [torch.from_numpy(inst.u0).cuda()]
    E.enoao_batch_step(b, ub, 40, 0.3)
    tb, nb, sb = E.enoao_batch_query(b)
    out["batch", coop] = (ub[0].cpu().numpy(), float(tb[0]), int(nb[0]), int(sb[0]))
print(json.dumps({"same": bool(np.array_equal(out[1][0], out[0][0])), "t": [out[1][1], out[0][1]],
                  "n": [out[1][2], out[0][2]], "coop_launches": out[1][3],
                  "batch_same": bool(np.array_equal(out["batch", 1][0], out[0][0]) and
                                     np.array_equal(out["batch", 0][0], out[0][0])),
                  "batch_n": [out["batch", 1][2], out["batch", 0][2]],
                  "batch_status": [out["batch", 1][3], out["batch", 0][3]]}), flush=True)
'''


def test_coop_beside_another_process():
    """A second process on the GPU while this one, which has made cooperative
    launches, is alive: the runtime may turn the second one's cooperative launch
    down, and the plan (or one-member batch) then takes the streaming kernels (no
    error, the same bits)."""
    import json
    import os
    import subprocess
    import sys
    torch = PT.torch_cuda()
    E = _E()
    inst = _case("e1", 2000, 3)
    plan = E.enoao_plan_create(E.problem_from_instance(inst))
    E.enoao_profile(plan, True)
    u = PT.to_dev(torch, inst.u0)
    E.enoao_solve(plan, u, 1e300, cfl=0.3, max_steps=5)
    assert E.enoao_profile_read(plan)["coop"][1] > 0
    torch.cuda.synchronize()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    print("cooperative solve in a second process", flush=True)
    r = subprocess.run([sys.executable, "-c", _CHILD], cwd=root, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print("second process:", res, flush=True)
    assert res["same"] and res["n"] == [40, 40] and res["t"][0] == res["t"][1]
    assert res["batch_same"] and res["batch_n"] == [40, 40] and res["batch_status"] == [0, 0]
    del plan
