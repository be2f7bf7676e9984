"""LDS-resident solver of small 1D problems: results are bitwise those of the streaming
kernels (same arithmetic), match the oracle, and the resident path is the one that ran."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12742_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _solve(torch, E, inst, order, resident, t_final=1e300, max_steps=40, cfl=0.3, profile=False):
    # the resident solver or the streaming kernels, never the cooperative solver
    # (which a lone member of more than 9 segments would take)
    E.enoao_set_resident(resident)
    E.enoao_set_coop(False)
    try:
        plan = E.enoao_plan_create(E.problem_from_instance(inst, order=order,
                                                           recon_vars=inst.meta.get("recon", 0)))
        if profile:
            E.enoao_profile(plan, True)
        u = PT.to_dev(torch, inst.u0)
        t, n = E.enoao_solve(plan, u, t_final, cfl=cfl, max_steps=max_steps)
        prof = E.enoao_profile_read(plan) if profile else None
    finally:
        E.enoao_set_resident(True)
        E.enoao_set_coop(True)
    return u.cpu(), t, n, prof


def _case(kind, n, seed):
    if kind == "adv":
        inst = W.advection(seed, n)
        x = W.nodes(-1.0, 1.0, n)
        inst.u0 = inst.u0 + np.where((x > -0.3) & (x < 0.25), 0.6, 0.0).reshape(1, 1, n)
        return inst
    if kind == "adv-left":
        inst = _case("adv", n, seed)
        inst.adv_speed = -0.8
        return inst
    if kind == "e1-comp":
        inst = W.riemann_1d(seed, n)
        inst.meta["recon"] = "component"
        return inst
    if kind == "e1-periodic":
        inst = W.riemann_1d(seed, n)
        inst.bc_x = "periodic"
        return inst
    return W.riemann_1d(seed, n)


# sizes up to the LDS limit of an Euler member (about 1890 nodes at order 5)
CASES = [("adv", 1, 5), ("adv", 200, 5), ("adv-left", 513, 7), ("adv", 3000, 5), ("e1", 5, 5), ("e1", 63, 5),
         ("e1", 512, 5), ("e1", 513, 7), ("e1-periodic", 700, 5), ("e1", 1024, 5), ("e1", 1500, 7),
         ("e1", 1700, 5), ("e1", 1800, 5), ("e1-comp", 900, 5), ("e1-comp", 600, 7)]


@pytest.mark.parametrize("kind,n,order", CASES, ids=[f"{k}-{n}-ao{o}" for k, n, o in CASES])
def test_resident_bitwise_equals_streaming_and_matches_oracle(kind, n, order):
    torch = PT.torch_cuda()
    E = _E()
    inst = _case(kind, n, 3 + n % 11)
    print(f"resident case {kind} N={n} order {order}", flush=True)
    ur, tr, nr, prof = _solve(torch, E, inst, order, True, profile=True)
    us, ts, ns, _ = _solve(torch, E, inst, order, False)
    assert prof["resident"][1] > 0, "the LDS-resident solver did not run"
    assert (tr, nr) == (ts, ns) and nr == 40
    assert torch.equal(ur, us), "resident and streaming results differ"
    ep = E.problem_from_instance(inst, order=order, recon_vars=inst.meta.get("recon", 0))
    # every step against the oracle; the stepped streaming run equals the resident one
    uo, no, to, _, _ = PT.lockstep_solve(torch, E, ep, inst.u0, 1e300, cfl=0.3, max_steps=40, what=f"{kind} N={n}")
    assert no == nr and to == tr
    assert np.array_equal(ur.numpy(), uo)


def test_resident_stops_at_t_final_and_resumes():
    torch = PT.torch_cuda()
    E = _E()
    inst = W.lax_tube(200)
    ur, tr, nr, _ = _solve(torch, E, inst, 5, True, t_final=0.26, max_steps=1 << 40)
    us, ts, ns, _ = _solve(torch, E, inst, 5, False, t_final=0.26, max_steps=1 << 40)
    assert tr == ts == 0.26 and nr == ns
    assert torch.equal(ur, us)


# member sizes spanning every size class of each kernel (workgroups per CU as the
# LDS allows, at most as the registers allow: two for Euler, three for advection)
BATCHES = [("e1", 5, (128, 300, 77, 1000, 5, 640, 1800)), ("e1", 7, (100, 513, 1500, 1000, 20, 900, 1700)),
           ("e1-comp", 5, (150, 700, 77, 1000, 1700)), ("adv", 5, (200, 1500, 3000, 6000, 64, 900, 4000))]


@pytest.mark.parametrize("kind,order,sizes", BATCHES, ids=[f"{k}-ao{o}" for k, o, _ in BATCHES])
def test_resident_batch_matches_streaming_batch(kind, order, sizes):
    torch = PT.torch_cuda()
    E = _E()
    insts = [_case(kind, n, 40 + k) for k, n in enumerate(sizes)]
    probs = [E.problem_from_instance(i, order=order, recon_vars=i.meta.get("recon", 0)) for i in insts]
    print(f"resident batch {kind} order {order} sizes {sizes}", flush=True)
    outs = []
    for resident in (True, False):
        E.enoao_set_resident(resident)
        try:
            b = E.enoao_batch_create(probs)
            E.enoao_batch_profile(b, True)
            us = [PT.to_dev(torch, i.u0) for i in insts]
            tf = [1e300, 0.01, 1e300, 2e-4] + [1e300] * (len(sizes) - 4)
            E.enoao_batch_step(b, us, 7, 0.3, t_final=tf)
            E.enoao_batch_step(b, us, 5, 0.3, t_final=tf)
            t, steps, status = E.enoao_batch_query(b)
            prof = E.enoao_batch_profile_read(b)
        finally:
            E.enoao_set_resident(True)
        assert (status == 0).all()
        assert (prof["resident"][1] > 0) == resident
        outs.append(([u.cpu() for u in us], t, steps))
    (ua, ta, sa), (ub, tb, sb) = outs
    assert (ta == tb).all() and (sa == sb).all()
    assert sa[0] == 12 and sa[3] < 12 and ta[3] == 2e-4
    for a, b in zip(ua, ub):
        assert torch.equal(a, b)


def test_resident_reports_nonphysical_state():
    torch = PT.torch_cuda()
    E = _E()
    inst = W.riemann_1d(2, 128)
    u0 = inst.u0.copy()
    u0[2, 0, 40] = 0.25 * u0[1, 0, 40] ** 2 / u0[0, 0, 40]  # E below the kinetic energy: p < 0
    inst.u0 = u0
    plan = E.enoao_plan_create(E.problem_from_instance(inst))
    E.enoao_profile(plan, True)
    u = PT.to_dev(torch, inst.u0)
    with pytest.raises(E.EnoaoError) as ei:
        E.enoao_solve(plan, u, 1.0, cfl=0.3, max_steps=200)
    assert ei.value.status == E.ENONPHYSICAL
    assert E.enoao_profile_read(plan)["resident"][1] > 0
