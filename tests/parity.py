"""Helpers of the GPU parity tests: problem translation, device round trips and the
comparison rules.

Comparison rules (the HIP path against the FP64 oracle), applied to every cell:
  * states and L: per component c, max |gpu - oracle| <= RTOL * max |oracle_c|
    (RTOL = 1e-12; a component that is identically zero in the oracle is scaled
    by the largest component instead);
  * stencil selections: the GPU's record of every face, field and side is replayed
    by the oracle (oracle.rhs_replay / step_replay).  Where the GPU picked another
    candidate than the oracle, the pick must lie in the oracle's tie set there (the
    candidates an evaluation with rounding-level different indicators could take
    under Section 3.2's two principles: a deciding comparison within 1e-14 of its
    rounding scale); a pick outside it fails the test.  The oracle then takes the
    GPU's pick, so the value comparison covers every cell with no exception.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O

RTOL = 1e-12
DT_RTOL = 1e-14  # device CFL step against the oracle's, from the same state


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def oracle_problem(ep):
    """oracle Problem equal to an enoao.Problem"""
    return O.Problem(ep.equation, nx=ep.nx, ny=ep.ny, order=ep.order, x_lo=ep.x_lo, x_hi=ep.x_hi,
                     y_lo=ep.y_lo, y_hi=ep.y_hi, bc_x=ep.bc_x, bc_y=ep.bc_y, gamma=ep.gamma,
                     adv_speed=ep.adv_speed, delta=ep.delta, recon_vars=ep.recon_vars)


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def assert_close_by_component(gpu, ref, rtol=RTOL, what="state"):
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    assert gpu.shape == ref.shape
    assert np.isfinite(gpu).all(), f"{what}: non-finite GPU values"
    overall = np.abs(ref).max()
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        if scale == 0.0:
            scale = overall if overall > 0 else 1.0
        d = np.abs(gpu[c] - ref[c])
        worst = d.max()
        assert worst <= rtol * scale, (
            f"{what}[{c}]: max |diff| {worst:.3e} > {rtol:.0e} * {scale:.3e} at {np.unravel_index(d.argmax(), d.shape)}")


def check_rhs(op, u, L_gpu, sel_gpu, what="L", rtol=RTOL):
    """GPU L and selection record of one evaluation against the oracle replaying the
    GPU's picks at near ties.  Returns (number of face sides the oracle flags as near
    ties, number where the GPU took another candidate of the tie set)."""
    sel_gpu = np.asarray(sel_gpu)
    Lr, selr, tier, nbad = O.rhs_replay(op, u, sel_gpu)
    _, sel_own, _ = O.rhs(op, u, with_selection=True)
    assert nbad == 0, f"{what}: {nbad} GPU selections outside the oracle's tie sets"
    assert np.array_equal(selr, sel_gpu)
    assert_close_by_component(L_gpu, Lr, rtol=rtol, what=what)
    return int((tier != 0).sum()), int((sel_own != sel_gpu).sum())


def check_step(op, u, dt, u_gpu, recs_gpu, what="u", rtol=RTOL):
    """One GPU step (its three stage records) against the oracle's step from the same
    state with the GPU's picks replayed at near ties."""
    ur, nbad = O.step_replay(op, u, dt, recs_gpu)
    assert nbad == 0, f"{what}: {nbad} GPU selections outside the oracle's tie sets"
    assert_close_by_component(u_gpu, ur, rtol=rtol, what=what)
    return ur


def gpu_step_recorded(torch, E, plan_rec, u, dt):
    """One host-dt step of a recording plan: (new state on the host, three stage records)."""
    v = to_dev(torch, u)
    E.enoao_step(plan_rec, v, dt)
    recs = E.enoao_get_step_selection(plan_rec)
    return v.cpu().numpy(), recs


def workers():
    """host threads for the oracle (its calls release the interpreter lock)"""
    return max(1, min(16, os.cpu_count() or 1))


def lockstep_solve(torch, E, ep, u0, t_final, cfl=0.0, max_steps=1 << 40, what="", pool=None, dt_fixed=0.0):
    """A CFL time loop on the GPU checked step by step against the oracle.

    The GPU advances a recording plan one controlled step per enoao_solve call (the
    device computes dt from the state, or takes dt_fixed > 0, and clips the last step
    to t_final); after each
    step its state, step size and three stage records are copied out.  Each step is
    then checked independently, from the GPU's state before it: the oracle's CFL step
    from that state must equal the GPU's to DT_RTOL (and clip alike), and the oracle's
    step replaying the GPU's records must match the GPU's new state to RTOL at every
    cell.  Finally the same run as one enoao_solve call of a plan without a record (the
    device-side loop over captured graphs) must give bitwise the same state, step
    count and end time.  Returns (final state, steps, t, flagged face sides, GPU picks
    that differ from the oracle's own)."""
    op = oracle_problem(ep)
    rec_ep = type(ep).from_buffer_copy(ep)
    rec_ep.flags |= E.F_RECORD_SELECTION
    plan = E.enoao_plan_create(rec_ep)
    u = to_dev(torch, u0)
    states = [np.ascontiguousarray(u0, dtype=np.float64)]
    dts, recs = [], []
    t = 0.0
    while len(dts) < max_steps:
        rem = t_final - t
        if not rem > 0.0:
            break
        dt, n = E.enoao_solve(plan, u, rem, cfl=cfl, dt_fixed=dt_fixed, max_steps=1)
        assert n == 1, f"{what}: step {len(dts)} not taken"
        last = dt == rem
        t = t_final if last else t + dt
        dts.append((dt, last))
        recs.append(E.enoao_get_step_selection(plan))
        states.append(u.cpu().numpy())
    E.enoao_plan_check(plan)

    def check(k):
        dt, last = dts[k]
        dto = dt_fixed if dt_fixed > 0.0 else O.cfl_dt(op, states[k], cfl)
        rem = t_final - sum_t[k]
        clip = dto >= rem * (1.0 - 1e-10)
        assert clip == last, f"{what}: step {k} clipped on one side only"
        if clip:
            dto = rem
        assert abs(dt - dto) <= DT_RTOL * dto, f"{what}: step {k}: dt {dt!r} against oracle {dto!r}"
        ur, nbad = O.step_replay(op, states[k], dto, recs[k])
        assert nbad == 0, f"{what}: step {k}: {nbad} GPU selections outside the oracle's tie sets"
        assert_close_by_component(states[k + 1], ur, what=f"{what} u after step {k}")
        _, own_sel, own_tie = O.rhs(op, states[k], with_selection=True)
        return int((own_tie != 0).sum()), int((own_sel != recs[k][:own_sel.size]).sum())

    # times at the start of every step, accumulated as both time loops do
    sum_t = [0.0]
    for dt, last in dts:
        sum_t.append(t_final if last else sum_t[-1] + dt)
    if pool is None:
        with ThreadPoolExecutor(workers()) as ex:
            stats = list(ex.map(check, range(len(dts))))
    else:
        stats = list(pool.map(check, range(len(dts))))

    # the device-side loop of one call reproduces the per-step trajectory bitwise
    plain = E.enoao_plan_create(ep)
    v = to_dev(torch, u0)
    t1, n1 = E.enoao_solve(plain, v, t_final, cfl=cfl, dt_fixed=dt_fixed, max_steps=max_steps)
    assert n1 == len(dts) and t1 == t, f"{what}: one-call solve took {n1} steps to {t1!r}"
    assert np.array_equal(v.cpu().numpy(), states[-1]), f"{what}: one-call solve differs from the stepped run"
    return states[-1], len(dts), t, sum(s[0] for s in stats), sum(s[1] for s in stats)
