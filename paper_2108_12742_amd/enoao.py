"""Python binding of libenoao.so (include/enoao.h): argument marshalling only.

The functions carry the C names.  States are torch float64 CUDA (HIP) tensors,
C-contiguous, shape (ncomp, ny, nx); streams are torch.cuda.Stream objects (or
None for torch's current stream).  Every step of the method runs in the HIP
kernels of the library; if the library is missing the import fails loudly --
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libenoao.so")

ADVECTION, EULER1D, EULER2D = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
CHAR_ROE, COMPONENT = 0, 1  # reconstruction variables of the Euler systems
_RV = {"characteristic": CHAR_ROE, "component": COMPONENT}
F_RECORD_SELECTION = 1
MAX_EXTENT = 2**31 - 1024  # largest nx or ny (ENOAO_MAX_EXTENT); nx * ny <= 2**31
NCOMP = {ADVECTION: 1, EULER1D: 3, EULER2D: 4}
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ENONPHYSICAL = range(6)
_EQ = {"advection": ADVECTION, "euler1d": EULER1D, "euler2d": EULER2D}
_BC = {"periodic": BC_PERIODIC, "transmissive": BC_TRANSMISSIVE}


class Problem(ctypes.Structure):
    """enoao_problem"""
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("equation", ctypes.c_int32), ("order", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("recon_vars", ctypes.c_int32),
        ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
        ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("adv_speed", ctypes.c_double), ("delta", ctypes.c_double),
        ("flags", ctypes.c_uint32), ("reserved1", ctypes.c_uint32),
    ]

    @property
    def ncomp(self):
        return NCOMP[self.equation]

    @property
    def shape(self):
        return (self.ncomp, self.ny, self.nx)


def make_problem(equation, nx, ny=1, order=5, x_lo=-1.0, x_hi=1.0, y_lo=-1.0, y_hi=1.0,
                 bc_x=BC_PERIODIC, bc_y=BC_PERIODIC, gamma=1.4, adv_speed=1.0, delta=1e-5,
                 record_selection=False, recon_vars=CHAR_ROE) -> Problem:
    eq = _EQ[equation] if isinstance(equation, str) else int(equation)
    rv = _RV[recon_vars] if isinstance(recon_vars, str) else int(recon_vars)
    bcx = _BC[bc_x] if isinstance(bc_x, str) else int(bc_x)
    bcy = _BC[bc_y] if isinstance(bc_y, str) else int(bc_y)
    return Problem(ctypes.sizeof(Problem), eq, order, nx, ny, rv, x_lo, x_hi, y_lo, y_hi, bcx, bcy,
                   gamma, adv_speed, delta, F_RECORD_SELECTION if record_selection else 0, 0)


def problem_from_instance(inst, order=5, delta=1e-5, record_selection=False, recon_vars=CHAR_ROE) -> Problem:
    """Problem for a workloads.Instance."""
    return make_problem(inst.equation, inst.nx, inst.ny, order, inst.x_lo, inst.x_hi, inst.y_lo,
                        inst.y_hi, inst.bc_x, inst.bc_y, inst.gamma, inst.adv_speed, delta,
                        record_selection, recon_vars)


class EnoaoError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {enoao_status_string(status)} (status {status})")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run python -m paper_2108_12742_amd.build "
                              "(the ENO-AO path has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, pp = ctypes.c_void_p, ctypes.POINTER(Problem)
        st = ctypes.c_int
        sig = {
            "enoao_plan_create": ([pp, vp, ctypes.POINTER(vp)], st),
            "enoao_plan_destroy": ([vp], st),
            "enoao_workspace_bytes": ([pp], ctypes.c_size_t),
            "enoao_rhs": ([vp, vp, vp, vp], st),
            "enoao_step": ([vp, vp, ctypes.c_double, vp], st),
            "enoao_solve": ([vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), vp], st),
            "enoao_plan_check": ([vp, vp], st),
            "enoao_step_noalloc": ([pp, vp, ctypes.c_double, vp], st),
            "enoao_selection_size": ([vp], ctypes.c_size_t),
            "enoao_get_selection": ([vp, vp, ctypes.c_size_t, vp], st),
            "enoao_get_step_selection": ([vp, vp, ctypes.c_size_t, vp], st),
            "enoao_batch_create": ([pp, ctypes.c_int32, vp, ctypes.POINTER(vp)], st),
            "enoao_batch_destroy": ([vp], st),
            "enoao_batch_step": ([vp, ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_double), vp], st),
            "enoao_batch_reset": ([vp, vp], st),
            "enoao_batch_query": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int32), vp], st),
            "enoao_set_launch": ([ctypes.c_int32, ctypes.c_int32], st),
            "enoao_set_resident": ([ctypes.c_int32], st),
            "enoao_set_coop": ([ctypes.c_int32], st),
            "enoao_set_shortcut": ([ctypes.c_int32], st),
            "enoao_plan_set_tiles": ([vp, ctypes.c_int32, vp], st),
            "enoao_batch_set_tiles": ([vp, ctypes.c_int32, vp], st),
            "enoao_plan_set_launch": ([vp, ctypes.c_int32], st),
            "enoao_batch_set_launch": ([vp, ctypes.c_int32], st),
            "enoao_plan_set_launch_kinds": ([vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32], st),
            "enoao_batch_set_launch_kinds": ([vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32], st),
            "enoao_profile": ([vp, ctypes.c_int32], st),
            "enoao_profile_read": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_int32, vp], st),
            "enoao_batch_profile": ([vp, ctypes.c_int32], st),
            "enoao_batch_profile_read": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int32, vp], st),
            "enoao_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "enoao_pool_member_bytes": ([pp], ctypes.c_size_t),
            "enoao_pool_create": ([pp, ctypes.c_int32, ctypes.c_size_t, vp, ctypes.POINTER(vp)], st),
            "enoao_pool_destroy": ([vp], st),
            "enoao_pool_set_launch": ([vp, ctypes.c_int32], st),
            "enoao_pool_admit": ([vp, pp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_int32), vp], st),
            "enoao_pool_step": ([vp, ctypes.c_int32, vp], st),
            "enoao_pool_poll": ([vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double), ctypes.c_int32, vp], st),
            "enoao_pool_retire": ([vp, ctypes.c_int32, vp, ctypes.c_int32, vp], st),
            "enoao_pool_retire_async": ([vp, ctypes.c_int32, vp, vp, vp], st),
            "enoao_pool_usage": ([vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                  ctypes.POINTER(ctypes.c_int32)], st),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status, what):
    if status != OK:
        raise EnoaoError(status, what)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, shape=None, what="state"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a GPU torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{what} must be contiguous float64")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def enoao_status_string(status) -> str:
    return lib().enoao_status_string(int(status)).decode()


class Plan:
    def __init__(self, handle, problem):
        self.handle = handle
        self.problem = problem

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().enoao_plan_destroy(self.handle)
            except Exception:  # noqa: BLE001 (interpreter shutdown)
                pass
            self.handle = None


class Batch:
    def __init__(self, handle, problems):
        self.handle = handle
        self.problems = problems

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().enoao_batch_destroy(self.handle)
            except Exception:  # noqa: BLE001
                pass
            self.handle = None


def enoao_workspace_bytes(problem: Problem) -> int:
    return lib().enoao_workspace_bytes(ctypes.byref(problem))


def enoao_plan_create(problem: Problem, stream=None) -> Plan:
    h = ctypes.c_void_p()
    _check(lib().enoao_plan_create(ctypes.byref(problem), _stream(stream), ctypes.byref(h)), "enoao_plan_create")
    return Plan(h, problem)


def enoao_plan_destroy(plan: Plan):
    if plan.handle:
        _check(lib().enoao_plan_destroy(plan.handle), "enoao_plan_destroy")
        plan.handle = None


def enoao_rhs(plan: Plan, u, L, stream=None):
    shape = plan.problem.shape
    _check(lib().enoao_rhs(plan.handle, _dev_ptr(u, shape), _dev_ptr(L, shape, "L"), _stream(stream)), "enoao_rhs")


def enoao_step(plan: Plan, u, dt, stream=None):
    _check(lib().enoao_step(plan.handle, _dev_ptr(u, plan.problem.shape), float(dt), _stream(stream)), "enoao_step")


def enoao_solve(plan: Plan, u, t_final, cfl=0.0, dt_fixed=0.0, max_steps=1 << 62, stream=None):
    """Returns (t reached, steps taken)."""
    t = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().enoao_solve(plan.handle, _dev_ptr(u, plan.problem.shape), float(t_final), float(cfl),
                             float(dt_fixed), int(max_steps), ctypes.byref(t), ctypes.byref(n),
                             _stream(stream)), "enoao_solve")
    return t.value, n.value


def enoao_step_noalloc(problem: Problem, u, dt, stream=None):
    """One step of `problem` on u in place, in the library's per-device scratch array."""
    _check(lib().enoao_step_noalloc(ctypes.byref(problem), _dev_ptr(u, problem.shape), float(dt),
                                    _stream(stream)), "enoao_step_noalloc")


def enoao_plan_check(plan: Plan, stream=None):
    _check(lib().enoao_plan_check(plan.handle, _stream(stream)), "enoao_plan_check")


def enoao_selection_size(plan: Plan) -> int:
    return lib().enoao_selection_size(plan.handle)


def enoao_get_selection(plan: Plan, stream=None) -> np.ndarray:
    n = enoao_selection_size(plan)
    out = np.zeros(n, np.uint8)
    _check(lib().enoao_get_selection(plan.handle, out.ctypes.data_as(ctypes.c_void_p), n, _stream(stream)),
           "enoao_get_selection")
    return out


def enoao_get_step_selection(plan: Plan, stream=None) -> np.ndarray:
    """the three stage records of the last step, stage 1 first (3 * enoao_selection_size)"""
    n = 3 * enoao_selection_size(plan)
    out = np.zeros(n, np.uint8)
    _check(lib().enoao_get_step_selection(plan.handle, out.ctypes.data_as(ctypes.c_void_p), n, _stream(stream)),
           "enoao_get_step_selection")
    return out


def enoao_batch_create(problems, stream=None) -> Batch:
    arr = (Problem * len(problems))(*problems)
    h = ctypes.c_void_p()
    _check(lib().enoao_batch_create(arr, len(problems), _stream(stream), ctypes.byref(h)), "enoao_batch_create")
    return Batch(h, list(problems))


def enoao_batch_destroy(batch: Batch):
    if batch.handle:
        _check(lib().enoao_batch_destroy(batch.handle), "enoao_batch_destroy")
        batch.handle = None


def enoao_batch_step(batch: Batch, states, nsteps, cfl, t_final=None, stream=None):
    ptrs = (ctypes.c_void_p * len(states))(*[_dev_ptr(u, p.shape).value for u, p in zip(states, batch.problems)])
    tf = None
    if t_final is not None:
        tf = (ctypes.c_double * len(states))(*[float(x) for x in t_final])
    _check(lib().enoao_batch_step(batch.handle, ptrs, int(nsteps), float(cfl), tf, _stream(stream)),
           "enoao_batch_step")


def enoao_batch_reset(batch: Batch, stream=None):
    _check(lib().enoao_batch_reset(batch.handle, _stream(stream)), "enoao_batch_reset")


def enoao_batch_query(batch: Batch, stream=None, raise_on_failure=False):
    """(times, step counts, member status flags) as numpy arrays."""
    n = len(batch.problems)
    t = (ctypes.c_double * n)()
    s = (ctypes.c_int64 * n)()
    f = (ctypes.c_int32 * n)()
    st = lib().enoao_batch_query(batch.handle, t, s, f, _stream(stream))
    if st not in (OK, ENONPHYSICAL) or (raise_on_failure and st != OK):
        _check(st, "enoao_batch_query")
    return np.array(t[:]), np.array(s[:]), np.array(f[:])


PROFILE_KINDS = ("sweep_x_s1", "sweep_x_s2", "sweep_x_s3", "sweep_y_s1", "sweep_y_s2", "sweep_y_s3",
                 "step_control", "state_maxima", "resident", "coop")


def enoao_profile(plan: Plan, enable: bool):
    _check(lib().enoao_profile(plan.handle, 1 if enable else 0), "enoao_profile")


def enoao_profile_read(plan: Plan, stream=None):
    """{kind: (mean ms, launches)} of the kernels timed since enoao_profile(plan, True)."""
    n = len(PROFILE_KINDS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().enoao_profile_read(plan.handle, ms, cnt, n, _stream(stream)), "enoao_profile_read")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PROFILE_KINDS)}


def enoao_batch_profile(batch: Batch, enable: bool):
    _check(lib().enoao_batch_profile(batch.handle, 1 if enable else 0), "enoao_batch_profile")


def enoao_batch_profile_read(batch: Batch, stream=None):
    n = len(PROFILE_KINDS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().enoao_batch_profile_read(batch.handle, ms, cnt, n, _stream(stream)), "enoao_batch_profile_read")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PROFILE_KINDS)}


def enoao_set_resident(enable: bool):
    _check(lib().enoao_set_resident(1 if enable else 0), "enoao_set_resident")


def enoao_set_coop(enable: bool):
    _check(lib().enoao_set_coop(1 if enable else 0), "enoao_set_coop")


def enoao_set_shortcut(enable: bool):
    _check(lib().enoao_set_shortcut(1 if enable else 0), "enoao_set_shortcut")


def enoao_set_launch(workgroups_per_cu: int):
    _check(lib().enoao_set_launch(int(workgroups_per_cu), 0), "enoao_set_launch")


def enoao_plan_set_launch(plan: Plan, workgroups_per_cu: int):
    _check(lib().enoao_plan_set_launch(plan.handle, int(workgroups_per_cu)), "enoao_plan_set_launch")


def enoao_batch_set_launch(batch: Batch, workgroups_per_cu: int):
    _check(lib().enoao_batch_set_launch(batch.handle, int(workgroups_per_cu)), "enoao_batch_set_launch")


def _kinds(workgroups_per_cu):
    vals = [int(w) for w in workgroups_per_cu]
    return (ctypes.c_int32 * max(len(vals), 1))(*vals), len(vals)


def enoao_plan_set_launch_kinds(plan: Plan, workgroups_per_cu):
    """Workgroups per CU per kernel kind (x-sweep stages 1..3, y-sweep stages 1..3; 0 = uniform)."""
    arr, n = _kinds(workgroups_per_cu)
    _check(lib().enoao_plan_set_launch_kinds(plan.handle, arr, n), "enoao_plan_set_launch_kinds")


def enoao_batch_set_launch_kinds(batch: Batch, workgroups_per_cu):
    arr, n = _kinds(workgroups_per_cu)
    _check(lib().enoao_batch_set_launch_kinds(batch.handle, arr, n), "enoao_batch_set_launch_kinds")


def enoao_plan_set_tiles(plan: Plan, y_strip_columns: int, stream=None):
    _check(lib().enoao_plan_set_tiles(plan.handle, int(y_strip_columns), _stream(stream)), "enoao_plan_set_tiles")


def enoao_batch_set_tiles(batch: Batch, y_strip_columns: int, stream=None):
    _check(lib().enoao_batch_set_tiles(batch.handle, int(y_strip_columns), _stream(stream)), "enoao_batch_set_tiles")


class Pool:
    def __init__(self, handle, like, max_members):
        self.handle = handle
        self.like = like
        self.max_members = max_members
        self.members = {}  # slot -> Problem of the admitted member (shape checks at retire)

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().enoao_pool_destroy(self.handle)
            except Exception:  # noqa: BLE001
                pass
            self.handle = None


def enoao_pool_member_bytes(problem: Problem) -> int:
    return lib().enoao_pool_member_bytes(ctypes.byref(problem))


def enoao_pool_create(like: Problem, max_members: int, arena_bytes: int, stream=None) -> Pool:
    h = ctypes.c_void_p()
    _check(lib().enoao_pool_create(ctypes.byref(like), int(max_members), int(arena_bytes), _stream(stream),
                                   ctypes.byref(h)), "enoao_pool_create")
    return Pool(h, like, int(max_members))


def enoao_pool_destroy(pool: Pool):
    if pool.handle:
        _check(lib().enoao_pool_destroy(pool.handle), "enoao_pool_destroy")
        pool.handle = None


def enoao_pool_set_launch(pool: Pool, workgroups_per_cu: int):
    _check(lib().enoao_pool_set_launch(pool.handle, int(workgroups_per_cu)), "enoao_pool_set_launch")


def enoao_pool_admit(pool: Pool, problem: Problem, u0, t_final=1e300, max_steps=1 << 62, cfl=0.3, stream=None):
    """Admit a member; u0 is a numpy array (copied from host) or a GPU tensor.  Returns the
    slot, or None when the pool has no room now (ENOMEM)."""
    slot = ctypes.c_int32()
    if isinstance(u0, np.ndarray):
        a = np.ascontiguousarray(u0, dtype=np.float64)
        if a.shape != problem.shape:
            raise ValueError(f"u0 has shape {a.shape}, expected {problem.shape}")
        st = lib().enoao_pool_admit(pool.handle, ctypes.byref(problem), a.ctypes.data_as(ctypes.c_void_p), 1,
                                    float(t_final), int(max_steps), float(cfl), ctypes.byref(slot), _stream(stream))
    else:
        st = lib().enoao_pool_admit(pool.handle, ctypes.byref(problem), _dev_ptr(u0, problem.shape), 0,
                                    float(t_final), int(max_steps), float(cfl), ctypes.byref(slot), _stream(stream))
    if st == ENOMEM:
        return None
    if st == OK:
        pool.members[slot.value] = problem
    _check(st, "enoao_pool_admit")
    return slot.value


def enoao_pool_step(pool: Pool, nsteps=1, stream=None):
    _check(lib().enoao_pool_step(pool.handle, int(nsteps), _stream(stream)), "enoao_pool_step")


def enoao_pool_poll(pool: Pool, stream=None):
    """(done, status, steps, t) per slot as numpy arrays (done = -1 for a free slot)."""
    n = pool.max_members
    d = (ctypes.c_int32 * n)()
    f = (ctypes.c_int32 * n)()
    s = (ctypes.c_int64 * n)()
    t = (ctypes.c_double * n)()
    _check(lib().enoao_pool_poll(pool.handle, d, f, s, t, n, _stream(stream)), "enoao_pool_poll")
    return np.array(d[:]), np.array(f[:]), np.array(s[:]), np.array(t[:])


def enoao_pool_retire(pool: Pool, slot: int, shape=None, out=None, stream=None):
    """Free a member.  With `shape` (and no `out`) its state is returned as a numpy array;
    `out` may be a GPU tensor to receive it on the device.  The library copies the
    member's whole state, so `out` and `shape` must match the admitted problem's
    (ncomp, ny, nx): anything else raises ValueError before the call."""
    prob = pool.members.get(int(slot))
    if prob is None:
        raise ValueError(f"slot {slot} holds no admitted member")
    if out is not None:
        ptr = _dev_ptr(out, prob.shape, what="out")
        _check(lib().enoao_pool_retire(pool.handle, int(slot), ptr, 0, _stream(stream)), "enoao_pool_retire")
        del pool.members[int(slot)]
        return out
    if shape is not None:
        if tuple(shape) != tuple(prob.shape):
            raise ValueError(f"shape {tuple(shape)} does not match the member's {tuple(prob.shape)}")
        a = np.empty(prob.shape, np.float64)
        _check(lib().enoao_pool_retire(pool.handle, int(slot), a.ctypes.data_as(ctypes.c_void_p), 1, _stream(stream)),
               "enoao_pool_retire")
        del pool.members[int(slot)]
        return a
    _check(lib().enoao_pool_retire(pool.handle, int(slot), None, 1, _stream(stream)), "enoao_pool_retire")
    del pool.members[int(slot)]
    return None


def enoao_pool_retire_async(pool: Pool, slot: int, out=None, info=None, stream=None):
    """Free a member without synchronising: the copy of its state to `out` (a GPU
    tensor of the member's shape, or None) and of its progress to `info` (a GPU
    float64 tensor of 4 elements: done, status, steps, t; or None) are enqueued on
    the stream; the slot and its arena space are free at once (later admissions on
    the same stream reuse them after this work)."""
    prob = pool.members.get(int(slot))
    if prob is None:
        raise ValueError(f"slot {slot} holds no admitted member")
    optr = _dev_ptr(out, prob.shape, what="out") if out is not None else None
    iptr = _dev_ptr(info, (4,), what="info") if info is not None else None
    _check(lib().enoao_pool_retire_async(pool.handle, int(slot), optr, iptr, _stream(stream)),
           "enoao_pool_retire_async")
    del pool.members[int(slot)]
    return out


def enoao_pool_usage(pool: Pool):
    """(arena bytes used, arena bytes total, members)."""
    u = ctypes.c_size_t()
    t = ctypes.c_size_t()
    m = ctypes.c_int32()
    _check(lib().enoao_pool_usage(pool.handle, ctypes.byref(u), ctypes.byref(t), ctypes.byref(m)), "enoao_pool_usage")
    return u.value, t.value, m.value
