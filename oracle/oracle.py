"""ctypes binding of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py; never by the product package.

States are numpy float64 arrays of shape (ncomp, ny, nx) (1D: (ncomp, 1, nx)),
C-contiguous, over the grid nodes x_i = x_lo + i*dx.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ADVECTION, EULER1D, EULER2D = 0, 1, 2
PERIODIC, TRANSMISSIVE = 0, 1
CHAR_ROE, COMPONENT = 0, 1  # reconstruction variables of the Euler systems
MISMATCH = 7  # status of a replayed selection outside the oracle's tie set
NCOMP = {ADVECTION: 1, EULER1D: 3, EULER2D: 4}


class _Problem(ctypes.Structure):
    _fields_ = [
        ("equation", ctypes.c_int32), ("order", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
        ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("adv_speed", ctypes.c_double), ("delta", ctypes.c_double),
        ("recon_vars", ctypes.c_int32),
    ]


@dataclass
class Problem:
    equation: int
    nx: int
    ny: int = 1
    order: int = 5
    x_lo: float = -1.0
    x_hi: float = 1.0
    y_lo: float = -1.0
    y_hi: float = 1.0
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    gamma: float = 1.4
    adv_speed: float = 1.0
    delta: float = 1e-5
    recon_vars: int = 0  # CHAR_ROE or COMPONENT

    @property
    def ncomp(self):
        return NCOMP[self.equation]

    @property
    def shape(self):
        return (self.ncomp, self.ny, self.nx)

    @property
    def dx(self):
        return (self.x_hi - self.x_lo) / self.nx

    @property
    def dy(self):
        return (self.y_hi - self.y_lo) / self.ny

    def c_struct(self):
        return _Problem(self.equation, self.order, self.nx, self.ny, self.x_lo, self.x_hi,
                        self.y_lo, self.y_hi, self.bc_x, self.bc_y, self.gamma,
                        self.adv_speed, self.delta, self.recon_vars)


class OracleError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle  # noqa: WPS433 (build on first use)
            build_oracle.build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        pp = ctypes.POINTER(_Problem)
        L.ref_num_candidates.argtypes = [ctypes.c_int]
        L.ref_candidates.argtypes = [ctypes.c_int, dp, dp, dp]
        L.ref_reconstruct.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, dp, ip, ip]
        L.ref_reconstruct_replay.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int, dp, ip, ip,
                                             ctypes.POINTER(ctypes.c_uint)]
        L.ref_indicator_scales.argtypes = [ctypes.c_int, dp, dp, dp]
        L.ref_euler_flux.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.ref_roe_eigen.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp, dp]
        L.ref_selection_size.argtypes = [pp]
        L.ref_selection_size.restype = ctypes.c_int64
        L.ref_alpha.argtypes = [pp, dp, dp, dp]
        L.ref_rhs.argtypes = [pp, dp, dp, u8, u8]
        L.ref_step.argtypes = [pp, dp, ctypes.c_double]
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.ref_rhs_replay.argtypes = [pp, dp, dp, u8, u8, u8, i64p]
        L.ref_step_replay.argtypes = [pp, dp, ctypes.c_double, u8, i64p]
        L.ref_dt.argtypes = [pp, dp, ctypes.c_double, dp]
        L.ref_solve.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int64, dp, ctypes.POINTER(ctypes.c_int64)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what}: oracle status {st}")


def num_candidates(order):
    return lib().ref_num_candidates(order)


def candidates(order, f):
    """All candidates' fluxes at x_{j+1/2} and indicators, for window f (len 2h+1)."""
    f = _f64(f)
    K = num_candidates(order)
    flux = np.zeros(K)
    ind = np.zeros(K)
    _check(lib().ref_candidates(order, _dp(f), _dp(flux), _dp(ind)), "candidates")
    return flux, ind


def reconstruct(order, f, delta=1e-5, mag=None):
    """(fhat, selected candidate, near-tie flag) for one side of one face."""
    f = _f64(f)
    m = None if mag is None else _f64(mag)
    out = ctypes.c_double()
    sel = ctypes.c_int()
    tie = ctypes.c_int()
    _check(lib().ref_reconstruct(order, _dp(f), None if m is None else _dp(m), delta,
                                 ctypes.byref(out), ctypes.byref(sel), ctypes.byref(tie)),
           "reconstruct")
    return out.value, sel.value, tie.value


def reconstruct_replay(order, f, forced, delta=1e-5, mag=None):
    """(fhat, selection, near-tie flag, tie set as a list of candidates, in tie set) for one
    side of one face, taking candidate `forced` when the oracle's tie set holds it."""
    f = _f64(f)
    m = None if mag is None else _f64(mag)
    out = ctypes.c_double()
    sel = ctypes.c_int()
    tie = ctypes.c_int()
    tset = ctypes.c_uint()
    st = lib().ref_reconstruct_replay(order, _dp(f), None if m is None else _dp(m), delta, int(forced),
                                      ctypes.byref(out), ctypes.byref(sel), ctypes.byref(tie),
                                      ctypes.byref(tset))
    if st not in (0, MISMATCH):
        _check(st, "reconstruct_replay")
    K = num_candidates(order)
    return out.value, sel.value, tie.value, [k for k in range(K) if tset.value >> k & 1], st == 0


def indicator_scales(order, f, mag=None):
    """forward-error scale of every candidate's indicator (the near-tie margin's unit)"""
    f = _f64(f)
    m = None if mag is None else _f64(mag)
    out = np.zeros(num_candidates(order))
    _check(lib().ref_indicator_scales(order, _dp(f), None if m is None else _dp(m), _dp(out)), "scales")
    return out


def euler_flux(dim, gamma, U):
    U = _f64(U)
    F = np.zeros_like(U)
    _check(lib().ref_euler_flux(dim, gamma, _dp(U), _dp(F)), "euler_flux")
    return F


def roe_eigen(dim, gamma, UL, UR):
    n = dim + 2
    UL, UR = _f64(UL), _f64(UR)
    R = np.zeros((n, n))
    Lm = np.zeros((n, n))
    lam = np.zeros(n)
    _check(lib().ref_roe_eigen(dim, gamma, _dp(UL), _dp(UR), _dp(R), _dp(Lm), _dp(lam)),
           "roe_eigen")
    return R, Lm, lam


def alpha(p: Problem, u):
    u = _f64(u)
    assert u.shape == p.shape
    ax = np.zeros(4)
    ay = np.zeros(4)
    ps = p.c_struct()
    _check(lib().ref_alpha(ctypes.byref(ps), _dp(u), _dp(ax), _dp(ay)), "alpha")
    return ax[:p.ncomp], ay[:p.ncomp]


def selection_size(p: Problem):
    ps = p.c_struct()
    return lib().ref_selection_size(ctypes.byref(ps))


def split_selection(p: Problem, flat):
    """Views of a flat selection array: x block (ncomp,2,ny,nx+1) [, y block (ncomp,2,ny+1,nx)]."""
    nc = p.ncomp
    nxb = nc * 2 * p.ny * (p.nx + 1)
    xs = flat[:nxb].reshape(nc, 2, p.ny, p.nx + 1)
    if p.equation != EULER2D:
        return xs, None
    ys = flat[nxb:].reshape(nc, 2, p.ny + 1, p.nx)
    return xs, ys


def rhs(p: Problem, u, with_selection=False):
    u = _f64(u)
    assert u.shape == p.shape
    L = np.zeros_like(u)
    ps = p.c_struct()
    if with_selection:
        n = selection_size(p)
        sel = np.zeros(n, np.uint8)
        tie = np.zeros(n, np.uint8)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        _check(lib().ref_rhs(ctypes.byref(ps), _dp(u), _dp(L), sel.ctypes.data_as(u8),
                             tie.ctypes.data_as(u8)), "rhs")
        return L, sel, tie
    _check(lib().ref_rhs(ctypes.byref(ps), _dp(u), _dp(L), None, None), "rhs")
    return L


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def rhs_replay(p: Problem, u, force):
    """L(u) with the selection record `force` (layout of rhs(with_selection=True)) replayed
    wherever the oracle's tie set allows it.  Returns (L, selection, tie flags, number of
    face sides whose forced choice lies outside the tie set)."""
    u = _f64(u)
    assert u.shape == p.shape
    n = selection_size(p)
    force = np.ascontiguousarray(force, dtype=np.uint8).reshape(-1)
    assert force.size == n, (force.size, n)
    L = np.zeros_like(u)
    sel = np.zeros(n, np.uint8)
    tie = np.zeros(n, np.uint8)
    nbad = ctypes.c_int64()
    ps = p.c_struct()
    st = lib().ref_rhs_replay(ctypes.byref(ps), _dp(u), _dp(L), _u8(force), _u8(sel), _u8(tie),
                              ctypes.byref(nbad))
    if st not in (0, MISMATCH):
        _check(st, "rhs_replay")
    return L, sel, tie, nbad.value


def step_replay(p: Problem, u, dt, force):
    """One SSP-RK3 step replaying three stage records `force` (stage 1, 2, 3, each of
    selection_size(p) entries) where the tie sets allow it.  Returns (state, number of
    face sides outside the tie sets over the three stages)."""
    v = _f64(u).copy()
    assert v.shape == p.shape
    n = selection_size(p)
    force = np.ascontiguousarray(force, dtype=np.uint8).reshape(-1)
    assert force.size == 3 * n, (force.size, n)
    nbad = ctypes.c_int64()
    ps = p.c_struct()
    st = lib().ref_step_replay(ctypes.byref(ps), _dp(v), float(dt), _u8(force), ctypes.byref(nbad))
    if st not in (0, MISMATCH):
        _check(st, "step_replay")
    return v, nbad.value


def step(p: Problem, u, dt):
    """One SSP-RK3 step; returns the new state (input untouched)."""
    v = _f64(u).copy()
    assert v.shape == p.shape
    ps = p.c_struct()
    _check(lib().ref_step(ctypes.byref(ps), _dp(v), float(dt)), "step")
    return v


def cfl_dt(p: Problem, u, cfl):
    u = _f64(u)
    out = ctypes.c_double()
    ps = p.c_struct()
    _check(lib().ref_dt(ctypes.byref(ps), _dp(u), float(cfl), ctypes.byref(out)), "dt")
    return out.value


def solve(p: Problem, u, t_final, cfl=0.0, dt_fixed=0.0, max_steps=1 << 40):
    """Advance to t_final; returns (state, t, steps)."""
    v = _f64(u).copy()
    assert v.shape == p.shape
    t = ctypes.c_double()
    n = ctypes.c_int64()
    ps = p.c_struct()
    _check(lib().ref_solve(ctypes.byref(ps), _dp(v), float(t_final), float(cfl), float(dt_fixed),
                           int(max_steps), ctypes.byref(t), ctypes.byref(n)), "solve")
    return v, t.value, n.value
