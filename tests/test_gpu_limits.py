"""Problems at the size limits, checked on sampled cells.

The oracle cannot evaluate these grids whole, so each check takes the window of
the input around a sampled cell (wrapping periodically) as a small problem with
zero-gradient ends and compares the cells far enough from the window's ends that
the ends cannot reach them: G nodes for one evaluation of L, 3G for an SSP-RK3
step (three evaluations).  That is exact only when the Lax-Friedrichs alpha of
the window equals the full grid's (Section 2's global splitting):
  * advection: alpha = |a| whatever the data;
  * Euler 2D, one evaluation of L: the data repeat with period 24 in both
    directions, so every window of 49 x 49 cells holds all the grid's values (a
    49-wide window split by the periodic seam keeps 25 consecutive cells on one
    side) and the per-field maxima are the grid's.  Later stages take alpha from
    the stage states, which the seam makes differ, so steps are checked another
    way: on a grid whose extents are multiples of the period, the solution stays
    periodic and equals, node by node, that of the 24 x 24 periodic problem.
The grid spacing is 1 in both setups (domain [0, n)), so the windows' spacing
is bitwise the grid's.  Every compared cell is compared: the windows are checked to
hold no face the oracle flags as a near tie (the GPU's selection records of these
grids are not copied out, so a tie could not be replayed), and the data are chosen so
that they hold none.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import parity as PT

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

W = 24  # window half width: 2W + 1 cells per direction


def _E():
    from paper_2108_12742_amd import enoao as E
    return E


def _assert_tie_free(p, tie, what):
    assert not (np.asarray(tie) != 0).any(), f"{what}: the oracle flags a near tie in the window"


def _compare_windows(got, ref, radius, what):
    """got/ref: lists of (nc, ny, nx) windows; compares the cells whose distance from
    every window end exceeds radius, to the parity tolerance of the whole set."""
    g = np.stack(got)
    r = np.stack(ref)
    sl = [slice(None), slice(None)] + [slice(radius + 1, n - radius - 1) if n > 1 else slice(None)
                                       for n in g.shape[2:]]
    g, r = g[tuple(sl)], r[tuple(sl)]
    # components first, for the helper's per-component scale
    g = np.moveaxis(g, 1, 0)
    r = np.moveaxis(r, 1, 0)
    PT.assert_close_by_component(g, r, what=what)


def _samples_1d(n, rng, k=24):
    fixed = [0, 1, 5, 62, 63, 64, 126, 1 << 20, n // 2, n - 64, n - 63, n - 2, n - 1]
    return sorted(set(fixed + [int(v) for v in rng.integers(0, n, k)]))


@pytest.mark.parametrize("order", [5, 7])
def test_advection_at_max_extent(order):
    """1D advection with nx = ENOAO_MAX_EXTENT (2^31 - 1024 nodes, 16 GiB per state):
    L and one SSP-RK3 step on sampled windows, including both ends of the periodic grid."""
    torch = PT.torch_cuda()
    E = _E()
    n = E.MAX_EXTENT
    free, _ = torch.cuda.mem_get_info()
    need = 5 * n * 8 + (8 << 30)
    if free < need:
        pytest.skip(f"needs {need >> 30} GiB of free device memory, {free >> 30} GiB free")
    print(f"advection n = {n}, order {order}: building input", flush=True)
    u = torch.arange(n, dtype=torch.float64, device="cuda")
    r = torch.remainder(u, 777.0)
    u.mul_(2.0 * np.pi / 1000.0).sin_()
    u.add_((r < 388.5).to(torch.float64))
    del r
    u = u.view(1, 1, n)
    ep = E.make_problem("advection", n, order=order, x_lo=0.0, x_hi=float(n))
    plan = E.enoao_plan_create(ep)
    L = torch.empty_like(u)
    print("rhs ...", flush=True)
    E.enoao_rhs(plan, u, L)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    samples = _samples_1d(n, rng)
    idx = [torch.tensor([(s + k) % n for k in range(-W, W + 1)], device="cuda") for s in samples]
    uw = [u[0, 0, i].cpu().numpy().reshape(1, 1, -1) for i in idx]
    Lw = [L[0, 0, i].cpu().numpy().reshape(1, 1, -1) for i in idx]
    del L
    op = O.Problem(O.ADVECTION, nx=2 * W + 1, order=order, x_lo=0.0, x_hi=float(2 * W + 1),
                   bc_x=O.TRANSMISSIVE)
    G = 4 if order == 5 else 5
    ref = []
    for s, w in zip(samples, uw):
        Lr, _, tie = O.rhs(op, w, with_selection=True)
        _assert_tie_free(op, tie, f"window at {s}")
        ref.append(Lr)
    _compare_windows(Lw, ref, G, "L on sampled windows")
    print("step ...", flush=True)
    dt = 0.4
    E.enoao_step(plan, u, dt)
    torch.cuda.synchronize()
    got = [u[0, 0, i].cpu().numpy().reshape(1, 1, -1) for i in idx]
    _compare_windows(got, [O.step(op, w, dt) for w in uw], 3 * G, "u after one step on sampled windows")


def _euler_table(period=24, seed=3):
    """Conserved variables (4, period, period) of a smooth field with a discontinuous
    block: positive density and pressure, |velocity| < 0.8."""
    rng = np.random.default_rng(seed)
    a = 2.0 * np.pi * np.arange(period) / period
    X, Y = np.meshgrid(a, a)  # X varies along x (columns), Y along y (rows)
    ph = rng.uniform(0.0, 2.0 * np.pi, 6)
    block = ((np.arange(period)[None, :] < 11) & (np.arange(period)[:, None] < 15)).astype(float)
    rho = 1.0 + 0.3 * np.sin(X + ph[0]) * np.cos(Y + ph[1]) + 0.8 * block
    vx = 0.4 * np.sin(Y + ph[2]) + 0.2 * block
    vy = 0.4 * np.cos(X + ph[3]) - 0.3 * block
    p = 1.0 + 0.25 * np.cos(X + Y + ph[4]) + 1.5 * block
    E_ = p / 0.4 + 0.5 * rho * (vx * vx + vy * vy)
    return np.stack([rho, rho * vx, rho * vy, E_])


@pytest.mark.parametrize("order", [5, 7])
def test_euler2d_beyond_32bit_planes_rhs(order):
    """2D Euler on 30000 x 24003 nodes: 3 * nx * ny > 2^31, so the offsets of the last
    conserved variables exceed 32 bits, and both extents leave ragged tiles.  L on
    sampled windows (corners, the periodic seam in y, interior)."""
    torch = PT.torch_cuda()
    E = _E()
    nx, ny, P = 30000, 24003, 24
    free, _ = torch.cuda.mem_get_info()
    need = 6 * 4 * nx * ny * 8 + (8 << 30)
    if free < need:
        pytest.skip(f"needs {need >> 30} GiB of free device memory, {free >> 30} GiB free")
    print(f"euler2d {nx}x{ny}, order {order}: building input", flush=True)
    u = _tiled_state(torch, nx, ny, P)
    ep = E.make_problem("euler2d", nx, ny, order=order, x_lo=0.0, x_hi=float(nx), y_lo=0.0, y_hi=float(ny))
    plan = E.enoao_plan_create(ep)
    L = torch.empty_like(u)
    print("rhs ...", flush=True)
    E.enoao_rhs(plan, u, L)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    pts = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (ny // 2, nx // 2), (7, nx - 20), (ny - 9, 31)]
    pts += [(int(a), int(b)) for a, b in zip(rng.integers(0, ny, 6), rng.integers(0, nx, 6))]

    def window(t, y, x):
        rows = torch.tensor([(y + k) % ny for k in range(-W, W + 1)], device="cuda")
        cols = torch.tensor([(x + k) % nx for k in range(-W, W + 1)], device="cuda")
        return t[:, rows][:, :, cols].cpu().numpy()

    uw = [window(u, y, x) for y, x in pts]
    Lw = [window(L, y, x) for y, x in pts]
    m = 2 * W + 1
    op = O.Problem(O.EULER2D, nx=m, ny=m, order=order, x_lo=0.0, x_hi=float(m), y_lo=0.0, y_hi=float(m),
                   bc_x=O.TRANSMISSIVE, bc_y=O.TRANSMISSIVE)
    G = 4 if order == 5 else 5
    ref = []
    for pt, w in zip(pts, uw):
        Lr, _, tie = O.rhs(op, w, with_selection=True)
        _assert_tie_free(op, tie, f"window at {pt}")
        ref.append(Lr)
    _compare_windows(Lw, ref, G, "L on sampled windows")


def _tiled_state(torch, nx, ny, period):
    tab = torch.from_numpy(_euler_table(period)).cuda()
    ii = torch.arange(nx, device="cuda") % period
    jj = torch.arange(ny, device="cuda") % period
    return tab[:, jj][:, :, ii].contiguous()


def _assert_tiles(torch, t, ref, what, rows_per_chunk=1024):
    """Every node of t (nc, ny, nx) on the device against ref (nc, P, P) tiled over the grid,
    to the parity tolerance (per component, relative to the component's largest value)."""
    nc, ny, nx = t.shape
    period = ref.shape[1]
    refd = torch.from_numpy(np.ascontiguousarray(ref)).cuda()
    ii = torch.arange(nx, device="cuda") % period
    for q in range(nc):
        scale = float(np.abs(ref[q]).max())
        worst = 0.0
        for r0 in range(0, ny, rows_per_chunk):
            r1 = min(r0 + rows_per_chunk, ny)
            rows = torch.arange(r0, r1, device="cuda") % period
            d = (t[q, r0:r1] - refd[q][rows][:, ii]).abs().max().item()
            assert np.isfinite(d), f"{what}[{q}]: non-finite values in rows {r0}..{r1}"
            worst = max(worst, d)
        assert worst <= PT.RTOL * scale, f"{what}[{q}]: max |diff| {worst:.3e} > {PT.RTOL:.0e} * {scale:.3e}"


@pytest.mark.parametrize("order", [5, 7])
def test_euler2d_beyond_32bit_planes_periodic_tiling(order):
    """2D Euler on 30000 x 24000 nodes tiled by a 24 x 24 pattern (3 * nx * ny > 2^31; the
    x extent leaves ragged tiles): the periodic grid evolves exactly like the 24 x 24
    periodic problem, so every node of L, of one fixed-dt step and of two CFL-controlled
    steps is checked against the oracle's solution of that small problem."""
    torch = PT.torch_cuda()
    E = _E()
    nx, ny, P = 30000, 24000, 24
    free, _ = torch.cuda.mem_get_info()
    need = 6 * 4 * nx * ny * 8 + (8 << 30)
    if free < need:
        pytest.skip(f"needs {need >> 30} GiB of free device memory, {free >> 30} GiB free")
    tab = _euler_table(P)
    op = O.Problem(O.EULER2D, nx=P, ny=P, order=order, x_lo=0.0, x_hi=float(P), y_lo=0.0, y_hi=float(P))
    Lr, _, tie = O.rhs(op, tab, with_selection=True)
    _assert_tie_free(op, tie, "24 x 24 pattern")
    dt = 0.1
    ur = O.step(op, tab, dt)
    us, ts, ns = O.solve(op, tab, 1e30, cfl=0.3, max_steps=2)
    print(f"euler2d {nx}x{ny}, order {order}: building input", flush=True)
    u = _tiled_state(torch, nx, ny, P)
    ep = E.make_problem("euler2d", nx, ny, order=order, x_lo=0.0, x_hi=float(nx), y_lo=0.0, y_hi=float(ny))
    plan = E.enoao_plan_create(ep)
    L = torch.empty_like(u)
    print("rhs ...", flush=True)
    E.enoao_rhs(plan, u, L)
    torch.cuda.synchronize()
    _assert_tiles(torch, L, Lr, "L")
    del L
    print("step ...", flush=True)
    u2 = u.clone()
    E.enoao_step(plan, u2, dt)
    torch.cuda.synchronize()
    _assert_tiles(torch, u2, ur, "u after one step")
    del u2
    print("solve ...", flush=True)
    t, n = E.enoao_solve(plan, u, 1e30, cfl=0.3, max_steps=2)
    torch.cuda.synchronize()
    assert n == ns == 2 and abs(t / ts - 1) <= 1e-14
    _assert_tiles(torch, u, us, "u after two CFL steps")
    E.enoao_plan_check(plan)
