"""Helpers of the GPU parity tests: problem translation, device round trips and the
comparison rules.

Comparison rules (the HIP path against the FP64 oracle):
  * states and L: per component c, max |gpu - oracle| <= RTOL * max |oracle_c|
    (RTOL = 1e-12; a component that is identically zero in the oracle is scaled
    by the largest component instead);
  * stencil selections: identical, except at faces the oracle flags as near
    ties (a deciding comparison within 1e-14 of its rounding scale); there the
    GPU's choice must still be one the oracle could have taken, and the cells
    next to such a face are left out of the value comparison.
"""
import numpy as np
import pytest

from oracle import oracle as O

RTOL = 1e-12


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def oracle_problem(ep):
    """oracle Problem equal to an enoao.Problem"""
    return O.Problem(ep.equation, nx=ep.nx, ny=ep.ny, order=ep.order, x_lo=ep.x_lo, x_hi=ep.x_hi,
                     y_lo=ep.y_lo, y_hi=ep.y_hi, bc_x=ep.bc_x, bc_y=ep.bc_y, gamma=ep.gamma,
                     adv_speed=ep.adv_speed, delta=ep.delta)


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def assert_close_by_component(gpu, ref, mask=None, rtol=RTOL, what="state"):
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
        if mask is not None:
            d = np.where(mask, d, 0.0)
        worst = d.max()
        assert worst <= rtol * scale, (
            f"{what}[{c}]: max |diff| {worst:.3e} > {rtol:.0e} * {scale:.3e} at {np.unravel_index(d.argmax(), d.shape)}")


def compare_selection(p, sel_gpu, sel_ref, tie_ref):
    """Returns a boolean mask (ny, nx) of cells whose value comparison is valid."""
    sel_gpu = np.asarray(sel_gpu)
    diff = sel_gpu != sel_ref
    bad = diff & (tie_ref == 0)
    assert not bad.any(), f"{int(bad.sum())} selection mismatches at non-tie faces (first at flat {np.argmax(bad)})"
    mask = np.ones((p.ny, p.nx), bool)
    if not diff.any():
        return mask
    xs, ys = O.split_selection(p, diff)
    fx = xs.any(axis=(0, 1))  # (ny, nx+1)
    for iy, i in zip(*np.nonzero(fx)):
        for x in (i - 1, i):
            mask[iy, x % p.nx] = False
    if ys is not None:
        fy = ys.any(axis=(0, 1))  # (ny+1, nx)
        for i, ix in zip(*np.nonzero(fy)):
            for y in (i - 1, i):
                mask[y % p.ny, ix] = False
    return mask
