"""The kernels evaluate the candidate fluxes of the table of numerical fluxes in Newton
form on the undivided-difference table: each candidate's row is a lower candidate's row
plus a rational multiple of one undivided difference.  These identities are checked here
exactly (rational arithmetic) against the rows re-derived from the polynomial
reconstruction of Section 3.1, so the GPU's flux arithmetic is pinned independently of
the oracle's literal rows."""
from fractions import Fraction as Fr
from math import comb

import pytest

from tests.exact_recon import flux_coefficients

# (candidate, parent, difference level, first node of the difference, multiplier);
# nodes are window positions, f_j = window[H]
NEWTON = {
    5: [(1, 0, 1, 3, Fr(1, 2)), (2, 1, 2, 2, Fr(-1, 6)), (3, 2, 3, 1, Fr(-1, 12)),
        (4, 2, 3, 2, Fr(-1, 12)), (5, 3, 4, 1, Fr(-1, 20))],
    7: [(1, 0, 1, 4, Fr(1, 2)), (2, 1, 2, 3, Fr(-1, 6)), (3, 2, 3, 2, Fr(-1, 12)),
        (4, 2, 3, 3, Fr(-1, 12)), (5, 3, 4, 2, Fr(-1, 20)), (6, 5, 5, 1, Fr(1, 60)),
        (7, 5, 5, 2, Fr(1, 60)), (8, 6, 6, 1, Fr(1, 105))],
}
STENCILS = {5: [(0, 0), (0, 1), (1, 1), (2, 1), (1, 2), (2, 2)],
            7: [(0, 0), (0, 1), (1, 1), (2, 1), (1, 2), (2, 2), (3, 2), (2, 3), (3, 3)]}


def _half(order):
    return order // 2 + 1  # window f_{j-H} .. f_{j+H}


def _row(order, m, n):
    H = _half(order)
    r = [Fr(0)] * (2 * H + 1)
    for i, v in enumerate(flux_coefficients(m, n)):
        r[H - m + i] = v
    return r


def _difference(order, level, first):
    v = [Fr(0)] * (2 * _half(order) + 1)
    for q in range(level + 1):
        v[first + q] = Fr((-1) ** (level - q) * comb(level, q))
    return v


@pytest.mark.parametrize("order", [5, 7])
def test_newton_form_equals_flux_rows(order):
    rows = [_row(order, m, n) for m, n in STENCILS[order]]
    H = _half(order)
    assert rows[0] == [Fr(int(i == H)) for i in range(2 * H + 1)]
    built = {0: rows[0]}
    for k, parent, level, first, mult in NEWTON[order]:
        d = _difference(order, level, first)
        built[k] = [a + mult * b for a, b in zip(built[parent], d)]
        assert built[k] == rows[k], (order, k)
    assert sorted(built) == list(range(len(rows)))


# The kernels evaluate the top candidate (S_{j-2}^{j+2}, order 7: S_{j-3}^{j+3}) of both
# sides of a face in conserved-variable form: its indicators come from (2H-1)-th
# undivided differences D_p of the face's 2H+2 nodes, and the sum of its two one-sided
# values from a symmetric stencil S plus kappa D_1 (Section 3.2's candidate rows, split
# as in Section 2).  The constants below are the kernels'; they are checked exactly
# against the polynomial definition of Section 3.1 on random rational data.
def _top_d(order, x, p):
    if order == 5:
        return (x[p + 5] - x[p]) + 5 * (x[p + 1] - x[p + 4]) + 10 * (x[p + 3] - x[p + 2])
    return (x[p + 7] - x[p]) + 7 * (x[p + 1] - x[p + 6]) + 21 * (x[p + 5] - x[p + 2]) + 35 * (x[p + 3] - x[p + 4])


def _top_s(order, x):
    H = _half(order)
    s = [x[H - k] + x[H + 1 + k] for k in range(H)]
    if order == 5:
        return s[0] + Fr(-7, 30) * (s[1] - s[0]) + Fr(1, 30) * (s[2] - s[1])
    return (s[0] + Fr(-113, 420) * (s[1] - s[0]) + Fr(13, 210) * (s[2] - s[1])
            + Fr(-1, 140) * (s[3] - s[2]))


TOP_KAPPA = {5: Fr(-1, 30), 7: Fr(1, 140)}


@pytest.mark.parametrize("order", [5, 7])
def test_top_candidate_conserved_form(order):
    import random
    from tests.exact_recon import indicator
    H = _half(order)
    rng = random.Random(order)
    for _ in range(25):
        F = [Fr(rng.randint(-60, 60), rng.randint(1, 7)) for _ in range(2 * H + 2)]
        U = [Fr(rng.randint(-60, 60), rng.randint(1, 7)) for _ in range(2 * H + 2)]
        a = Fr(rng.randint(1, 40), rng.randint(1, 9))
        # split windows: plus side nodes 0 .. 2H, minus side the mirror 2H+1 .. 1
        gp = [F[t] + a * U[t] for t in range(2 * H + 1)]
        gm = [F[2 * H + 1 - k] - a * U[2 * H + 1 - k] for k in range(2 * H + 1)]
        hp, ip = indicator(H - 1, H - 1, gp, H)
        hm, im = indicator(H - 1, H - 1, gm, H)
        d = [(_top_d(order, F, p), _top_d(order, U, p)) for p in range(3)]
        assert ip == min(abs(d[0][0] + a * d[0][1]), abs(d[1][0] + a * d[1][1]))
        assert im == min(abs(d[2][0] - a * d[2][1]), abs(d[1][0] - a * d[1][1]))
        assert hp + hm == _top_s(order, F) + a * TOP_KAPPA[order] * d[1][1]


@pytest.mark.parametrize("order", [5, 7])
def test_top_form_constant_data(order):
    # constant data: every difference and every correction of S is exactly zero in
    # floating point too, so a uniform state gives bitwise equal fluxes at every face
    H = _half(order)
    for c in (0.1, 1.0 / 3.0, 7.25e3):
        x = [c] * (2 * H + 2)
        assert all(_top_d(order, x, p) == 0.0 for p in range(3))
        s = [x[H - k] + x[H + 1 + k] for k in range(H)]
        assert all(s[k + 1] - s[k] == 0.0 for k in range(H - 1))
