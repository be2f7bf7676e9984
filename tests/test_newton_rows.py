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
