"""Exact rational polynomial reconstruction from cell averages (test helper).

Independent restatement of the definitions of Section 3.1: on the stencil
S_{j-m}^{j+n} of unit cells I_k = [k - 1/2, k + 1/2] (k relative to j), the
polynomial P of degree m+n whose averages over the stencil's cells equal the
data (Eq. Polynomial_Construction); fhat_{j+1/2} = P(1/2); delta_L / delta_R
= |average of P over the left / right neighbour cell - that cell's average|
(Eq. New_Smoothness_Indicator, the general case).
"""
from fractions import Fraction as Fr


def _cell_moment(k, d):
    """average of x^d over [k - 1/2, k + 1/2]"""
    a, b = Fr(2 * k - 1, 2), Fr(2 * k + 1, 2)
    return (b ** (d + 1) - a ** (d + 1)) / (d + 1)


def _solve(A, rhs):
    n = len(A)
    M = [list(row) + [r] for row, r in zip(A, rhs)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def poly_from_averages(m, n, averages):
    """coefficients a_d (d = 0..m+n) of P with the given averages on cells -m..n"""
    cells = list(range(-m, n + 1))
    A = [[_cell_moment(k, d) for d in range(m + n + 1)] for k in cells]
    return _solve(A, [Fr(v) for v in averages])


def poly_eval(a, x):
    return sum(c * Fr(x) ** d for d, c in enumerate(a))


def poly_cell_average(a, k):
    return sum(c * _cell_moment(k, d) for d, c in enumerate(a))


def flux_coefficients(m, n):
    """exact coefficients of fhat_{j+1/2} on f_{j-m} .. f_{j+n}"""
    out = []
    for i in range(m + n + 1):
        e = [0] * (m + n + 1)
        e[i] = 1
        out.append(poly_eval(poly_from_averages(m, n, e), Fr(1, 2)))
    return out


def indicator(m, n, window, h):
    """exact (fhat, IS) for stencil S_{j-m}^{j+n} from a window f_{j-h} .. f_{j+h} of exact values"""
    f = [Fr(v) for v in window]
    j = h
    if m == 0 and n == 0:
        dL = (abs(f[j] - f[j - 1]) + abs(f[j - 1] - f[j - 2])) / 2
        dR = (abs(f[j] - f[j + 1]) + abs(f[j + 1] - f[j + 2])) / 2
        return f[j], min(dL, dR)
    a = poly_from_averages(m, n, f[j - m:j + n + 1])
    dL = abs(poly_cell_average(a, -m - 1) - f[j - m - 1])
    dR = abs(poly_cell_average(a, n + 1) - f[j + n + 1])
    return poly_eval(a, Fr(1, 2)), min(dL, dR)
