"""Pins of the oracle's single-face reconstruction against the paper and exact arithmetic.

Each test fixes part of the oracle by something other than the oracle itself:
exact rational reconstruction from the definitions of Section 3.1, the paper's
printed modified-wavenumber tables, the paper's candidate lists, and the
reconstruction principle restated from the text of Section 3.2.
"""
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import oracle as O
from tests import exact_recon as X

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _candidate_sets():
    sets = {}
    with open(os.path.join(GOLDEN, "candidate_sets.txt")) as fh:
        for line in fh:
            if line.startswith("#") or ":" not in line:
                continue
            key, val = line.split(":", 1)
            sets[key.strip()] = [tuple(int(t) for t in pair.split()) for pair in val.split(",")]
    return sets


SETS = _candidate_sets()
CANDS = {5: SETS["order5"], 7: SETS["order7"]}
H = {5: 3, 7: 4}


def _wavenumber_rows():
    rows = {}
    with open(os.path.join(GOLDEN, "modified_wavenumbers.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            mn, re_part, im_part = line.split("|")
            m, n = (int(t) for t in mn.split())
            rows[(m, n)] = ([Fr(t) for t in re_part.split()], [Fr(t) for t in im_part.split()])
    return rows


WAVE = _wavenumber_rows()


def _oracle_coefficients(order):
    """Flux coefficients of every oracle candidate, read off with scaled unit windows."""
    h = H[order]
    K = O.num_candidates(order)
    coef = np.zeros((K, 2 * h + 1))
    for q in range(2 * h + 1):
        w = np.zeros(2 * h + 1)
        w[q] = 420.0  # common multiple of every divisor in the flux table: exact
        flux, _ = O.candidates(order, w)
        coef[:, q] = flux / 420.0
    return coef


@pytest.mark.parametrize("order", [5, 7])
def test_candidate_lists(order):
    assert O.num_candidates(order) == len(CANDS[order])


@pytest.mark.parametrize("order", [5, 7])
def test_flux_rows_exact(order):
    """P1: each candidate flux row equals P(x_{j+1/2}) of the exact cell-average polynomial."""
    h = H[order]
    K = O.num_candidates(order)
    for k, (m, n) in enumerate(CANDS[order]):
        exact = X.flux_coefficients(m, n)
        for q in range(2 * h + 1):
            w = [0] * (2 * h + 1)
            w[q] = 420
            flux, _ = O.candidates(order, np.array(w, float))
            off = q - h  # offset of window slot q from j
            want = exact[off + m] * 420 if -m <= off <= n else Fr(0)
            assert Fr(flux[k]) == want, (order, k, q)
    assert K == len(CANDS[order])


@pytest.mark.parametrize("order", [5, 7])
def test_modified_wavenumbers_match_paper(order):
    """P2: the Fourier symbol of each oracle flux row equals the paper's Re/Im tables."""
    h = H[order]
    coef = _oracle_coefficients(order)
    kap = np.linspace(0.0, math.pi, 181)
    for k, (m, n) in enumerate(CANDS[order]):
        offs = np.arange(-h, h + 1)
        sym = (coef[k][None, :] * np.exp(1j * np.outer(kap, offs))).sum(1) * (1 - np.exp(-1j * kap))
        kp = -1j * sym
        re_c, im_c = WAVE[(m, n)]
        re = sum(float(c) * np.sin((i + 1) * kap) for i, c in enumerate(re_c))
        im = float(im_c[0]) + sum(float(c) * np.cos((i + 1) * kap) for i, c in enumerate(im_c[1:]))
        np.testing.assert_allclose(kp.real, re, atol=1e-13)
        np.testing.assert_allclose(kp.imag, im, atol=1e-13)


def test_stability_filter_gives_paper_candidates():
    """A4: the linearly stable stencils of S_{j-3}^{j+3} (Im kappa' <= 0), minus the one
    dropped for dispersion, are exactly the order-7 candidates; those inside S_{j-2}^{j+2}
    are exactly the order-5 candidates.  Symbols from the exact flux rows."""
    kap = np.linspace(1e-3, math.pi, 2000)
    stable = []
    for m in range(4):
        for n in range(4):
            c = [float(v) for v in X.flux_coefficients(m, n)]
            offs = np.arange(-m, n + 1)
            sym = (np.array(c)[None, :] * np.exp(1j * np.outer(kap, offs))).sum(1) * (1 - np.exp(-1j * kap))
            im = (-1j * sym).imag
            if im.max() <= 1e-12:
                stable.append((m, n))
            # and the printed Im table agrees with the exact rows
            _, im_c = WAVE[(m, n)]
            im_tab = float(im_c[0]) + sum(float(v) * np.cos((i + 1) * kap) for i, v in enumerate(im_c[1:]))
            np.testing.assert_allclose(im, im_tab, atol=1e-12)
    dropped = SETS["dropped"]
    assert sorted(set(stable) - set(dropped)) == sorted(CANDS[7])
    assert sorted(s for s in CANDS[7] if s[0] <= 2 and s[1] <= 2) == sorted(CANDS[5])


@pytest.mark.parametrize("order", [5, 7])
def test_indicators_brute_force(order):
    """P3: oracle IS equals the literal definition (exact polynomial integrated over the
    neighbour cells) on integer data, where FP64 is exact."""
    rng = np.random.default_rng(order)
    h = H[order]
    for trial in range(60):
        w = rng.integers(-9, 10, size=2 * h + 1).astype(float)
        flux, ind = O.candidates(order, w)
        for k, (m, n) in enumerate(CANDS[order]):
            fh, is_exact = X.indicator(m, n, [int(v) for v in w], h)
            assert Fr(ind[k]) == is_exact, (trial, k)
            assert abs(flux[k] - float(fh)) <= 1e-15 * (1 + abs(float(fh)))


def _priority(m, n):
    """Text of Section 3.2: higher order first, central before upwind-biased at equal order."""
    return (m + n + 1, 1 if m == n - 1 else 0)


def _rule(IS, order, delta):
    cands = CANDS[order]
    ok = [k for k in range(len(IS)) if IS[k] <= delta]
    if ok:
        return max(ok, key=lambda k: _priority(*cands[k]))
    lo = min(IS)
    return max((k for k in range(len(IS)) if IS[k] == lo), key=lambda k: _priority(*cands[k]))


@pytest.mark.parametrize("order", [5, 7])
def test_selection_rule_integer_data(order):
    """P6/P7: on small integers (exact indicators, frequent exact ties) the oracle's choice
    equals the reconstruction principle restated from the text, applied to exact IS."""
    rng = np.random.default_rng(100 + order)
    h = H[order]
    counts = np.zeros(O.num_candidates(order), int)
    for trial in range(400):
        w = rng.integers(0, 4, size=2 * h + 1).astype(float)
        exact = [X.indicator(m, n, [int(v) for v in w], h) for (m, n) in CANDS[order]]
        IS = [e[1] for e in exact]
        for delta in (0.0, 1e-5, 1.0):
            k = _rule(IS, order, Fr(delta))
            fhat, sel, _ = O.reconstruct(order, w, delta)
            assert sel == k, (trial, delta, w, IS)
            assert abs(fhat - float(exact[k][0])) <= 1e-15 * (1 + abs(fhat))
            counts[sel] += 1
    assert (counts > 0).sum() >= len(counts) - 1  # nearly every candidate exercised


@pytest.mark.parametrize("order", [5, 7])
def test_selection_rule_random_data(order):
    rng = np.random.default_rng(200 + order)
    h = H[order]
    for trial in range(2000):
        scale = 10.0 ** rng.uniform(-7, 1)
        w = scale * rng.standard_normal(2 * h + 1)
        _, ind = O.candidates(order, w)
        _, sel, _ = O.reconstruct(order, w, 1e-5)
        assert sel == _rule(list(ind), order, 1e-5)


@pytest.mark.parametrize("order", [5, 7])
def test_step_data_picks_first_order(order):
    """P5: a jump between j and j+1 leaves S_j^j as the only stencil with IS = 0."""
    h = H[order]
    for jump in (1e-3, 1.0, 1e3):
        w = np.where(np.arange(2 * h + 1) <= h, 2.0, 2.0 + jump)
        fhat, sel, tie = O.reconstruct(order, w, 1e-5)
        assert sel == 0 and fhat == 2.0 and tie == 0
        # jump between j-1 and j: S_j^{j+1} (central, order 2) has IS = 0 and wins over S_j^j
        w = np.where(np.arange(2 * h + 1) <= h - 1, 2.0, 2.0 + jump)
        fhat, sel, tie = O.reconstruct(order, w, 1e-5)
        assert sel == 1 and fhat == 2.0 + jump


@pytest.mark.parametrize("order", [5, 7])
def test_polynomial_window_selects_top(order):
    """A degree-(order-1) polynomial has a vanishing top indicator: the top candidate is
    chosen and reproduces the polynomial's h at x_{j+1/2} exactly."""
    h = H[order]
    rng = np.random.default_rng(order)
    for _ in range(20):
        a = [Fr(int(v)) for v in rng.integers(-3, 4, size=order)]
        # cell averages of the polynomial with coefficients a on unit cells around j
        w = [X.poly_cell_average(a, q - h) for q in range(2 * h + 1)]
        fhat, sel, _ = O.reconstruct(order, np.array([float(v) for v in w]), 1e-5)
        assert sel == O.num_candidates(order) - 1
        assert abs(fhat - float(X.poly_eval(a, Fr(1, 2)))) <= 1e-12 * (1 + abs(fhat))


def test_near_tie_flags():
    """The oracle's tie flag: raised at IS_k = delta, not raised for structural ties or for
    generic data."""
    order, h = 5, 3
    # window whose top indicator is exactly delta: 5th differences equal to delta
    d = 1e-5
    base = np.zeros(2 * h + 1)
    base[0] = -d  # delta_L of S_{j-2}^{j+2} = |-f0| = d ; delta_R = 0 -> IS = 0 actually
    _, sel, tie = O.reconstruct(order, base, d)
    assert sel == 5  # IS_5 = min(d, 0) = 0
    w = np.array([0, 0, 0, 0, 0, 0, 1.0])  # delta_R of S_{j-2}^{j+2} = 1, delta_L = 0
    _, sel, tie = O.reconstruct(order, w, d)
    assert sel == 5 and tie == 0
    # IS_5 exactly delta (both sides equal): flagged
    w = np.array([-d, 0, 0, 0, 0, 0, d])
    _, ind = O.candidates(order, w)
    assert ind[5] == d
    _, sel, tie = O.reconstruct(order, w, d)
    assert sel == 5 and tie == 1
    # generic random data: flags are rare
    rng = np.random.default_rng(7)
    flags = sum(O.reconstruct(order, rng.standard_normal(7), 1e-5)[2] for _ in range(3000))
    assert flags <= 3


def test_structural_tie_not_flagged():
    """S_{j-2}^{j+1} and S_{j-1}^{j+2} share one fourth difference; when both indicators are
    realised by it they tie exactly in every implementation, so no flag is raised."""
    # f1..f5 a perturbed cubic (small shared fourth difference), f0 and f6 far off: the shared
    # difference is the smallest indicator of all, in the fallback branch
    w = np.array([1000.0, 1.0, 8.0, 27.01, 64.0, 125.0, -1000.0])
    _, ind = O.candidates(5, w)
    assert ind[3] == ind[4] and ind[4] == ind.min() and ind.min() > 1e-5
    _, sel, tie = O.reconstruct(5, w, 1e-5)
    assert sel == 4 and tie == 0
    assert sel == _rule(list(ind), 5, 1e-5)
    # perturb f0 so that the other side of S_{j-2}^{j+1} becomes equally small (opposite sign,
    # so the fifth difference stays large): the realisation is no longer robust
    w2 = w.copy()
    w2[0] = w[0] - (w[0] - 4 * w[1] + 6 * w[2] - 4 * w[3] + w[4]) - ind[3]
    _, ind2 = O.candidates(5, w2)
    _, sel2, tie2 = O.reconstruct(5, w2, 1e-5)
    assert tie2 == 1


def test_exact_zero_indicators_not_flagged():
    """With delta = 0 the first principle compares indicators with zero.  An indicator that
    is exactly zero because one of its delta rows reads only equal values is zero in every
    implementation, so no flag is raised.  The oracle evaluates a row as a sum of products,
    so equal values whose multiples round (0.3) can leave a residue where a difference
    table gets zero: that comparison is within rounding and stays flagged, as does a zero
    that comes from cancellation among unequal values (a fifth difference of a quartic)."""
    for order, K in ((5, 6), (7, 9)):
        n = 7 if order == 5 else 9
        for w in (np.full(n, 0.25), np.zeros(n)):
            fhat, sel, tie = O.reconstruct(order, w, 0.0)
            assert sel == K - 1 and tie == 0 and fhat == w[0]
        # equal values on the left row only: still an exact zero for the top candidate
        w = np.full(n, 2.0)
        w[-1] = 7.0
        _, ind = O.candidates(order, w)
        assert ind[K - 1] == 0.0
        _, sel, tie = O.reconstruct(order, w, 0.0)
        assert sel == K - 1 and tie == 0
    w = np.full(7, 0.3)
    _, ind = O.candidates(5, w)
    assert ind[5] != 0.0
    assert O.reconstruct(5, w, 0.0)[2] == 1
    # quartic on small integers: every fifth difference cancels to an exact zero, but from
    # unequal values, so the comparison with delta = 0 is flagged
    x = np.arange(-3.0, 4.0)
    w = x ** 4 - 2 * x ** 3 + x
    _, ind = O.candidates(5, w)
    assert ind[5] == 0.0
    _, sel, tie = O.reconstruct(5, w, 0.0)
    assert sel == 5 and tie == 1
