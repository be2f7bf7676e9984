"""Pins of the oracle's tie sets and of the replay of another evaluation's selections.

The parity tests compare the HIP path with the oracle at every cell, with no cell left
out: where the GPU picks another candidate than the oracle at a near tie, the oracle
replays the GPU's pick, provided the pick lies in the oracle's tie set (the candidates
that an evaluation of the same indicators with rounding errors below the near-tie
margin could select under the two principles of Section 3.2).  These tests fix that set
by brute force over perturbed indicators, with the principle restated from the text,
and fix the replay by exact identities: replaying the oracle's own record changes
nothing, a pick outside the set is refused and counted, and an allowed pick takes that
candidate's row of the flux table.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12742_amd import workloads as W

H = {5: 3, 7: 4}
TIE_EPS = 1e-14
# candidate stencils S_{j-m}^{j+n} in the oracle's order (increasing priority)
CANDS = {5: [(0, 0), (0, 1), (1, 1), (2, 1), (1, 2), (2, 2)],
         7: [(0, 0), (0, 1), (1, 1), (2, 1), (1, 2), (2, 2), (3, 2), (2, 3), (3, 3)]}


def _priority(m, n):
    """Section 3.2: higher order first, central before upwind-biased at equal order."""
    return (m + n + 1, 1 if m == n - 1 else 0)


def _rule(IS, order, delta):
    """The two principles of Section 3.2 restated: the highest-priority candidate whose
    indicator does not exceed delta, else the smallest indicator (higher priority on ties)."""
    cands = CANDS[order]
    ok = [k for k in range(len(IS)) if IS[k] <= delta]
    if ok:
        return max(ok, key=lambda k: _priority(*cands[k]))
    lo = min(IS)
    return max((k for k in range(len(IS)) if IS[k] == lo), key=lambda k: _priority(*cands[k]))


def _perturbed_outcomes(order, w, delta):
    """Every choice of the restated rule over indicators moved by -0.9, 0 or +0.9 times the
    near-tie margin.  Exact zeros stay (a zero of equal values is exact everywhere) and
    bitwise-equal indicators move together (one shared difference row)."""
    _, IS = O.candidates(order, w)
    sc = O.indicator_scales(order, w)
    groups = {}
    for k, v in enumerate(IS):
        groups.setdefault(v, []).append(k)
    keys = [g for g in groups.values() if IS[g[0]] != 0.0]
    outs = set()
    for signs in itertools.product((-1, 0, 1), repeat=len(keys)):
        P = IS.copy()
        for sgn, g in zip(signs, keys):
            e = 0.9 * TIE_EPS * min(sc[k] for k in g)
            for k in g:
                P[k] = max(IS[k] + sgn * e, 0.0)
        outs.add(_rule(list(P), order, delta))
    return outs


def _near_delta_windows(order, rng, n):
    """windows with delta within a few units in the last place of one indicator"""
    h = H[order]
    for _ in range(n):
        w = rng.standard_normal(2 * h + 1) * 10.0 ** rng.uniform(-6, 0)
        _, IS = O.candidates(order, w)
        k = rng.integers(len(IS))
        yield w, IS[k] * (1.0 + rng.uniform(-3e-16, 3e-16))


def _near_fallback_windows(order, rng, n):
    """small integers plus noise far below the margin: near ties between different rows,
    decided by the second principle (delta = 0)"""
    h = H[order]
    for _ in range(n):
        yield rng.integers(0, 4, size=2 * h + 1) + 1e-17 * rng.standard_normal(2 * h + 1), 0.0


@pytest.mark.parametrize("order", [5, 7])
def test_tie_set_covers_every_perturbed_choice(order):
    """Brute force: every choice the restated rule makes on indicators perturbed within
    the margin lies in the oracle's tie set, and the set holds the oracle's own choice."""
    rng = np.random.default_rng(31 + order)
    wide = 0
    n_near = 120 if order == 5 else 40
    for w, delta in itertools.chain(_near_delta_windows(order, rng, n_near),
                                    _near_fallback_windows(order, rng, n_near)):
        _, sel, tie, tset, _ = O.reconstruct_replay(order, w, -1, delta)
        assert sel in tset
        outs = _perturbed_outcomes(order, w, delta)
        assert outs <= set(tset), (w.tolist(), delta, outs, tset)
        if len(outs) > 1:
            assert tie == 1
            wide += 1
    assert wide >= 20  # the windows really exercise near ties


@pytest.mark.parametrize("order", [5, 7])
def test_tie_set_is_the_choice_without_near_tie(order):
    """Generic data: no flag, and the tie set is the choice alone, so a replay can change
    nothing there."""
    rng = np.random.default_rng(300 + order)
    h = H[order]
    for _ in range(1500):
        w = rng.standard_normal(2 * h + 1) * 10.0 ** rng.uniform(-7, 1)
        _, sel, tie, tset, _ = O.reconstruct_replay(order, w, -1, 1e-5)
        if tie == 0:
            assert tset == [sel]


@pytest.mark.parametrize("order", [5, 7])
def test_replay_takes_allowed_pick_and_refuses_others(order):
    """At a near tie an allowed pick returns that candidate's row of the flux table; a pick
    outside the set keeps the oracle's choice and reports the mismatch."""
    rng = np.random.default_rng(900 + order)
    K = O.num_candidates(order)
    seen_alt = seen_bad = 0
    for w, delta in _near_delta_windows(order, rng, 200):
        flux, _ = O.candidates(order, w)
        fh0, sel, _, tset, _ = O.reconstruct_replay(order, w, -1, delta)
        for k in range(K):
            fh, s, _, _, ok = O.reconstruct_replay(order, w, k, delta)
            if k in tset:
                assert ok and s == k and fh == flux[k]
                seen_alt += k != sel
            else:
                assert not ok and s == sel and fh == fh0
                seen_bad += 1
    assert seen_alt > 0 and seen_bad > 0


def _problems():
    adv = W.advection(3, 131)
    u = adv.u0.copy()
    x = W.nodes(-1.0, 1.0, 131)
    u[0, 0] += np.where((x > -0.45) & (x < 0.1), 0.8, 0.0)
    yield O.Problem(O.ADVECTION, nx=131, delta=0.0), u
    e1 = W.riemann_1d(4, 150)
    yield O.Problem(O.EULER1D, nx=150, x_lo=0.0, x_hi=1.0, bc_x=O.TRANSMISSIVE), e1.u0
    yield O.Problem(O.EULER1D, nx=150, x_lo=0.0, x_hi=1.0, bc_x=O.TRANSMISSIVE, order=7, delta=0.0), e1.u0
    e2 = W.quadrants(5, 30, 22)
    yield O.Problem(O.EULER2D, nx=30, ny=22), e2.u0
    yield O.Problem(O.EULER2D, nx=30, ny=22, delta=0.0), e2.u0


@pytest.mark.parametrize("case", range(5))
def test_replay_of_own_record_is_identical(case):
    """Replaying the oracle's own selection record reproduces L and a step bitwise."""
    p, u = list(_problems())[case]
    L, sel, tie = O.rhs(p, u, with_selection=True)
    L2, sel2, tie2, nbad = O.rhs_replay(p, u, sel)
    assert nbad == 0 and np.array_equal(L, L2) and np.array_equal(sel, sel2) and np.array_equal(tie, tie2)
    dt = 0.5 * O.cfl_dt(p, u, 0.3)
    recs = []
    v = u.copy()
    Lv, s1, _ = O.rhs(p, v, with_selection=True)
    w1 = v + dt * Lv
    Lv, s2, _ = O.rhs(p, w1, with_selection=True)
    w2 = 0.75 * v + 0.25 * (w1 + dt * Lv)
    _, s3, _ = O.rhs(p, w2, with_selection=True)
    recs = np.concatenate([s1, s2, s3])
    u_ref = O.step(p, u, dt)
    u_rep, nbad = O.step_replay(p, u, dt, recs)
    assert nbad == 0 and np.array_equal(u_ref, u_rep)


def test_replay_counts_picks_outside_the_tie_set():
    """A record with a wrong pick at faces without a near tie is refused there: every such
    face side is counted and L keeps the oracle's value."""
    p, u = list(_problems())[3]
    L, sel, tie = O.rhs(p, u, with_selection=True)
    bad = sel.copy()
    idx = np.flatnonzero(tie == 0)[::97]
    bad[idx] = (bad[idx] + 1) % 6
    L2, _, _, nbad = O.rhs_replay(p, u, bad)
    assert nbad == idx.size and np.array_equal(L, L2)
    # an out-of-range index is refused too
    bad = sel.copy()
    bad[idx[:3]] = 200
    assert O.rhs_replay(p, u, bad)[3] == 3


def test_replayed_alternative_moves_only_its_two_cells():
    """Forcing an allowed alternative at one flagged face side changes L only at the two
    cells next to that face.  The threshold is set to one indicator of the face's
    plus-side window, which makes that comparison an exact tie."""
    p0, u = list(_problems())[0]
    a = p0.adv_speed
    h = H[5]
    changed = 0
    for f in range(1, p0.nx):
        win = np.array([u[0, 0, (f - 1 - h + q) % p0.nx] for q in range(2 * h + 1)])
        fp = 0.5 * (a * win + abs(a) * win)
        mp = 0.5 * (np.abs(a * win) + abs(a) * np.abs(win))
        _, IS = O.candidates(5, fp)
        for k in range(5, -1, -1):
            if IS[k] == 0.0:
                continue
            _, s0, _, tset, _ = O.reconstruct_replay(5, fp, -1, float(IS[k]), mag=mp)
            if len(tset) > 1:
                break
        else:
            continue
        p = O.Problem(O.ADVECTION, nx=p0.nx, delta=float(IS[k]))
        L, sel, tie = O.rhs(p, u, with_selection=True)
        i = f  # plus side of face f (between nodes f-1 and f), field 0
        assert tie[i] == 1 and s0 == sel[i]
        force = sel.copy()
        force[i] = [c for c in tset if c != s0][0]
        L2, sel2, _, nbad = O.rhs_replay(p, u, force)
        assert nbad == 0 and sel2[i] == force[i]
        moved = np.flatnonzero(L2[0, 0] != L[0, 0])
        assert set(moved.tolist()) <= {(f - 1) % p.nx, f % p.nx}
        changed += moved.size > 0
    assert changed > 5
