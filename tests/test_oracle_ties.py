"""Exact-arithmetic pins of complete clipping's choice among maximisers
(Thm 3.1 and the case analysis of its proof; coordinate ascent, eq. 4).

The reference here is written from the definitions alone, in rational
arithmetic (fractions.Fraction): D(beta) is evaluated exactly at beta = 0 and
at every positive breakpoint, and the smallest beta attaining the maximum is
the multiplier (the reading "smallest maximiser").  Coordinate ascent repeats
that for each constraint with the other multipliers fixed, and the bound is
D at the final multipliers, all exact.  Relaxed clipping before it is the
closed form of Thm 3.2 in rationals.

The inputs make the decision a tie in exact arithmetic:
* relaxed clipping by a constraint followed by complete clipping with the
  same constraint, where the dual is flat on the segment in which only the
  clipped coordinate's breakpoint is still ahead;
* duplicated constraints (the second copy's slope at 0+ is exactly zero or
  negative once the first multiplier is optimal);
* exactly tied breakpoints, at and away from the crossing.
Each case comes in two forms: dyadic data, on which every float64 operation
of the oracle is exact (results must be equal), and data whose clip points
and breakpoints are not representable, where the oracle's float64 pipeline
sees rounding residue in place of the exact zeros and must still take the
exact decision (multipliers equal up to float64 rounding, i.e. the same
candidate; bound equal up to rounding).
"""
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import complete, relaxed

INF = float("inf")


# ------------------------------------------------ exact rational reference

def ex_dual(a, c, g, h, lo, hi, beta):
    v = [aj + beta * gj for aj, gj in zip(a, g)]
    return sum(min(vj * l, vj * u) for vj, l, u in zip(v, lo, hi)) + c + beta * h


def ex_single(a, c, g, h, lo, hi):
    """Exact maximum of D over beta >= 0 and its smallest maximiser."""
    m = sum(min(gj * l, gj * u) for gj, l, u in zip(g, lo, hi)) + h
    if m > 0:
        return INF, F(0)
    cands = {F(0)}
    for aj, gj in zip(a, g):
        if gj != 0 and -aj / gj > 0:
            cands.add(-aj / gj)
    cands = sorted(cands)
    vals = [ex_dual(a, c, g, h, lo, hi, b) for b in cands]
    best = max(vals)
    return best, min(b for b, v in zip(cands, vals) if v == best)


def ex_coord_ascent(a, c, G, h, lo, hi, passes=1):
    k, n = len(G), len(a)
    beta = [F(0)] * k
    for _ in range(passes):
        for kk in range(k):
            ak = [a[j] + sum(beta[p] * G[p][j] for p in range(k) if p != kk) for j in range(n)]
            ck = c + sum(beta[p] * h[p] for p in range(k) if p != kk)
            L, b = ex_single(ak, ck, G[kk], h[kk], lo, hi)
            if L == INF:
                return INF, [F(0)] * k
            beta[kk] = b
    v = [a[j] + sum(beta[p] * G[p][j] for p in range(k)) for j in range(n)]
    L = sum(min(vj * l, vj * u) for vj, l, u in zip(v, lo, hi)) + c + sum(b * hh for b, hh in zip(beta, h))
    return L, beta


def ex_relaxed_parallel(G, h, lo, hi):
    """Thm 3.2 for every constraint against the original box, tightest kept."""
    nlo, nhi = list(lo), list(hi)
    for g, hh in zip(G, h):
        m = sum(min(gj * l, gj * u) for gj, l, u in zip(g, lo, hi)) + hh
        if m > 0:
            return None
        for i, gi in enumerate(g):
            if gi > 0:
                nhi[i] = min(nhi[i], lo[i] - m / gi)
            elif gi < 0:
                nlo[i] = max(nlo[i], hi[i] - m / gi)
    if any(l > u for l, u in zip(nlo, nhi)):
        return None
    return nlo, nhi


def fr(x):
    return [F(v) for v in np.ravel(x)]


def right_slope_is_zero(a, c, g, h, lo, hi, beta):
    """Exact right slope of D at beta is zero: beta starts a flat segment."""
    m = sum(min(gj * l, gj * u) for gj, l, u in zip(g, lo, hi)) + h
    ahead = sum(abs(gj) * (u - l) for aj, gj, l, u in zip(a, g, lo, hi)
                if gj != 0 and -aj / gj > beta)
    return m + ahead == 0


def run_both(a, c, G, h, lo, hi, passes=1, clip=True):
    """Exact pipeline (rational) and the oracle's float64 pipeline on the same
    float64 inputs.  Returns ((L, beta, box) exact, (L, beta, inf, box) oracle)."""
    ex_box = (fr(lo), fr(hi))
    o_lo, o_hi = lo[None].astype(np.float64), hi[None].astype(np.float64)
    o_inf = False
    if clip:
        r = ex_relaxed_parallel([fr(g) for g in G], fr(h), *ex_box)
        o_lo, o_hi, oi = relaxed.clip_parallel(G[None], h[None], o_lo, o_hi)
        o_inf = bool(oi[0])
        if r is None:
            return None, (None, None, o_inf, None)
        ex_box = r
    L, beta = ex_coord_ascent(fr(a), F(float(c)), [fr(g) for g in G], fr(h), *ex_box, passes)
    oL, ob, oinf = complete.coord_ascent(a[None], np.array([c]), G[None], h[None], o_lo, o_hi,
                                         passes=passes)
    return (L, beta, ex_box), (oL[0], ob[0], o_inf or bool(oinf[0]), (o_lo[0], o_hi[0]))


def check_same(ex, orc, exact_equal):
    L, beta, box = ex
    oL, ob, oinf, obox = orc
    if L == INF:
        assert oinf and oL == INF
        return
    assert not oinf
    for bx, bo in zip(beta, ob):
        if exact_equal:
            assert F(float(bo)) == bx, (bo, bx)
        else:    # the same candidate: equal up to float64 rounding
            assert abs(float(bx) - bo) <= 1e-12 * max(1.0, abs(float(bx))), (bo, float(bx))
    scale = 1.0 + abs(float(L))
    if exact_equal:
        assert F(float(oL)) == L, (oL, L)
    else:
        assert abs(float(oL) - float(L)) <= 1e-12 * scale, (oL, float(L))


# --------------------------------------------------- hand-built tie cases

def flat_after_clip(g0):
    """Box [-1,1]^4, one constraint g.x + h <= 0 that relaxed clipping
    tightens on coordinate 0 only (g0 = 2: dyadic clip point 1/4; g0 = 7:
    -9/14, not representable, and the float64 slope on the flat segment comes
    out as rounding residue instead of zero).  Objective breakpoints q_1 = 1 (weight 2) and
    q_0 = 3 (weight -m after clipping): the dual rises with slope 2 on
    [0, 1] and is exactly flat on [1, 3], so beta* = 1."""
    g = np.array([g0, 1.0, -1.0, 0.5])
    h = np.array([g0])                    # m = -(g0 + 2.5) + h = -2.5
    lo, hi = -np.ones(4), np.ones(4)
    a = np.array([-3.0 * g0, -1.0, -1.0, 0.25])
    return a, 0.5, g[None], h, lo, hi


@pytest.mark.parametrize("g0", [2.0, 7.0], ids=["dyadic", "rounded"])
def test_flat_dual_after_relaxed_clipping_by_the_same_constraint(g0):
    a, c, G, h, lo, hi = flat_after_clip(g0)
    ex, orc = run_both(a, c, G, h, lo, hi)
    L, beta, box = ex
    assert beta == [F(1)]                                      # smallest maximiser
    assert right_slope_is_zero(fr(a), F(c), fr(G[0]), F(h[0]), box[0], box[1], beta[0])
    assert box[1][0] == F(-1) + F(5, 2) / F(g0)                # the clip of Thm 3.2
    check_same(ex, orc, exact_equal=(g0 == 2.0))
    # the same problem with the only remaining breakpoint being the clipped
    # coordinate's: flat from 0, beta* = 0 (the constraint adds nothing)
    a2 = a.copy()
    a2[1] = 1.0
    ex, orc = run_both(a2, c, G, h, lo, hi)
    assert ex[1] == [F(0)]
    check_same(ex, orc, exact_equal=(g0 == 2.0))


@pytest.mark.parametrize("den", [1.0, 3.0], ids=["dyadic", "rounded"])
def test_duplicated_constraints(den):
    # the second copy of a constraint: after the first multiplier is optimal
    # the slope at 0+ of the copy is the first's right slope there (<= 0), so
    # its multiplier is 0; a third constraint between the copies changes that
    lo, hi = -np.ones(5), np.ones(5)
    g = np.array([1.0, -2.0, 0.5, 1.0, 0.0]) * np.array([den, 1.0, 1.0, 1.0, 1.0])
    g2 = np.array([0.0, 1.0, 1.0, -1.0, 2.0])
    a = np.array([-2.0, 1.5, -0.75, -1.0, 1.0])
    for G, hh in ((np.stack([g, g]), np.array([0.25, 0.25])),
                  (np.stack([g, g2, g]), np.array([0.25, -0.5, 0.25]))):
        for passes in (1, 2):
            ex, orc = run_both(a, 0.0, G, hh, lo, hi, passes=passes, clip=False)
            if G.shape[0] == 2:
                assert ex[1][1] == 0 and ex[1][0] > 0
            check_same(ex, orc, exact_equal=(den == 1.0))
            ex, orc = run_both(a, 0.0, G, hh, lo, hi, passes=passes, clip=True)
            check_same(ex, orc, exact_equal=(den == 1.0))


@pytest.mark.parametrize("den", [1.0, 3.0], ids=["dyadic", "rounded"])
def test_tied_breakpoints(den):
    lo, hi = -np.ones(6), np.ones(6)
    # three coordinates share q = 2/den (weights 2 den, 4 den, den; den = 3
    # makes it 2/3, rounded alike for all three), one more has q = 1/4
    # (weight 2), the rest none
    g = np.array([den, 2.0 * den, 0.5 * den, -1.0, 0.5, 0.0])
    a = np.array([-2.0, -4.0, -1.0, 0.25, 0.25, 3.0])
    # the right slope is m past the tie and m + 7 den between 1/4 and the
    # tie: the crossing inside the tie (m = -1), or a flat segment from 1/4
    # up to the tie (m = -7 den)
    for m_target in (-1.0, -7.0 * den):
        h = m_target + (3.5 * den + 1.5)      # m = -(sum |g|) + h on [-1,1]^6
        ex, orc = run_both(a, 0.0, g[None], np.array([h]), lo, hi, clip=False)
        assert ex[1][0] == (F(2) / F(den) if m_target == -1.0 else F(1, 4))
        check_same(ex, orc, exact_equal=(den == 1.0))


# ----------------------------------------------- structured random cases

def structured_problem(rng, dyadic):
    n = int(rng.integers(2, 7))
    k = int(rng.integers(1, 4))
    lo = rng.integers(-8, 1, n) / 8.0
    hi = lo + rng.integers(1, 17, n) / 8.0
    coef = [0.5, 1.0, 2.0, 4.0] if dyadic else [1.0, 3.0, 5.0, 7.0]
    G = rng.choice(coef, (k, n)) * rng.choice([-1.0, 1.0], (k, n))
    G[rng.random((k, n)) < 0.15] = 0.0
    for p in range(1, k):
        if rng.random() < 0.3:
            G[p] = G[rng.integers(p)]                  # duplicated constraint
    xs = lo + rng.integers(0, 9, n) / 8.0 * (hi - lo)
    xs = np.round(xs * 8.0) / 8.0
    h = -(G @ xs) - rng.choice([0.0, 0.125, 0.25], k)
    a = rng.integers(-16, 17, n) / 8.0
    if rng.random() < 0.5:                              # tied breakpoints
        q = rng.integers(1, 9) / 4.0
        sel = rng.random(n) < 0.5
        gj = np.where(G[0] != 0.0, G[0], 1.0)
        a = np.where(sel & (G[0] != 0.0), -q * gj, a)
    return a, 0.25, G, h, lo, hi


@pytest.mark.parametrize("dyadic", [True, False], ids=["dyadic", "rounded"])
def test_structured_ties_take_the_exact_decision(dyadic):
    rng = np.random.default_rng(2024 if dyadic else 2025)
    flat = ties = checked = 0
    for _ in range(150):
        a, c, G, h, lo, hi = structured_problem(rng, dyadic)
        for passes in (1, 2):
            ex, orc = run_both(a, c, G, h, lo, hi, passes=passes)
            if ex is None:
                assert orc[2], "exact relaxed clipping empties the box, the oracle did not"
                continue
            check_same(ex, orc, exact_equal=dyadic)
            checked += 1
            L, beta, box = ex
            if L == INF or passes > 1:
                continue
            # count the decisions that were exact ties (one pass: constraint
            # kk is maximised with the earlier multipliers in place)
            for kk in range(G.shape[0]):
                ak = [F(float(a[j])) + sum(beta[p] * F(float(G[p][j])) for p in range(kk))
                      for j in range(len(a))]
                ck = F(c) + sum(beta[p] * F(float(h[p])) for p in range(kk))
                if right_slope_is_zero(ak, ck, fr(G[kk]), F(float(h[kk])), box[0], box[1], beta[kk]):
                    flat += 1
                qs = [-aj / F(float(gj)) for aj, gj in zip(ak, G[kk]) if gj != 0]
                if beta[kk] > 0 and qs.count(beta[kk]) > 1:
                    ties += 1
    assert checked > 200
    assert flat > 20 and ties > 5, (flat, ties)


def test_rounding_residue_is_what_the_tolerance_absorbs():
    # on the rounded flat case the float64 right slope at beta* is rounding
    # residue, not zero, and lies inside the oracle's own bound
    a, c, G, h, lo, hi = flat_after_clip(7.0)
    nlo, nhi, _ = relaxed.clip_parallel(G[None], h[None], lo[None], hi[None])
    left, right = complete.dual_slopes(a, G[0], h[0], nlo[0], nhi[0], np.float64(1.0))
    tol = complete.slope_tol(G[0], h[0], nlo[0], nhi[0])
    assert right != 0.0 and abs(right) <= tol
    assert tol < 1e-12 and left == pytest.approx(2.0)


@pytest.mark.parametrize("sign", [1, -1])
def test_a_near_tie_that_is_not_a_tie(sign):
    # the flat case of flat_after_clip(2) with the clipped coordinate's end
    # moved by 2^-31 (no relaxed clipping): the slope on [1, 3] is +-2^-30,
    # far above float64 rounding, so the exact decision is to go on to 3
    # (slope > 0) or to stop at 1 (slope < 0); a tolerance sized to float32
    # weights (2^-18 of the scale) would stop at 1 in both cases
    a, c, G, h, lo, hi = flat_after_clip(2.0)
    hi = hi.copy()
    hi[0] = 0.25 + sign * 2.0 ** -31
    ex, orc = run_both(a, c, G, h, lo, hi, clip=False)
    assert ex[1] == [F(3) if sign > 0 else F(1)]
    check_same(ex, orc, exact_equal=True)
