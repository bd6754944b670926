"""Complete clipping: min of a.x + c over box ∩ {G x + h <= 0} (test
infrastructure: part of the FP64 oracle).

Single constraint (Thm 3.1, proof in the appendix): the optimum equals the
maximum over beta >= 0 of the dual
    D(beta) = min over the box of (a + beta g).x + c + beta h,
a concave piecewise-linear function of beta.  Coordinate j changes the side
of the box it minimises on at its breakpoint q_j = -a_j / g_j.  For beta
right of a point, coordinate j sits at the end that maximises g_j x_j while
q_j is still ahead (a_j + beta g_j has the sign of a_j, opposite to g_j) and
at the end that minimises it once q_j has been passed; so the right slope of
D is
    D'(beta+) = m + sum over {j : q_j > beta} of w_j,
    m = min over the box of g.x + h,   w_j = |g_j| (hi_j - lo_j).
D rises while that slope is positive, so beta* = 0 when D'(0+) <= 0 (the
constraint is redundant over the box), else the smallest positive
breakpoint whose right slope is <= 0.  The slope tends to m; m > 0 means the
feasible set is empty and the optimum is +inf (case 1 of the proof).

Three independent single-constraint solvers pin each other:
``single_enum`` (evaluate D at 0 and at every positive breakpoint, O(n^2)),
``single_max`` (the right slope above at every candidate, batched) and
``knapsack_greedy`` (the primal fractional-knapsack greedy of the
knapsack-equivalence appendix).

Several constraints: ``coord_ascent`` runs passes of exact 1-D maximisations
over the multipliers, one constraint at a time in the given order (eq. 4),
and returns D(beta), a valid lower bound for any beta >= 0 (weak duality).

Readings taken:
* The candidates for beta* are {0} together with the positive breakpoints;
  a redundant constraint gets beta* = 0.
* The multiplier being optimised is left out of the objective it is
  optimised against (the others keep their current values): identical in a
  single pass from beta = 0, needed for more than one pass.
* Coefficients g_j = 0 give no breakpoint.
* Among maximisers the smallest beta is reported; breakpoints that are equal
  are passed together.
* Near-ties (the oracle's own rounding): a right slope within ``slope_tol``
  of zero counts as zero.  Relaxed clipping followed by complete clipping
  with the same constraint leaves the dual exactly flat on the segment where
  only the clipped coordinate's breakpoint is still ahead (that weight
  equals -m), and duplicated constraints leave the second one's slope at 0+
  exactly zero; in float64 those exact zeros come out as rounding residue of
  either sign.  The tolerance is a bound on that residue, so the oracle
  takes the decision exact arithmetic takes (the smallest maximiser); it is
  derived from float64 rounding below and shares nothing with any other
  implementation.
"""
import numpy as np

from .box import f64, concretize_min

U64 = 2.0 ** -53   # unit roundoff of float64


def slope_tol(g, h, lo, hi):
    """Bound on the float64 rounding residue of a computed right slope.

    E = sum_j |g_j| max(|lo_j|, |hi_j|) + |h| bounds every term of m and
    sum_j w_j <= 2E.  Forming m (n products and n + 1 additions) is off by at
    most gamma_{n+1} E, the weights (a difference and a product each) by
    gamma_2 w_j, their partial sum by gamma_n sum_j w_j, and the final
    addition by one more unit: together at most 3 gamma_{n+2} E.  A box
    produced by float64 relaxed clipping moves a clipped coordinate's end by
    the rounding of lo_i - m_k/g_i, i.e. the slope by at most
    (gamma_{n+1} + 2u) E over the clipped coordinates, which is why an
    exactly flat segment is recognised.  gamma_k = k u / (1 - k u) <= 1.01 k u
    for these n, so (4n + 16) u E covers the sum.  g, lo, hi: [..., n];
    h: [...]."""
    n = np.shape(g)[-1]
    E = (np.abs(g) * np.maximum(np.abs(lo), np.abs(hi))).sum(-1) + np.abs(h)
    return (4 * n + 16) * U64 * E


def dual_value(a, c, g, h, lo, hi, beta):
    """D(beta) = min over the box of (a + beta g).x + c + beta h.
    a, g, lo, hi: [..., n]; c, h, beta: [...]."""
    a, g = f64(a), f64(g)
    beta = f64(beta)
    v = a + beta[..., None] * g
    return concretize_min(v[..., None, :], (f64(c) + beta * f64(h))[..., None],
                          f64(lo), f64(hi))[..., 0]


def dual_slopes(a, g, h, lo, hi, beta):
    """Left and right slopes of D at beta (Thm 3.1): the right slope is
    m + sum_{q_j > beta} w_j, the left one m + sum_{q_j >= beta} w_j (only
    coordinates with a positive breakpoint count; at beta = 0 the left slope
    is returned as +inf, since beta cannot decrease there).  Batched:
    a, g, lo, hi: [..., n]; h, beta: [...].  Returns (left, right)."""
    a, g, lo, hi = f64(a), f64(g), f64(lo), f64(hi)
    h, beta = f64(h), f64(beta)
    m = np.minimum(g * lo, g * hi).sum(-1) + h
    w = np.abs(g) * (hi - lo)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(g != 0.0, -a / np.where(g != 0.0, g, 1.0), -np.inf)
    b = beta[..., None]
    right = m + np.where(q > b, w, 0.0).sum(-1)
    left = m + np.where((q >= b) & (q > 0.0), w, 0.0).sum(-1)
    left = np.where(beta > 0.0, left, np.inf)
    return left, right


def single_enum(a, c, g, h, lo, hi):
    """Thm 3.1 by enumeration: D at beta = 0 and at every positive
    breakpoint; one problem (vectors of length n).  Returns (L, beta)."""
    a, g, lo, hi = f64(a), f64(g), f64(lo), f64(hi)
    c, h = float(c), float(h)
    m = float(np.minimum(g * lo, g * hi).sum() + h)
    if m > 0.0:
        return np.inf, 0.0
    cands = [0.0]
    for j in range(a.size):
        if g[j] != 0.0:
            q = -a[j] / g[j]
            if q > 0.0:
                cands.append(q)
    cands = sorted(set(cands))
    best, best_beta = -np.inf, 0.0
    for beta in cands:
        d = float(dual_value(a, c, g, h, lo, hi, np.float64(beta)))
        if d > best:
            best, best_beta = d, beta
    return best, best_beta


def single_max(a, c, g, h, lo, hi):
    """Thm 3.1 through the right slope of D at every candidate, batched over
    rows: a, g, lo, hi: [R, n]; c, h: [R].

    The positive breakpoints are put in increasing order (a library sort);
    the weight still ahead of candidate i is the sum of the weights of the
    breakpoints strictly greater than it (equal breakpoints form one group
    and are passed together), so the right slope at i is m plus that sum.
    beta* is 0 when the slope at 0+ (m plus every candidate's weight) is
    within the rounding tolerance of zero or below, else the first candidate
    whose right slope is.  Returns (L [R], beta [R], infeasible [R])."""
    a, g, lo, hi = f64(a), f64(g), f64(lo), f64(hi)
    c, h = f64(c), f64(h)
    n = a.shape[-1]
    m = np.minimum(g * lo, g * hi).sum(-1) + h
    w = np.abs(g) * (hi - lo)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(g != 0.0, -a / np.where(g != 0.0, g, 1.0), 0.0)
    cand = (g != 0.0) & (q > 0.0)
    key = np.where(cand, q, np.inf)
    order = np.argsort(key, axis=-1, kind="stable")
    ks = np.take_along_axis(key, order, -1)
    ws = np.take_along_axis(np.where(cand, w, 0.0), order, -1)
    tol = slope_tol(g, h, lo, hi)
    infeas = m > 0.0
    if n == 0:
        beta = np.zeros(m.shape)
    else:
        ahead_incl = np.cumsum(ws[..., ::-1], axis=-1)[..., ::-1]          # sum_{p >= i}
        ahead_excl = np.concatenate([ahead_incl[..., 1:], np.zeros(m.shape + (1,))], -1)
        # last position of the group of equal breakpoints that i belongs to
        pos = np.broadcast_to(np.arange(n), ks.shape)
        last = np.concatenate([ks[..., :-1] != ks[..., 1:], np.ones(m.shape + (1,), bool)], -1)
        end = np.minimum.accumulate(np.where(last, pos, n)[..., ::-1], axis=-1)[..., ::-1]
        right = m[..., None] + np.take_along_axis(ahead_excl, end, -1)
        ok = (right <= tol[..., None]) & np.isfinite(ks)
        first = np.argmax(ok, axis=-1)
        q_star = np.take_along_axis(ks, first[..., None], -1)[..., 0]
        at_zero = m + ahead_incl[..., 0] <= tol
        beta = np.where(at_zero | ~ok.any(-1), 0.0, q_star)
    beta = np.where(infeas, 0.0, beta)
    L = dual_value(a, c, g, h, lo, hi, beta)
    L = np.where(infeas, np.inf, L)
    return L, beta, infeas


def knapsack_greedy(a, c, g, h, lo, hi):
    """Primal fractional-knapsack greedy for one problem (knapsack-equivalence
    appendix).  Start from the box minimiser of a.x (ties broken toward the
    smaller constraint value); if it violates g.x + h <= 0, move coordinates
    toward their other end in increasing order of cost per unit of constraint
    decrease, which is the ratio -a_j/g_j, the last one fractionally.
    Returns (L, infeasible)."""
    a, g, lo, hi = f64(a), f64(g), f64(lo), f64(hi)
    c, h = float(c), float(h)
    x0 = np.where(a > 0.0, lo, np.where(a < 0.0, hi, np.where(g > 0.0, lo, hi)))
    x1 = np.where(x0 == lo, hi, lo)
    viol = float(g @ x0 + h)
    obj = float(a @ x0 + c)
    if viol <= 0.0:
        return obj, False
    dg = g * (x1 - x0)               # change of the constraint if j moves fully
    da = a * (x1 - x0)               # change of the objective (>= 0)
    helpful = dg < 0.0
    idx = np.nonzero(helpful)[0]
    ratio = da[idx] / (-dg[idx])
    idx = idx[np.argsort(ratio, kind="stable")]
    for j in idx:
        if -dg[j] >= viol:
            obj += da[j] * (viol / -dg[j])
            return obj, False
        viol += dg[j]
        obj += da[j]
    return np.inf, True


def coord_ascent(a, c, G, h, lo, hi, active=None, passes=1):
    """Coordinate ascent over the multipliers of several constraints (eq. 4),
    batched: a: [R, n], c: [R], G: [R, k, n], h: [R, k],
    lo/hi: [R, n], active: [R, k] bool.  Each step maximises D exactly in
    beta_k with the other multipliers fixed, using ``single_max``.
    Returns (L [R], beta [R, k], infeasible [R]); infeasible rows have
    L = +inf (some single constraint is empty over the box)."""
    a, c, G, h, lo, hi = f64(a), f64(c), f64(G), f64(h), f64(lo), f64(hi)
    R, k, n = G.shape
    if active is None:
        active = np.ones((R, k), bool)
    beta = np.zeros((R, k))
    infeas = np.zeros(R, bool)
    for _ in range(passes):
        for kk in range(k):
            others = beta.copy()
            others[:, kk] = 0.0
            a_k = a + np.einsum("rk,rkn->rn", others, G)
            c_k = c + (others * h).sum(-1)
            g_k = np.where(active[:, kk:kk + 1], G[:, kk], 0.0)
            h_k = np.where(active[:, kk], h[:, kk], -1.0)
            _, b_k, inf_k = single_max(a_k, c_k, g_k, h_k, lo, hi)
            beta[:, kk] = np.where(active[:, kk], b_k, 0.0)
            infeas |= active[:, kk] & inf_k
    beta = np.where(infeas[:, None], 0.0, beta)
    v = a + np.einsum("rk,rkn->rn", beta, G)
    L = concretize_min(v[:, None, :], (c + (beta * h).sum(-1))[:, None], lo, hi)[:, 0]
    L = np.where(infeas, np.inf, L)
    return L, beta, infeas
