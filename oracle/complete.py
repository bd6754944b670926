"""Complete clipping: min of a.x + c over box ∩ {G x + h <= 0}.

Single constraint (Thm 3.1, proof in the appendix): the optimum equals
max over beta >= 0 of the dual D(beta) = min_box (a + beta g).x + c + beta h,
a concave piecewise-linear function whose breakpoints are q_j = -a_j / g_j.
If min_box(g.x + h) > 0 the feasible set is empty and the optimum is +inf
(case 1 of the proof).

Three independent single-constraint solvers are kept so that each pins the
others: ``single_enum`` (evaluate D at 0 and at every positive breakpoint,
O(n^2)), ``single_sort`` (sort breakpoints, accumulate the supergradient,
take the first sign change -- the procedure of Alg. 1 for one constraint)
and ``knapsack_greedy`` (the primal fractional-knapsack greedy of the
knapsack-equivalence appendix).

Several constraints: ``coord_ascent`` runs passes of exact 1-D maximisations
over the multipliers, one constraint at a time in the given order (eq. 4 and
Alg. 1), and returns D(beta), which is a valid lower bound for any beta >= 0.

Readings taken:
* The candidates for beta* are {0} together with the positive breakpoints:
  if the supergradient is already <= 0 before the first breakpoint (the
  constraint is redundant over the box) beta* = 0.  A literal reading of
  Alg. 1 would pick the first breakpoint instead.
* Alg. 1's comments call the supergradient "nondecreasing" and the cumulative
  sum one "of sorted breakpoints": the supergradient is non-increasing in the
  sorted index (D is concave) and the sum runs over the sorted weights
  |g_j| eps_j.
* Alg. 1 builds the breakpoints of constraint k from a + beta^T G including
  beta_k; the multiplier being optimised is excluded (identical in a single
  pass from beta = 0, needed for more than one pass).
* Coefficients g_j = 0 give no breakpoint (key +inf, weight 0).
* Among equal maximisers the smallest beta is reported; the optimum value is
  unique and is what callers compare.
* Near-ties: a supergradient within TIE_REL * sum_j |g_j| max(|lo_j|, |hi_j|)
  of zero counts as zero, so the smallest near-maximiser is taken.  Relaxed
  clipping followed by complete clipping with the same constraint makes the
  dual exactly flat on [0, q] (the clipped coordinate's weight equals -m);
  without a tolerance the choice inside that flat segment, and with it every
  later coordinate-ascent step, would be decided by rounding.  Any beta >= 0
  stays a valid bound; for one constraint the loss is at most the tolerance
  times the step in beta.
"""
import numpy as np

from .box import f64, concretize_min

TIE_REL = 2.0 ** -18


def dual_value(a, c, g, h, lo, hi, beta):
    """D(beta) = min over the box of (a + beta g).x + c + beta h.
    a, g, lo, hi: [..., n]; c, h, beta: [...]."""
    a, g = f64(a), f64(g)
    beta = f64(beta)
    v = a + beta[..., None] * g
    return concretize_min(v[..., None, :], (f64(c) + beta * f64(h))[..., None],
                          f64(lo), f64(hi))[..., 0]


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


def single_sort(a, c, g, h, lo, hi):
    """Thm 3.1 by sorting breakpoints (the one-constraint case of Alg. 1),
    batched over leading dims.  a, g, lo, hi: [R, n]; c, h: [R].

    In centre/radius terms the supergradient just right of the i-th sorted
    breakpoint is  g.xh + h + sum_{j>i} |g_j| eps_j - sum_{j<=i} |g_j| eps_j;
    before the first breakpoint it is g.xh + h + sum_j |g_j| eps_j (= the max
    of the constraint over the box).  beta* is 0 if that is <= 0, else the
    first breakpoint whose right supergradient is <= 0.
    Returns (L [R], beta [R], infeasible [R])."""
    a, g, lo, hi = f64(a), f64(g), f64(lo), f64(hi)
    c, h = f64(c), f64(h)
    xh = (lo + hi) / 2.0
    eps = (hi - lo) / 2.0
    e = np.abs(g) * eps
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(g != 0.0, -a / np.where(g != 0.0, g, 1.0), np.inf)
    order = np.argsort(q, axis=-1, kind="stable")
    qs = np.take_along_axis(q, order, -1)
    es = np.take_along_axis(e, order, -1)
    base = (g * xh).sum(-1) + h
    tol = TIE_REL * (np.abs(g) * np.maximum(np.abs(lo), np.abs(hi))).sum(-1)
    cum = np.cumsum(es, axis=-1)                   # sum_{j<=i}
    total = cum[..., -1:] if es.shape[-1] else np.zeros(base.shape + (1,))
    sg = base[..., None] + (total - cum) - cum      # right supergradient
    before_first = base + total[..., 0]
    m = base - total[..., 0]
    infeas = m > 0.0
    nonpos = sg <= tol[..., None]
    has = nonpos.any(-1)
    istar = np.argmax(nonpos, axis=-1)
    q_star = np.take_along_axis(qs, istar[..., None], -1)[..., 0] if qs.shape[-1] else np.zeros(base.shape)
    beta = np.where(before_first <= tol, 0.0, np.where(has, np.maximum(q_star, 0.0), 0.0))
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
    """Coordinate ascent over the multipliers of several constraints (eq. 4,
    Alg. 1), batched: a: [R, n], c: [R], G: [R, k, n], h: [R, k],
    lo/hi: [R, n], active: [R, k] bool.  Each step maximises D exactly in
    beta_k with the other multipliers fixed, using ``single_sort``.
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
            _, b_k, inf_k = single_sort(a_k, c_k, g_k, h_k, lo, hi)
            beta[:, kk] = np.where(active[:, kk], b_k, 0.0)
            infeas |= active[:, kk] & inf_k
    beta = np.where(infeas[:, None], 0.0, beta)
    v = a + np.einsum("rk,rkn->rn", beta, G)
    L = concretize_min(v[:, None, :], (c + (beta * h).sum(-1))[:, None], lo, hi)[:, 0]
    L = np.where(infeas, np.inf, L)
    return L, beta, infeas
