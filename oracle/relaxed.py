"""Relaxed clipping of a box by linear constraints G x + h <= 0.

* Single constraint (Thm 3.2): with m = min over the box of g.x + h, the box
  is empty iff m > 0 (proof of Thm 3.2; the a-priori infeasibility test of
  the complete-clipping section).  Otherwise coordinate i is tightened to
  x_i^clip = (-sum_{j != i}(g_j xh_j - |g_j| eps_j) - h) / g_i: an upper bound
  when g_i > 0, a lower bound when g_i < 0, nothing when g_i = 0.
* Parallel (Alg. 2): every constraint is applied to the ORIGINAL box and the
  tightest result per coordinate is kept.
* Sequential (Alg. 3): constraints are applied one after another, each to
  the box left by the previous one.

Readings taken (the paper is inconsistent here):
* sign convention: constraints are G x + h <= 0 throughout (Thm 3.2 and
  Alg. 1); Alg. 2's header writes A x <= c.
* Alg. 2 tests ``A_ki >= 0`` and would divide by zero for A_ki = 0; Thm 3.2
  says a zero coefficient changes nothing, which is what is done.
* Alg. 3 prints the update of x^(new) outside the coordinate loop; the text
  of the sequential-clipping appendix (compute from the current box, update
  all coordinates, then go to the next constraint) is followed.
* A box is reported infeasible when some constraint has m > 0 or when some
  coordinate ends with lo > hi (the appendix notes the latter signals an
  empty region; it prints "smaller" where "larger" is meant).
"""
import numpy as np

from .box import f64


def constraint_min(g, h, lo, hi):
    """m = min over the box of g.x + h.  g: [..., k, n], h: [..., k],
    lo/hi: [..., n] -> [..., k]."""
    g, h, lo, hi = f64(g), f64(h), f64(lo), f64(hi)
    return np.minimum(g * lo[..., None, :], g * hi[..., None, :]).sum(-1) + h


def clip_single_literal(g, h, lo, hi):
    """Thm 3.2 for ONE constraint written out literally with the O(n^2)
    sum over j != i, in the centre/radius form.  g: [n], h: scalar.
    Returns (new_lo, new_hi, infeasible)."""
    g, lo, hi = f64(g), f64(lo), f64(hi)
    h = float(h)
    n = g.size
    xh = (lo + hi) / 2.0
    eps = (hi - lo) / 2.0
    m = float(np.sum(g * xh - np.abs(g) * eps) + h)
    new_lo, new_hi = lo.copy(), hi.copy()
    if m > 0.0:
        return new_lo, new_hi, True
    for i in range(n):
        if g[i] == 0.0:
            continue
        s = 0.0
        for j in range(n):
            if j != i:
                s += g[j] * xh[j] - abs(g[j]) * eps[j]
        x_clip = (-s - h) / g[i]
        if g[i] > 0.0:
            new_hi[i] = min(new_hi[i], x_clip)
        else:
            new_lo[i] = max(new_lo[i], x_clip)
    return new_lo, new_hi, bool(np.any(new_lo > new_hi))


def clip_candidates(g, h, lo, hi):
    """Per-constraint closed-form candidates, vectorised.

    Using sum_{j != i} = m - h - (g_i xh_i - |g_i| eps_i), the clip value is
    lo_i - m/g_i for g_i > 0 and hi_i - m/g_i for g_i < 0 (same value as the
    literal form).  g: [..., k, n], h: [..., k], lo/hi: [..., n].
    Returns (m [...,k], cand_hi [...,k,n] (+inf where g<=0),
    cand_lo [...,k,n] (-inf where g>=0))."""
    g, h, lo, hi = f64(g), f64(h), f64(lo), f64(hi)
    m = constraint_min(g, h, lo, hi)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = m[..., None] / g
    cand_hi = np.where(g > 0.0, lo[..., None, :] - r, np.inf)
    cand_lo = np.where(g < 0.0, hi[..., None, :] - r, -np.inf)
    return m, cand_hi, cand_lo


def clip_parallel(G, h, lo, hi, active=None):
    """Alg. 2 (parallel relaxed clipping) for a batch.

    G: [B, k, n], h: [B, k], lo/hi: [B, n]; ``active``: [B, k] bool mask of
    used constraint slots (None = all).  Returns (lo', hi', infeasible[B])."""
    G, h, lo, hi = f64(G), f64(h), f64(lo), f64(hi)
    if active is None:
        active = np.ones(h.shape, bool)
    m, cand_hi, cand_lo = clip_candidates(G, h, lo, hi)
    cand_hi = np.where(active[..., None], cand_hi, np.inf)
    cand_lo = np.where(active[..., None], cand_lo, -np.inf)
    new_hi = np.minimum(hi, cand_hi.min(axis=-2) if G.shape[-2] else hi)
    new_lo = np.maximum(lo, cand_lo.max(axis=-2) if G.shape[-2] else lo)
    infeas = np.any(np.where(active, m > 0.0, False), axis=-1) | np.any(new_lo > new_hi, axis=-1)
    return new_lo, new_hi, infeas


def clip_sequential(G, h, lo, hi, active=None):
    """Alg. 3 (sequential relaxed clipping): constraint k is applied to the
    box produced by constraints 1..k-1, in the given order."""
    G, h, lo, hi = f64(G), f64(h), f64(lo), f64(hi)
    B, k, n = G.shape
    if active is None:
        active = np.ones((B, k), bool)
    lo, hi = lo.copy(), hi.copy()
    infeas = np.zeros(B, bool)
    for kk in range(k):
        m, cand_hi, cand_lo = clip_candidates(G[:, kk:kk + 1], h[:, kk:kk + 1], lo, hi)
        a = active[:, kk]
        infeas |= a & (m[:, 0] > 0.0)
        upd = a & ~infeas
        hi = np.where(upd[:, None], np.minimum(hi, cand_hi[:, 0]), hi)
        lo = np.where(upd[:, None], np.maximum(lo, cand_lo[:, 0]), lo)
    infeas |= np.any(lo > hi, axis=-1)
    return lo, hi, infeas
