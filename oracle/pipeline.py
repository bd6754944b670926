"""The batched per-subdomain clip-and-verify pipeline, the slope adjoint and
Adam (FP64 oracle).

Steps, for one property whose root planes were cached by ``crown.root_pass``
and a batch of subdomains (input box + activation split list each):

(1) split -> input halfspace (eqs. 9-10 of the activation-BaB section): the
   branch z_j >= 0 gives  -Ahi_j x - chi_j <= 0  (because z_j <= Ahi_j x + chi_j);
   the branch z_j <= 0 gives  Alo_j x + clo_j <= 0 (because z_j >= Alo_j x + clo_j).
(2) relaxed clipping of the box (Thm 3.2 / Alg. 2, or Alg. 3).
(3) re-concretization of every cached plane over the clipped box (the
   "re-concretize cached linear constraints over the shrunk box" step of the
   relaxed-clipping section), intersected with the root bounds; a split
   neuron is fixed to its branch (l >= 0 for z >= 0, u <= 0 for z <= 0) as
   in Alg. 5, where children fix each split neuron's regime.
(4) (optional) complete clipping of unstable intermediate neurons: the cached
   lower plane (and the negated upper plane) are the objectives, the split
   halfspaces the constraints (Alg. 1).
(5) CROWN backward pass for the objective rows with the per-subdomain bounds.
(6) concretization of the final plane over the clipped box (Lemma A.2).
(7) complete clipping of each final plane against the subdomain's split
   halfspaces (Alg. 1, one pass); lb <- max(lb, result).

A subdomain is infeasible if (2) finds an empty constraint (or lo > hi), (3)/(4)
leave some neuron with l > u, or (7) finds a constraint empty over the clipped
box; its bounds are +inf.  It is verified if infeasible or every objective
row has lb > 0 (MinPool conjunction, appendix on Boolean properties).

The slope step (8): the gradient of sum(lb) after (7) with respect to the
alpha of every unstable lower-line entry, holding the (7) multipliers fixed
(Danskin), followed by projected Adam ascent (the experimental settings use
Adam on alpha with lr 0.1, 20 iterations, optional decay 0.98).

Readings taken:
* Intermediate bounds are intersected with the root bounds, and split
  neurons are fixed to their branch (the 2-D toy example leaves the split
  neuron unfixed to show clipping alone; ``Config.split_fix=False`` gives
  that behaviour).
* Optimised alpha is one value per (subdomain, objective row, neuron), the
  loss is the sum of the rows' bounds (separable per row).  Root planes use a
  fixed alpha (0.5).
* At a kink of the final dual (a coefficient of A + beta^T G that is zero in
  exact arithmetic, which happens at the breakpoint chosen by (7)) the
  subgradient uses the box midpoint for that coordinate: any point of
  [lo_j, hi_j] is a valid subgradient there; the midpoint is the symmetric
  choice.  ``kink_tol`` bounds the float64 residue such a zero leaves.
"""
from dataclasses import dataclass

import numpy as np

from . import relaxed as rx
from . import complete as cc
from . import crown
from .box import f64, concretize_min, concretize_min_shared, concretize_max_shared

U64 = 2.0 ** -53   # unit roundoff of float64


def kink_tol(k):
    """Relative bound on the float64 residue of a coefficient of
    A + beta^T G that exact arithmetic makes zero.  beta_k = -a'_j / g_kj is
    formed from a'_j = A_j + sum_{p != k} beta_p G_pj (off by at most
    gamma_k s_j, s_j = |A_j| + sum_p beta_p |G_pj|) and one rounded division;
    A_j + sum_p beta_p G_pj is then summed again (gamma_{k+1} s_j).  Together
    at most (2k + 2) u s_j (1 + 1%); (2k + 8) u leaves room.  k: number of
    constraint slots."""
    return (2 * k + 8) * U64


@dataclass
class Config:
    relaxed: str = "parallel"        # "parallel" | "sequential" | "none"
    reconcretize: bool = True        # step (3)
    split_fix: bool = True
    complete_intermediate: bool = False  # step (4)
    complete_final: bool = True      # step (7)
    ca_passes: int = 1
    alpha: float = 0.5
    order: bool = False              # constraint importance order (heuristics appendix)
    intermediate: str = "reconcretize"   # step (3): "reconcretize" | "crown" (fresh box)
    topk: int = -1                   # step (4) on the top-k neurons per layer by BaBSR score
                                     # (-1: every unstable neuron)
    babsr_weight: object = None      # [N] weights of the score (see babsr_weights)


def split_constraints(root, neuron, sign, count):
    """Step (1): halfspaces G x + h <= 0 of each subdomain's splits (eqs. 9-10).
    neuron/sign: [B, kmax]; count: [B].  Returns (G [B,k,n0], h [B,k],
    active [B,k])."""
    A_lo, c_lo, A_hi, c_hi, _, _ = root.stacked()
    B, k = neuron.shape
    active = np.arange(k)[None, :] < np.asarray(count)[:, None]
    idx = np.where(active, neuron, 0)
    neg = (np.asarray(sign) < 0)[..., None]
    G = np.where(neg, A_lo[idx], -A_hi[idx])
    h = np.where(neg[..., 0], c_lo[idx], -c_hi[idx])
    G = np.where(active[..., None], G, 0.0)
    h = np.where(active, h, 0.0)
    return G, h, active


def constraint_order(G, h, active, lo, hi):
    """Constraint importance order of the heuristics appendix: the distance
    d = |g.xc + h| / ||g||_2 of each constraint's hyperplane from the centre xc
    of the box, ascending (closest first); ties keep the list order.  Inactive
    slots and rows with g = 0 (no hyperplane) go last.  Returns order [B, k]:
    position -> constraint index.

    Readings taken: the centre is that of the box the constraints are applied
    to at that step (the original box for sequential relaxed clipping, the
    clipped box for complete clipping).  The paper also drops redundant
    constraints (satisfied on the whole box) and flags empty ones; neither
    changes a result here (a redundant constraint clips nothing and gets a
    zero multiplier, an empty one is detected where it is applied), so the
    order is all this step produces."""
    xc = 0.5 * (f64(lo) + f64(hi))
    num = np.abs(np.einsum("bkn,bn->bk", G, xc) + h)
    nrm = np.sqrt(np.einsum("bkn,bkn->bk", G, G))
    with np.errstate(divide="ignore", invalid="ignore"):
        d = np.where(nrm > 0.0, num / np.where(nrm > 0.0, nrm, 1.0), np.inf)
    d = np.where(active, d, np.inf)
    return np.argsort(d, axis=1, kind="stable")


def apply_order(order, G, h, active):
    """Constraint list permuted to ``order`` (position -> constraint index)."""
    return (np.take_along_axis(G, order[..., None], axis=1), np.take_along_axis(h, order, axis=1),
            np.take_along_axis(active, order, axis=1))


def reconcretize(root, lo, hi):
    """Step (3) without the fixes: bounds of every hidden neuron over each box.
    Returns (l [B, N], u [B, N])."""
    A_lo, c_lo, A_hi, c_hi, _, _ = root.stacked()
    return concretize_min_shared(A_lo, c_lo, lo, hi), concretize_max_shared(A_hi, c_hi, lo, hi)


def fix_bounds(root, l, u, neuron, sign, count, split_fix=True):
    """Intersect with the root bounds and fix split neurons to their branch.
    Returns (l, u, empty [B]) where empty marks some l > u."""
    _, _, _, _, l0, u0 = root.stacked()
    l = np.maximum(l, l0[None])
    u = np.minimum(u, u0[None])
    if split_fix:
        B, k = neuron.shape
        for s in range(k):
            act = s < np.asarray(count)
            b = np.nonzero(act)[0]
            j = neuron[b, s]
            pos = sign[b, s] > 0
            l[b[pos], j[pos]] = np.maximum(l[b[pos], j[pos]], 0.0)
            u[b[~pos], j[~pos]] = np.minimum(u[b[~pos], j[~pos]], 0.0)
    return l, u, np.any(l > u, axis=-1)


def babsr_weights(layers, C, t, root, alpha0=0.5):
    """Weights of the neuron-selection score (heuristics appendix): for
    neuron k, max(0, -mean_m Psi_mk), where Psi_mk is the coefficient with
    which the output of ReLU k enters the lower bound of objective row m
    (CROWN at the root bounds with the root slope).  Reading taken: the
    paper's "mean of the lower-bound A of neuron k" is this mean over the
    objective rows, taken once per property from the root pass."""
    l_list = [x[None] for x in root.l]
    u_list = [x[None] for x in root.u]
    _, _, psis = crown.backward(layers, C, t, l_list, u_list, alpha0, trace=True)
    return np.concatenate([np.maximum(0.0, -p[0].mean(axis=0)) for p in psis])


def babsr_scores(l, u, weight):
    """score_k = max(0, -l_k) max(0, u_k) / (u_k - l_k) * weight_k for unstable
    neurons (l_k < 0 < u_k), 0 otherwise.  l, u: [B, N]; weight: [N]."""
    unst = (l < 0.0) & (u > 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        icpt = np.where(unst, np.maximum(0.0, -l) * np.maximum(0.0, u) / np.where(unst, u - l, 1.0), 0.0)
    return icpt * weight[None, :]


def topk_select(l, u, weight, layer_sizes, k):
    """For every subdomain and hidden layer, the k unstable neurons with the
    largest score (ties: lower index first); mask [B, N]."""
    sc = babsr_scores(l, u, weight)
    unst = (l < 0.0) & (u > 0.0)
    sel = np.zeros(l.shape, bool)
    off = 0
    for n in layer_sizes:
        for b in range(l.shape[0]):
            idx = np.nonzero(unst[b, off:off + n])[0]
            # sort by score descending, index ascending
            order = idx[np.lexsort((idx, -sc[b, off + idx]))]
            sel[b, off + order[:k]] = True
        off += n
    return sel


def complete_intermediate(root, l, u, G, h, active, lo, hi, passes=1, select=None):
    """Step (4): complete clipping of every unstable neuron's cached lower plane
    (tightens l) and negated upper plane (tightens u); with ``select`` [B, N]
    only the selected neurons.  Returns (l, u, empty)."""
    A_lo, c_lo, A_hi, c_hi, _, _ = root.stacked()
    l, u = l.copy(), u.copy()
    empty = np.zeros(l.shape[0], bool)
    for b in range(l.shape[0]):
        mask = (l[b] < 0.0) & (u[b] > 0.0)
        if select is not None:
            mask &= select[b]
        js = np.nonzero(mask)[0]
        if js.size == 0 or not active[b].any():
            continue
        R = js.size
        Gr = np.broadcast_to(G[b], (R,) + G[b].shape)
        hr = np.broadcast_to(h[b], (R,) + h[b].shape)
        ar = np.broadcast_to(active[b], (R,) + active[b].shape)
        lor = np.broadcast_to(lo[b], (R, lo.shape[1]))
        hir = np.broadcast_to(hi[b], (R, hi.shape[1]))
        Ll, _, inf1 = cc.coord_ascent(A_lo[js], c_lo[js], Gr, hr, lor, hir, ar, passes)
        Lu, _, inf2 = cc.coord_ascent(-A_hi[js], -c_hi[js], Gr, hr, lor, hir, ar, passes)
        l[b, js] = np.maximum(l[b, js], Ll)
        u[b, js] = np.minimum(u[b, js], -Lu)
        empty[b] = bool(inf1.any() or inf2.any())
    return l, u, empty | np.any(l > u, axis=-1)


def crown_intermediate(layers, root, lo, hi, l, u, alpha0=0.5):
    """Bounds of a fresh box (input BaB): for hidden layers 2..L-1 in order,
    CROWN with objectives +I and -I on the layer's pre-activations over the
    cut network, using the box's own bounds of the earlier layers,
    concretized over each box and intersected with the bounds given (l, u
    [B, N]: valid bounds, e.g. the re-concretized cached planes)."""
    l, u = l.copy(), u.copy()
    off = layers[0][0].shape[0]
    for i in range(2, len(layers)):
        n_i = layers[i - 1][0].shape[0]
        sub = layers[:i]
        ll = split_layers(layers, l)[:i - 1]
        uu = split_layers(layers, u)[:i - 1]
        I = np.eye(n_i)
        A1, c1 = crown.backward(sub, I, np.zeros(n_i), ll, uu, alpha0)
        A2, c2 = crown.backward(sub, -I, np.zeros(n_i), ll, uu, alpha0)
        l[:, off:off + n_i] = np.maximum(l[:, off:off + n_i], concretize_min(A1, c1, lo, hi))
        u[:, off:off + n_i] = np.minimum(u[:, off:off + n_i], -concretize_min(A2, c2, lo, hi))
        off += n_i
    return l, u


def split_layers(net_layers, flat):
    """Cut [B, N] concatenated hidden quantities into per-layer arrays."""
    out, off = [], 0
    for W, _ in net_layers[:-1]:
        n = W.shape[0]
        out.append(flat[:, off:off + n])
        off += n
    return out


def final_clip(A, c, G, h, active, lo, hi, passes=1):
    """Step (7) for a batch: rows (b, m) of A [B, M, n] / c [B, M] against the
    constraints of subdomain b.  Returns (L [B, M], beta [B, M, k], empty [B])."""
    B, M, n = A.shape
    k = G.shape[1]
    rep = lambda x: np.repeat(x, M, axis=0)
    L, beta, inf = cc.coord_ascent(A.reshape(B * M, n), c.reshape(B * M), rep(G), rep(h),
                                   rep(lo), rep(hi), rep(active), passes)
    return L.reshape(B, M), beta.reshape(B, M, k), inf.reshape(B, M).any(-1)


def run(layers, root, C, t, lo, hi, neuron, sign, count, cfg=Config(), alpha=None, dense=None):
    """Steps (1)-(7) for a batch of subdomains; returns a dict of every
    intermediate result.  ``layers``: dense (W, b) list; lo/hi: [B, n0];
    alpha: None (use cfg.alpha) or per-layer [B, M, n_i] arrays.  ``dense``:
    (G [B,k,n0], h [B,k], active [B,k]) constraints used instead of splits
    (e.g. a parent's final plane in input BaB; no split fix then)."""
    lo, hi = f64(lo), f64(hi)
    out = {}
    if dense is not None:
        G, h, act = (f64(dense[0]), f64(dense[1]), np.asarray(dense[2], bool))
        B = lo.shape[0]
        neuron, sign, count = np.zeros((B, 0), int), np.zeros((B, 0), int), np.zeros(B, int)
    else:
        G, h, act = split_constraints(root, neuron, sign, count)
    if cfg.relaxed == "parallel":
        lo2, hi2, inf_clip = rx.clip_parallel(G, h, lo, hi, act)
    elif cfg.relaxed == "sequential":
        Gs, hs, acts = G, h, act
        if cfg.order:
            Gs, hs, acts = apply_order(constraint_order(G, h, act, lo, hi), G, h, act)
        lo2, hi2, inf_clip = rx.clip_sequential(Gs, hs, lo, hi, acts)
    else:
        lo2, hi2, inf_clip = lo.copy(), hi.copy(), np.zeros(lo.shape[0], bool)
    if cfg.order:
        # complete clipping (and the slope steps after it) take the
        # constraints closest to the clipped box's centre first
        out["order"] = constraint_order(G, h, act, lo2, hi2)
        G, h, act = apply_order(out["order"], G, h, act)
    out.update(G=G, h=h, active=act, lo=lo2, hi=hi2, infeasible_clip=inf_clip)
    # bounds are computed on the clipped box; an empty box keeps its values
    if cfg.reconcretize:
        l, u = reconcretize(root, lo2, hi2)
    else:
        _, _, _, _, l0, u0 = root.stacked()
        l = np.broadcast_to(l0, (lo.shape[0], l0.size)).copy()
        u = np.broadcast_to(u0, (lo.shape[0], u0.size)).copy()
    l, u, emp_r = fix_bounds(root, l, u, neuron, sign, count, cfg.split_fix)
    if cfg.intermediate == "crown":
        l, u = crown_intermediate(layers, root, lo2, hi2, l, u)
        emp_r = emp_r | np.any(l > u, axis=-1)
    out.update(l_reconc=l.copy(), u_reconc=u.copy(), empty_reconc=emp_r)
    emp_n = np.zeros_like(emp_r)
    if cfg.complete_intermediate:
        sel = None
        if cfg.topk >= 0:
            sel = topk_select(l, u, f64(cfg.babsr_weight), [W.shape[0] for W, _ in layers[:-1]],
                              cfg.topk)
            out["select"] = sel
        l, u, emp_n = complete_intermediate(root, l, u, G, h, act, lo2, hi2, cfg.ca_passes, sel)
    out.update(l=l, u=u, empty_neurons=emp_n)
    a = cfg.alpha if alpha is None else alpha
    A, c = crown.backward(layers, C, t, split_layers(layers, l), split_layers(layers, u), a)
    lb0 = concretize_min(A, c, lo2, hi2)
    out.update(A=A, c=c, lb_unclipped=lb0.copy())
    emp_f = np.zeros_like(emp_r)
    lb = lb0
    if cfg.complete_final and G.shape[1] > 0:
        L, beta, emp_f = final_clip(A, c, G, h, act, lo2, hi2, cfg.ca_passes)
        lb = np.maximum(lb0, L)
        out["beta"] = beta
    infeasible = inf_clip | emp_r | emp_n | emp_f
    lb = np.where(infeasible[:, None], np.inf, lb)
    out.update(lb=lb, infeasible=infeasible, empty_final=emp_f,
               verified=infeasible | np.all(lb > 0.0, axis=-1))
    return out


# ---------------------------------------------------------- slopes, step (8)

def bound_and_grad(layers, C, t, l_list, u_list, alpha, lo, hi, G, h, active,
                   complete=True, passes=1):
    """Post-(7) bound of every row and its gradient with respect to alpha.

    alpha: list of [B, M, n_i] (one per hidden layer).  The multipliers of (7)
    are held fixed (Danskin), so the bound is min over the box of
    (A + beta^T G).x + c + beta^T h and its derivative with respect to A is
    the minimising corner x* (midpoint at zero coefficients).  The adjoint
    then runs the CROWN recursion backwards:
        Omega_bar_k = Psi_bar_k W_k^T + b_k,   Psi_bar_0 = x*
        Psi_bar_{k+1} = Omega_bar_k * slope_k + intercept_k
        dlb/dalpha_k = Omega_bar_k * Psi_{k+1}   on lower-line entries.
    Returns (lb [B, M], grads list, beta or None, infeasible rows [B])."""
    lo, hi = f64(lo), f64(hi)
    A, c, psis = crown.backward(layers, C, t, l_list, u_list, alpha, trace=True)
    B, M, n = A.shape
    beta = None
    if complete and G.shape[1] > 0:
        L, beta, emp = final_clip(A, c, G, h, active, lo, hi, passes)
        Af = A + np.einsum("bmk,bkn->bmn", beta, G)
        cf = c + np.einsum("bmk,bk->bm", beta, h)
    else:
        emp = np.zeros(B, bool)
        Af, cf = A, c
    lb = concretize_min(Af, cf, lo, hi)
    scale = np.abs(A)
    if beta is not None:
        scale = scale + np.einsum("bmk,bkn->bmn", beta, np.abs(G))
    kink = np.abs(Af) <= kink_tol(G.shape[1]) * scale
    xstar = np.where(kink, (lo[:, None, :] + hi[:, None, :]) / 2.0,
                     np.where(Af > 0.0, lo[:, None, :], hi[:, None, :]))
    grads = [None] * (len(layers) - 1)
    Psi_bar = xstar
    for kk in range(len(layers) - 1):
        W, b = layers[kk]
        Om_bar = Psi_bar @ W.T + b
        l = f64(l_list[kk])[:, None, :]
        u = f64(u_list[kk])[:, None, :]
        slope, icpt, mask = crown.relu_relaxation(l, u, psis[kk], alpha[kk])
        grads[kk] = np.where(mask, Om_bar * psis[kk], 0.0)
        Psi_bar = Om_bar * slope + icpt
    for kk in range(len(grads)):
        grads[kk] = np.where(emp[:, None, None], 0.0, grads[kk])
    lb = np.where(emp[:, None], np.inf, lb)
    return lb, grads, beta, emp


def adam_ascent(param, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One projected Adam ascent step (Kingma & Ba; bias-corrected moments),
    then clamp to [0, 1].  Returns (param, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    param = np.clip(param + lr * mh / (np.sqrt(vh) + eps), 0.0, 1.0)
    return param, m, v


def alpha_opt(layers, C, t, l_list, u_list, lo, hi, G, h, active, steps=20,
              lr=0.1, alpha0=0.5, decay=1.0, complete=True, passes=1, b1=0.9, b2=0.999,
              eps=1e-8, state32=False):
    """Step (8) repeated: ``steps`` iterations of (bound, gradient, Adam) starting
    from alpha0 everywhere.  Returns (best lb over the iterations [B, M],
    per-iteration lb list, final alpha list).

    state32: the slopes and Adam moments are carried from one iteration to
    the next as float32 values (rounded to nearest after each update), which
    is how they cross the library's interface between its steps; every
    iteration still computes in float64 on the widened values."""
    B = lo.shape[0]
    M = C.shape[0]
    alpha = [np.full((B, M, W.shape[0]), alpha0) for W, _ in layers[:-1]]
    ms = [np.zeros_like(a) for a in alpha]
    vs = [np.zeros_like(a) for a in alpha]
    best = np.full((B, M), -np.inf)
    hist = []
    for s in range(1, steps + 1):
        lb, grads, _, _ = bound_and_grad(layers, C, t, l_list, u_list, alpha, lo, hi,
                                         G, h, active, complete, passes)
        hist.append(lb)
        best = np.maximum(best, lb)
        lr_s = lr * decay ** (s - 1)
        for kk in range(len(alpha)):
            alpha[kk], ms[kk], vs[kk] = adam_ascent(alpha[kk], grads[kk], ms[kk], vs[kk], s, lr_s,
                                                    b1, b2, eps)
            if state32:
                alpha[kk], ms[kk], vs[kk] = (x.astype(np.float32).astype(np.float64)
                                             for x in (alpha[kk], ms[kk], vs[kk]))
    return best, hist, alpha
