"""Branching rules of the two branch-and-bound loops (oracle side).

Activation BaB (Alg. 5): each picked subdomain is split on one unstable
neuron into the branches z <= 0 and z >= 0; the neuron is the one with the
largest BaBSR intercept score (the same score as the neuron-selection
heuristic of the heuristics appendix) among the unstable neurons not split
yet, ties to the lower index.

Input BaB (Alg. 4): each picked box is split in two along one input
dimension at its midpoint; both children inherit the parent's final plane
A x + c (the region where the objective can be negative, A x + c <= 0, is
the constraint they are clipped by).  Reading taken: the paper does not
name the input-splitting rule; the dimension with the largest
(hi_d - lo_d) * sum_m |A_md| (the largest possible change of the plane's
concretized bound) is taken, ties to the lower index.
"""
import numpy as np

from .box import f64
from .pipeline import babsr_scores


def branch_relu(l, u, weight, neuron, sign, count):
    """Neuron to split for every subdomain: [B] global index, -1 when no
    unstable neuron is left unsplit."""
    sc = babsr_scores(f64(l), f64(u), f64(weight))
    unst = (l < 0.0) & (u > 0.0)
    out = np.full(l.shape[0], -1, np.int64)
    for b in range(l.shape[0]):
        cand = unst[b].copy()
        cand[np.asarray(neuron[b, :count[b]], np.int64)] = False
        idx = np.nonzero(cand)[0]
        if idx.size:
            out[b] = idx[np.lexsort((idx, -sc[b, idx]))][0]
    return out


def children_relu(neuron, sign, count, lo, hi, chosen):
    """Children 2b (branch z <= 0) and 2b + 1 (branch z >= 0) of every
    subdomain b with a chosen neuron: the parent's splits plus the new one,
    the parent's box."""
    B, k = neuron.shape
    n2 = np.repeat(neuron, 2, axis=0)
    s2 = np.repeat(sign, 2, axis=0)
    c2 = np.repeat(count, 2)
    pad = np.zeros((2 * B, 1), n2.dtype)
    n2 = np.concatenate([n2, pad], 1)
    s2 = np.concatenate([s2, pad.astype(s2.dtype)], 1)
    for b in range(B):
        if chosen[b] < 0:
            continue
        for side, sg in ((0, -1), (1, 1)):
            r = 2 * b + side
            n2[r, c2[r]] = chosen[b]
            s2[r, c2[r]] = sg
            c2[r] += 1
    return n2, s2, c2, np.repeat(lo, 2, axis=0), np.repeat(hi, 2, axis=0)


def branch_input(lo, hi, A):
    """Input dimension to split for every box: [B].  A: [B, M, n]."""
    score = (f64(hi) - f64(lo)) * np.abs(f64(A)).sum(axis=1)
    # argmax returns the first maximum: ties go to the lower index
    return np.argmax(score, axis=1)


def children_input(lo, hi, dim):
    """Children 2b (lower half) and 2b + 1 (upper half) of each box, split at
    the midpoint of dimension dim[b] (computed in float32 like the boxes, so
    the two halves share their cut exactly)."""
    B = lo.shape[0]
    lo2 = np.repeat(lo, 2, axis=0).copy()
    hi2 = np.repeat(hi, 2, axis=0).copy()
    for b in range(B):
        d = dim[b]
        mid = np.float32(0.5) * (np.float32(lo[b, d]) + np.float32(hi[b, d]))
        hi2[2 * b, d] = mid
        lo2[2 * b + 1, d] = mid
    return lo2, hi2
