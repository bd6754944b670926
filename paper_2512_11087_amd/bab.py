"""Branch-and-bound loops around the batched clip-and-verify pass.

Activation BaB (Alg. 5) of one property or of many at once (a PropertySet:
one pool, each subdomain tagged with its property, all bounded in the same
launches): a subdomain is an input box with a list of ReLU
splits.  Each round takes up to `batch` unknown subdomains (oldest first),
splits each on one unstable neuron (cv_branch_relu: best BaBSR intercept
score), and bounds the 2x children with the full pass -- the new split is
turned into an input halfspace and clips the child's box (relaxed
clipping), the cached planes are re-concretized over it, the top-k critical
neurons are refined by complete clipping, CROWN bounds the objectives and
complete clipping tightens them.  Children that are infeasible or whose
every objective row has lb > 0 are verified and dropped.

Input BaB (Alg. 4, with the paper's reordering): a subdomain is an input
box with the final CROWN plane A x + c of its parent.  Each round splits
the picked boxes in two (cv_branch_input), clips both children by their
parent's plane (the region where the objective can be negative lies in
A x + c <= 0), bounds their hidden neurons afresh (cached planes
re-concretized, then CROWN over the box, cv_intermediate_bounds: the box
shrinks, so re-concretized root planes alone would not converge) and bounds
the objective with that plane as the constraint of complete clipping; each
child keeps its own plane for its children.  One objective row per run
(for several rows the violating region is a union, which one row's plane
cannot clip).

The pool lives in device memory; picking, filtering and appending are
tensor slicing.  Every bound, clip and branch is a library call.
"""
from dataclasses import dataclass, field

import torch

from . import api
from .pipeline import Batch, PassConfig, input_pass, plain_pass


@dataclass
class BabResult:
    verified: bool            # every subdomain verified or infeasible
    iterations: int
    visited: int              # subdomains bounded (children included)
    remaining: int            # unknown subdomains left (limits reached)
    stuck: int = 0            # unknown subdomains that cannot be split further
    history: list = field(default_factory=list)   # unknown count after each round
    per_property: list = None  # property set: verified flag of each property


def _verified(out):
    inf = out["infeasible"].bool()
    return inf | (out["lb"] > 0).all(dim=-1)


def activation_bab(prop, batch=1024, max_iters=100, max_domains=1 << 20, kmax=64,
                   cfg=PassConfig(complete_intermediate=True, topk=20)):
    """Activation BaB over the root box of one property, or of every property
    of a PropertySet at once (one pool; each subdomain carries its property
    index, children inherit it).  Returns BabResult (per_property for a set)."""
    root = prop.root
    weight = prop.babsr_weight()
    P = getattr(prop, "P", 1)
    if P > 1:
        lo, hi, pid = prop.boxes([1] * P)
    else:
        (lo, hi), pid = prop.boxes(1), None
    R0 = lo.shape[0]
    cons = api.Constraints.splits(torch.zeros(R0, kmax, dtype=torch.int32),
                                  torch.zeros(R0, kmax, dtype=torch.int8),
                                  torch.zeros(R0, dtype=torch.int32))
    out = plain_pass(prop, Batch(lo.clone(), hi.clone(), cons, pid=pid), cfg)
    done0 = _verified(out)
    if bool(done0.all()):
        return BabResult(True, 0, R0, 0, per_property=[True] * P if P > 1 else None)
    # pool: boxes, split lists, bounds (and property) of every unknown subdomain
    keep0 = ~done0
    pool = dict(lo=lo[keep0], hi=hi[keep0], neuron=cons.neuron[keep0], sign=cons.sign[keep0],
                count=cons.count[keep0], l=out["l"][keep0], u=out["u"][keep0])
    if pid is not None:
        pool["pid"] = pid[keep0]
    stuck_pid = []
    visited, stuck, it, hist = R0, 0, 0, []
    while pool["lo"].shape[0] > 0 and it < max_iters:
        it += 1
        D = pool["lo"].shape[0]
        take = min(batch, D)
        par = {k: v[:take] for k, v in pool.items()}
        rest = {k: v[take:] for k, v in pool.items()}
        pcons = api.Constraints(kmax, par["count"].contiguous(), par["neuron"].contiguous(),
                                par["sign"].contiguous())
        ppid = par["pid"].contiguous() if "pid" in par else None
        chosen, ccons, lo2, hi2 = api.branch_relu(root, par["l"].contiguous(), par["u"].contiguous(),
                                                  weight, pcons, par["lo"].contiguous(),
                                                  par["hi"].contiguous(), kmax, pid=ppid)
        cpid = ppid.repeat_interleave(2) if ppid is not None else None
        splittable = (chosen >= 0).repeat_interleave(2)
        out = plain_pass(prop, Batch(lo2, hi2, ccons, pid=cpid), cfg)
        visited += 2 * take
        done = _verified(out)
        keep = ~done & splittable
        # a parent with nothing left to split and an unverified bound cannot be refined
        stuck_mask = ~done & ~splittable
        stuck += int(stuck_mask.sum()) // 2
        if cpid is not None and bool(stuck_mask.any()):
            stuck_pid.append(cpid[stuck_mask])
        kids = dict(lo=lo2[keep], hi=hi2[keep], neuron=ccons.neuron[keep], sign=ccons.sign[keep],
                    count=ccons.count[keep], l=out["l"][keep], u=out["u"][keep])
        if cpid is not None:
            kids["pid"] = cpid[keep]
        pool = {k: torch.cat([rest[k], kids[k]], 0) for k in pool}
        hist.append(int(pool["lo"].shape[0]))
        if pool["lo"].shape[0] > max_domains:
            break
    remaining = int(pool["lo"].shape[0])
    per = None
    if P > 1:
        bad = torch.zeros(P, dtype=torch.bool)
        if remaining:
            bad[pool["pid"].long().cpu()] = True
        for sp_ in stuck_pid:
            bad[sp_.long().cpu()] = True
        per = [not bool(b) for b in bad]
    return BabResult(remaining == 0 and stuck == 0, it, visited, remaining, stuck, hist, per)


def input_bab(prop, batch=1024, max_iters=100, max_domains=1 << 20, cfg=PassConfig()):
    """Input BaB of a one-row property (prop.M == 1).  Returns BabResult."""
    if prop.M != 1:
        raise ValueError("input_bab bounds one objective row (see the module docstring)")
    lo, hi = prop.boxes(1)
    out = input_pass(prop, Batch(lo.clone(), hi.clone(), None), cfg)
    if bool(_verified(out).all()):
        return BabResult(True, 0, 1, 0)
    pool = dict(lo=lo, hi=hi, A=out["A"][:, 0, :], c=out["c"][:, 0])
    visited, it, hist = 1, 0, []
    while pool["lo"].shape[0] > 0 and it < max_iters:
        it += 1
        D = pool["lo"].shape[0]
        take = min(batch, D)
        par = {k: v[:take].contiguous() for k, v in pool.items()}
        rest = {k: v[take:] for k, v in pool.items()}
        _, lo2, hi2 = api.branch_input(par["lo"], par["hi"], par["A"][:, None, :])
        # both children take their parent's plane as the constraint A x + c <= 0
        G = par["A"].repeat_interleave(2, 0)[:, None, :].contiguous()
        h = par["c"].repeat_interleave(2, 0)[:, None].contiguous()
        ccons = api.Constraints.dense(G, h)
        out = input_pass(prop, Batch(lo2, hi2, ccons), cfg)
        visited += 2 * take
        keep = ~_verified(out)
        kids = dict(lo=lo2[keep], hi=hi2[keep], A=out["A"][keep][:, 0, :], c=out["c"][keep][:, 0])
        pool = {k: torch.cat([rest[k], kids[k]], 0) for k in pool}
        hist.append(int(pool["lo"].shape[0]))
        if pool["lo"].shape[0] > max_domains:
            break
    remaining = int(pool["lo"].shape[0])
    return BabResult(remaining == 0, it, visited, remaining, 0, hist)
