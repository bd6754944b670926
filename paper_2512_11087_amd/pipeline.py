"""The batched clip-and-verify pass over one property or a set of
properties (Batch.pid: the property of each subdomain), sequenced on the
device through the C ABI:

  split halfspaces + relaxed clipping     (clip_domains)
  re-concretization of cached planes      (concretize_planes)
  CROWN backward + concretization
  + complete clipping of the final plane  (bound_propagate)
  slope optimisation                      (alpha_step, repeated)

Every step is a HIP kernel; this module only allocates device buffers and
orders the calls on the current stream.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import api


@dataclass
class PassConfig:
    clip: str = "parallel"          # "parallel" | "sequential" | "none"
    complete_intermediate: bool = False
    complete_final: bool = True
    passes: int = 1
    alpha: float = 0.5
    order: bool = False             # constraint importance order (heuristics appendix)
    topk: int = -1                  # complete_intermediate on the top-k per layer (-1: all)


class Property:
    """A network, root box and specification resident on the device."""

    P = 1

    def __init__(self, layers, lo0, hi0, C, t, alpha0=0.5, planes="auto"):
        self.net = api.Net(layers)
        self.root = api.Root(self.net, lo0, hi0, alpha0, planes)
        self.C = api._f32(C)
        self.t = api._f32(t)
        self.M = self.C.shape[0]
        self.ws = api.Workspace()
        self.ws2 = api.Workspace()
        self._babsr = None

    def babsr_weight(self):
        """Per-neuron weights of the selection score, computed once."""
        if self._babsr is None:
            self._babsr = api.babsr_weights(self.net, self.root, self.C, self.t, self.ws)
        return self._babsr

    @classmethod
    def from_workload(cls, w):
        return cls(list(w.net.layers), w.lo0, w.hi0, w.C, w.t, w.alpha0)

    def boxes(self, B):
        lo = self.root.lo0.expand(B, -1).contiguous()
        hi = self.root.hi0.expand(B, -1).contiguous()
        return lo, hi


class PropertySet:
    """P properties over one network (each its own root box and objective),
    bounded in the same launches: ``root`` is an api.RootSet, C [P, M, n_out],
    t [P, M]; a batch's ``pid`` gives each subdomain's property."""

    def __init__(self, layers, lo0s, hi0s, Cs, ts, alpha0=0.5, planes="auto", net=None,
                 progress=None):
        """progress: called with the number of roots made so far after each."""
        self.net = net if net is not None else api.Net(layers)
        self.roots = []
        for lo, hi in zip(lo0s, hi0s):
            self.roots.append(api.Root(self.net, lo, hi, alpha0, planes))
            if progress is not None:
                progress(len(self.roots))
        self.root = api.RootSet(self.roots)
        self.P = len(self.roots)
        self.C = api._f32(np.stack([np.asarray(c, np.float32) for c in Cs]))
        self.t = api._f32(np.stack([np.asarray(x, np.float32) for x in ts]))
        self.M = self.C.shape[1]
        self.ws = api.Workspace()
        self.ws2 = api.Workspace()
        self._babsr = None

    def babsr_weight(self):
        """Per-property weights of the selection score [P, n_hidden]."""
        if self._babsr is None:
            self._babsr = api.babsr_weights(self.net, self.root, self.C, self.t, self.ws)
        return self._babsr

    @classmethod
    def from_workload(cls, w):
        """From a workload with extra["properties"] = list of (lo0, hi0, C, t)."""
        ps = w.extra["properties"]
        return cls(list(w.net.layers), [p[0] for p in ps], [p[1] for p in ps],
                   [p[2] for p in ps], [p[3] for p in ps], w.alpha0)

    def boxes(self, counts):
        """Root boxes of counts[p] subdomains of each property, grouped by
        property, and their pid [B]."""
        counts = [int(c) for c in counts]
        lo = torch.cat([r.lo0.expand(c, -1) for r, c in zip(self.roots, counts)]).contiguous()
        hi = torch.cat([r.hi0.expand(c, -1) for r, c in zip(self.roots, counts)]).contiguous()
        pid = torch.repeat_interleave(torch.arange(self.P, dtype=torch.int32),
                                      torch.tensor(counts)).to("cuda")
        return lo, hi, pid


@dataclass
class Batch:
    lo: torch.Tensor
    hi: torch.Tensor
    splits: api.Constraints
    ordered: api.Constraints = None   # splits in importance order over the clipped box
    pid: torch.Tensor = None          # int32 [B] property of each subdomain (property sets)

    def cons(self):
        """The constraints as complete clipping takes them."""
        return self.ordered if self.ordered is not None else self.splits


def make_batch(prop, neuron, sign, count, lo=None, hi=None, pid=None):
    B = neuron.shape[0]
    if lo is None:
        lo, hi = prop.boxes(B)
    return Batch(lo, hi, api.Constraints.splits(neuron, sign, count), pid=pid)


def plain_pass(prop, batch, cfg=PassConfig(), out=None, planes=False):
    """One pass of the hot path over a batch; boxes are clipped in place.
    Returns dict(infeasible, l, u, lb) and, with ``planes``, the final CROWN
    plane of every row (A [B, M, n_in], c [B, M]; valid lower planes)."""
    B = batch.lo.shape[0]
    out = out if out is not None else {}
    clip_cons = batch.splits
    if cfg.order and cfg.clip == "sequential" and batch.splits is not None:
        # sequential clipping takes the constraints closest to the box centre first
        clip_cons = batch.splits.with_order(
            api.constraint_order(prop.root, batch.lo, batch.hi, batch.splits, out.get("order0"),
                                 pid=batch.pid))
        out["order0"] = clip_cons.order
    if cfg.clip != "none" and batch.splits is not None:
        inf = api.clip_domains(prop.root, batch.lo, batch.hi, clip_cons, cfg.clip,
                               infeasible=out.get("infeasible"), pid=batch.pid)
    else:
        inf = out.get("infeasible")
        if inf is None:
            inf = torch.zeros(B, dtype=torch.uint8, device="cuda")
        else:
            inf.zero_()
    batch.ordered = None
    if cfg.order and batch.splits is not None:
        # complete clipping: the order over the clipped box
        batch.ordered = batch.splits.with_order(
            api.constraint_order(prop.root, batch.lo, batch.hi, batch.splits, out.get("order1"),
                                 pid=batch.pid))
        out["order1"] = batch.ordered.order
    weight, select = None, None
    if cfg.complete_intermediate and cfg.topk >= 0:
        weight = prop.babsr_weight()
        select = out.get("select")
        if select is None:
            select = torch.empty(B, prop.net.n_hidden, dtype=torch.uint8, device="cuda")
        out["select"] = select
    l, u, inf = api.concretize_planes(prop.root, batch.lo, batch.hi, batch.cons(),
                                      cfg.complete_intermediate, cfg.passes, inf,
                                      out.get("l"), out.get("u"), prop.ws2, cfg.topk, weight, select,
                                      pid=batch.pid)
    cons = batch.cons() if cfg.complete_final else None
    res = api.bound_propagate(prop.net, prop.root, prop.C, prop.t, l, u, batch.lo, batch.hi,
                              None, cfg.alpha, inf, cons, cfg.passes, want_plane=planes, ws=prop.ws,
                              pid=batch.pid)
    if planes:
        lb, A, c = res
        out.update(A=A, c=c)
    else:
        lb = res
    out.update(infeasible=inf, l=l, u=u, lb=lb)
    return out


def alpha_opt(prop, batch, l, u, infeasible, steps=20, lr=0.1, decay=1.0, alpha0=0.5,
              complete=True, passes=1, state=None):
    """Slope optimisation: ``steps`` x (bound, adjoint, Adam).  Returns the
    best bound over the iterations [B, M] and the final alpha.  The first
    call starts from alpha0 with zero Adam moments and the library keeps the
    running best, so no other kernel runs between the calls."""
    B = batch.lo.shape[0]
    M, nh = prop.M, prop.net.n_hidden
    if state is None:
        state = {}
    if state.get("alpha") is None:
        alpha = torch.empty(B, M, nh, device="cuda")
        state.update(alpha=alpha, m=torch.empty_like(alpha), v=torch.empty_like(alpha),
                     best=torch.empty(B, M, device="cuda"))
    alpha, best = state["alpha"], state["best"]
    if steps < 1:
        alpha.fill_(alpha0)
        best.fill_(-float("inf"))
        return best, alpha
    cons = batch.cons() if complete else None
    for s in range(1, steps + 1):
        api.alpha_step(prop.net, prop.root, prop.C, prop.t, l, u, alpha, batch.lo, batch.hi,
                       infeasible, cons, passes, state["m"], state["v"], s, lr * decay ** (s - 1),
                       ws=prop.ws, pid=batch.pid, alpha_init=alpha0 if s == 1 else -1.0,
                       best=best)
    return best, alpha


def input_pass(prop, batch, cfg=PassConfig(), out=None):
    """Bounding of fresh input boxes (input BaB): relaxed clipping by the
    boxes' constraints (batch.splits, e.g. the parent's final plane in dense
    form), intermediate bounds from the cached planes tightened by CROWN over
    each box, the CROWN bound and complete clipping of the final plane
    against the constraints.  Returns dict(infeasible, l, u, lb, A, c)."""
    B = batch.lo.shape[0]
    out = out if out is not None else {}
    if prop.P != 1:
        raise ValueError("input_pass bounds one property (fresh-box intermediate bounds)")
    if cfg.clip != "none" and batch.splits is not None:
        inf = api.clip_domains(prop.root, batch.lo, batch.hi, batch.splits, cfg.clip,
                               infeasible=out.get("infeasible"))
    else:
        inf = torch.zeros(B, dtype=torch.uint8, device="cuda")
    l, u, inf = api.concretize_planes(prop.root, batch.lo, batch.hi, None, False, 1, inf,
                                      out.get("l"), out.get("u"), prop.ws2)
    api.intermediate_bounds(prop.net, prop.root, batch.lo, batch.hi, l, u, inf, prop.ws2)
    cons = batch.splits if cfg.complete_final else None
    lb, A, c = api.bound_propagate(prop.net, prop.root, prop.C, prop.t, l, u, batch.lo, batch.hi,
                                   None, cfg.alpha, inf, cons, cfg.passes, want_plane=True,
                                   ws=prop.ws)
    out.update(infeasible=inf, l=l, u=u, lb=lb, A=A, c=c)
    return out


class AlphaBound(torch.autograd.Function):
    """lb(alpha) [B, M] as a differentiable function of the slopes alpha
    [B, M, n_hidden]: the forward pass runs the bound (backward pass,
    concretization, complete clipping) and the hand-written adjoint kernel in
    one call; backward scales the stored per-row gradient by the incoming
    gradient (lb[b, m] depends only on alpha[b, m, :]).  The complete-
    clipping multipliers are held at their optimum (Danskin)."""

    @staticmethod
    def forward(ctx, alpha, prop, batch, l, u, infeasible, complete, passes):
        cons = batch.cons() if complete else None
        lb, grad = api.alpha_step(prop.net, prop.root, prop.C, prop.t, l, u, alpha.detach(),
                                  batch.lo, batch.hi, infeasible, cons, passes, want_grad=True,
                                  ws=prop.ws, pid=batch.pid)
        ctx.save_for_backward(grad)
        return lb

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g.unsqueeze(-1) * grad, None, None, None, None, None, None, None


def bound(prop, batch, l, u, alpha, infeasible, complete=True, passes=1):
    """Differentiable bound: ``bound(...).sum().backward()`` fills alpha.grad."""
    return AlphaBound.apply(alpha, prop, batch, l, u, infeasible, complete, passes)


class AlphaOptGraph:
    """Slope optimisation (`steps` x alpha_step, fixed batch and bounds)
    captured once into a HIP graph and replayed: the step index and learning
    rate of every iteration are baked into its launches, the buffers are
    allocated before capture (the calls themselves only launch kernels).
    ``run()`` starts from alpha0 with zero Adam moments (the first step's
    launches do that) and returns the best bound [B, M] over the iterations
    (a buffer the graph writes)."""

    def __init__(self, prop, batch, l, u, infeasible, steps=20, lr=0.1, decay=1.0, alpha0=0.5,
                 complete=True, passes=1):
        B, M, nh = batch.lo.shape[0], prop.M, prop.net.n_hidden
        self.alpha = torch.full((B, M, nh), alpha0, device="cuda")
        self.m = torch.zeros_like(self.alpha)
        self.v = torch.zeros_like(self.alpha)
        self.best = torch.full((B, M), -float("inf"), device="cuda")
        self.lbs = [torch.empty(B, M, device="cuda") for _ in range(steps)]
        cons = batch.cons() if complete else None
        # size the workspace outside the capture
        api.alpha_step(prop.net, prop.root, prop.C, prop.t, l, u, self.alpha, batch.lo, batch.hi,
                       infeasible, cons, passes, self.m, self.v, 1, 0.0, ws=prop.ws, pid=batch.pid)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(self.graph, stream=side):
                for s in range(1, steps + 1):
                    api.alpha_step_into(prop.net, prop.root, prop.C, prop.t, l, u, self.alpha,
                                        batch.lo, batch.hi, infeasible, cons, passes, self.m,
                                        self.v, s, lr * decay ** (s - 1), self.lbs[s - 1], prop.ws,
                                        pid=batch.pid, alpha_init=alpha0 if s == 1 else -1.0,
                                        best=self.best)
        torch.cuda.current_stream().wait_stream(side)

    def run(self):
        self.graph.replay()
        return self.best


class StepGraph:
    """One whole step -- reset the boxes to ``lo0``/``hi0``, the plain pass
    (clipping, plane re-concretization, bound with complete clipping) and
    ``steps`` slope iterations -- captured once into a HIP graph and replayed.
    The calls only launch kernels into buffers allocated by an eager warm-up
    run (workspaces, outputs, slope state), so the graph holds the step's
    whole launch sequence.  ``run()`` returns (out, best): the plain pass's
    dict (infeasible, l, u, lb) and the best bound over the iterations; both
    are buffers the graph rewrites on every replay."""

    def __init__(self, prop, batch, lo0, hi0, steps=20, lr=0.1, decay=1.0, cfg=PassConfig()):
        self.prop, self.batch, self.lo0, self.hi0 = prop, batch, lo0, hi0
        B, M, nh = batch.lo.shape[0], prop.M, prop.net.n_hidden
        self.out = {}
        self.alpha = torch.full((B, M, nh), cfg.alpha, device="cuda")
        self.m = torch.zeros_like(self.alpha)
        self.v = torch.zeros_like(self.alpha)
        self.best = torch.full((B, M), -float("inf"), device="cuda")
        self.lbs = [torch.empty(B, M, device="cuda") for _ in range(steps)]

        def body():
            batch.lo.copy_(lo0)
            batch.hi.copy_(hi0)
            out = plain_pass(prop, batch, cfg, out=self.out)
            cons = batch.cons() if cfg.complete_final else None
            for s in range(1, steps + 1):
                api.alpha_step_into(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"],
                                    self.alpha, batch.lo, batch.hi, out["infeasible"], cons,
                                    cfg.passes, self.m, self.v, s, lr * decay ** (s - 1),
                                    self.lbs[s - 1], prop.ws, pid=batch.pid,
                                    alpha_init=cfg.alpha if s == 1 else -1.0, best=self.best)

        # eager warm-up: sizes every workspace and output buffer
        out = plain_pass(prop, batch, cfg, out=self.out)
        api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], self.alpha,
                       batch.lo, batch.hi, out["infeasible"],
                       batch.cons() if cfg.complete_final else None, cfg.passes, self.m, self.v, 1,
                       0.0, ws=prop.ws, pid=batch.pid)
        body()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(self.graph, stream=side):
                body()
        torch.cuda.current_stream().wait_stream(side)

    def run(self):
        self.graph.replay()
        return self.out, self.best


def chunked_verify(prop, batch, chunk, steps=10, lr=0.1, cfg=PassConfig(), state=None):
    """The plain pass and ``steps`` slope iterations over a batch too large
    for one call (the per-row matrices of a wide network), in consecutive
    chunks of at most ``chunk`` subdomains (0 or None: the most one call
    takes, ``Net.max_batch``).  Subdomains are independent, so every result
    equals that of one call over the whole batch.  Boxes are
    clipped in place.  Returns dict(infeasible [B], lb [B, M] plain bound,
    best [B, M] best bound over the slope iterations (the plain bound when
    steps = 0)).  ``state`` keeps the per-chunk buffers between calls."""
    B, M = batch.lo.shape[0], prop.M
    if not chunk:
        chunk = prop.net.max_batch(M, prop.P)
    state = state if state is not None else {}
    res = state.get("res")
    if res is None or res["lb"].shape[0] != B:
        res = dict(infeasible=torch.empty(B, dtype=torch.uint8, device="cuda"),
                   lb=torch.empty(B, M, device="cuda"), best=torch.empty(B, M, device="cuda"))
        state["res"] = res
    for s0 in range(0, B, chunk):
        s1 = min(B, s0 + chunk)
        sp = batch.splits
        cons = None
        if sp is not None:
            cons = api.Constraints.splits(sp.neuron[s0:s1], sp.sign[s0:s1],
                                          None if sp.count is None else sp.count[s0:s1])
        sub = Batch(batch.lo[s0:s1], batch.hi[s0:s1], cons,
                    pid=None if batch.pid is None else batch.pid[s0:s1])
        key = s1 - s0
        bufs = state.setdefault(("out", key), {})
        out = plain_pass(prop, sub, cfg, out=bufs)
        res["infeasible"][s0:s1] = out["infeasible"]
        res["lb"][s0:s1] = out["lb"]
        if steps > 0:
            ast = state.setdefault(("alpha", key), {})
            best, _ = alpha_opt(prop, sub, out["l"], out["u"], out["infeasible"], steps=steps,
                                lr=lr, alpha0=cfg.alpha, complete=cfg.complete_final,
                                passes=cfg.passes, state=ast)
            res["best"][s0:s1] = best
        else:
            res["best"][s0:s1] = out["lb"]
    return res
