"""Python binding of libclipverify: argument marshalling only.

Tensors are torch CUDA (HIP) tensors; every call enqueues on the current
torch stream.  The names follow the C ABI (cv_clip_domains ->
``clip_domains`` ...).  All arithmetic happens in the HIP library.
"""
import ctypes as C

import numpy as np
import torch

from . import _native as N


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    """Device pointer of a contiguous tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _f32(t, dev=None):
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32))
    t = t.to(device=dev or "cuda", dtype=torch.float32)
    return t.contiguous()


class Net:
    """A ReLU network (ReLU after every layer but the last).  ``layers``: list
    of (W [out, in], b [out]) float32 arrays (linear layers), or of objects
    with ``kind`` ("linear" | "conv"), ``W``, ``b`` and, for conv, ``stride``,
    ``pad``, ``in_shape`` and ``out_shape`` ((C, H, W); W [oc, ic, k, k])."""

    def __init__(self, layers):
        keep = []
        descs = (N.LayerDesc * len(layers))()
        sizes = []
        for i, ly in enumerate(layers):
            if isinstance(ly, tuple):
                kind, W, b = "linear", ly[0], ly[1]
            else:
                kind, W, b = ly.kind, ly.W, ly.b
            W = np.ascontiguousarray(W, dtype=np.float32)
            b = np.ascontiguousarray(b, dtype=np.float32)
            keep += [W, b]
            d = descs[i]
            if kind == "linear":
                d.kind = N.CV_LINEAR
                d.in_features, d.out_features = W.shape[1], W.shape[0]
            else:
                d.kind = N.CV_CONV2D
                (d.in_c, d.in_h, d.in_w), (d.out_c, d.out_h, d.out_w) = ly.in_shape, ly.out_shape
                d.kernel, d.stride, d.pad = W.shape[2], ly.stride, ly.pad
                d.in_features = int(np.prod(ly.in_shape))
                d.out_features = int(np.prod(ly.out_shape))
            d.W = W.ctypes.data
            d.b = b.ctypes.data
            sizes.append(d.out_features)
        h = C.c_void_p()
        N.call("cv_net_create", descs, len(layers), C.byref(h))
        self.handle = h
        del keep
        a, o, nh, nl = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        N.call("cv_net_info", h, C.byref(a), C.byref(o), C.byref(nh), C.byref(nl))
        self.n_in, self.n_out, self.n_hidden, self.n_layers = a.value, o.value, nh.value, nl.value
        self.hidden_sizes = sizes[:-1]

    @classmethod
    def from_network(cls, net):
        """From an object with ``.layers`` (see the class docstring)."""
        return cls(list(net.layers))

    def max_batch(self, M, P=1):
        """Largest number of subdomains with M objective rows that one
        bound_propagate / alpha_step call takes for this network (the
        library's own size check, asked by bisection; host only)."""
        need = C.c_size_t()
        ok = lambda B: N.lib().cv_alpha_step_workspace(self.handle, P, B, M, C.byref(need)) == 0
        lo, hi = 1, 1 << 30
        if not ok(lo):
            return 0
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if ok(mid):
                lo = mid
            else:
                hi = mid - 1
        return lo

    def alpha_step_workspace(self, B, M, P=1):
        """Bytes of device workspace one alpha_step call over B subdomains
        with M objective rows asks for (host only)."""
        need = C.c_size_t()
        N.call("cv_alpha_step_workspace", self.handle, P, B, M, C.byref(need))
        return int(need.value)

    TUNE_KINDS = {"relax": N.CV_TUNE_RELAX, "final": N.CV_TUNE_FINAL,
                  "adjoint": N.CV_TUNE_ADJOINT}

    def autotune(self, B, M):
        """Time every kernel variant of every layer on B x M synthetic rows and
        keep the fastest (cv_net_autotune); results do not depend on it."""
        N.call("cv_net_autotune", self.handle, int(B), int(M), _stream())
        return self.tuning()

    def tuning(self):
        """{(kind, layer): (variant, count)} for every tunable layer."""
        out = {}
        v, c = C.c_int(), C.c_int()
        for name, kind in self.TUNE_KINDS.items():
            for layer in range(1, self.n_layers + 1):
                if N.lib().cv_net_tuning(self.handle, kind, layer, C.byref(v), C.byref(c)) == 0:
                    out[(name, layer)] = (v.value, c.value)
        return out

    def set_tuning(self, kind, layer, variant):
        N.call("cv_net_set_tuning", self.handle, self.TUNE_KINDS[kind], int(layer), int(variant))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and N is not None and N._lib is not None:
            N._lib.cv_net_destroy(h)
            self.handle = None


class Root:
    """Root bounds and cached planes of a property (root box lo0, hi0)."""

    P = 1

    PLANES = {"auto": 0, "all": 1, "unstable": 2}

    def __init__(self, net, lo0, hi0, alpha0=0.5, planes="auto"):
        """planes: which cached planes stay on the device -- "all", "unstable"
        (root-unstable neurons only; splits of other neurons are then
        ignored) or "auto" (all unless they pass 2^28 coefficients a side)."""
        self.net = net
        self.lo0, self.hi0 = _f32(lo0), _f32(hi0)
        h = C.c_void_p()
        N.call("cv_root_create_ex", net.handle, _p(self.lo0), _p(self.hi0), float(alpha0),
               self.PLANES[planes], _stream(), C.byref(h))
        self.handle = h
        cnt = C.c_int()
        N.call("cv_root_unstable_count", h, C.byref(cnt))
        self.n_unstable = cnt.value

    def bounds(self):
        l0 = torch.empty(self.net.n_hidden, device="cuda")
        u0 = torch.empty_like(l0)
        N.call("cv_root_bounds", self.handle, _p(l0), _p(u0), _stream())
        return l0, u0

    def planes(self):
        n, d = self.net.n_hidden, self.net.n_in
        A_lo = torch.empty(n, d, device="cuda")
        A_hi = torch.empty_like(A_lo)
        c_lo = torch.empty(n, device="cuda")
        c_hi = torch.empty_like(c_lo)
        N.call("cv_root_planes", self.handle, _p(A_lo), _p(c_lo), _p(A_hi), _p(c_hi), _stream())
        return A_lo, c_lo, A_hi, c_hi

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and N is not None and N._lib is not None:
            N._lib.cv_root_destroy(h)
            self.handle = None


class RootSet:
    """Several properties over one network, bounded together
    (cv_rootset_create): calls taking a root accept a RootSet with ``pid``
    (int32 [B], the property of each subdomain); objectives are then
    per property, C [P, M, n_out] and t [P, M]."""

    def __init__(self, roots):
        roots = list(roots)
        if not roots:
            raise ValueError("RootSet needs at least one root")
        self.roots = roots          # the set borrows their device state
        self.net = roots[0].net
        self.P = len(roots)
        arr = (C.c_void_p * self.P)(*[r.handle.value for r in roots])
        h = C.c_void_p()
        N.call("cv_rootset_create", arr, self.P, C.byref(h))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and N is not None and N._lib is not None:
            N._lib.cv_root_destroy(h)
            self.handle = None


def _rh(root):
    return root.handle if root is not None else None


def _pid(pid):
    if pid is None:
        return None
    if pid.dtype != torch.int32 or not pid.is_cuda or not pid.is_contiguous():
        raise ValueError("pid must be a contiguous int32 CUDA tensor")
    return _p(pid)


class Constraints:
    """Per-subdomain constraints: ``splits(neuron, sign, count)`` (activation
    splits resolved with a Root's planes) or ``dense(G, h, count)``."""

    def __init__(self, kmax, count=None, neuron=None, sign=None, G=None, h=None, order=None):
        self.kmax = int(kmax)
        self.count, self.neuron, self.sign, self.G, self.h = count, neuron, sign, G, h
        self.order = order
        self.struct = N.Constraints(self.kmax, _p(count), _p(neuron), _p(sign), _p(G), _p(h),
                                    _p(order))

    def with_order(self, order):
        """The same constraints taken in ``order`` ([B, kmax] int32, position
        -> slot; None: slot order)."""
        return Constraints(self.kmax, self.count, self.neuron, self.sign, self.G, self.h, order)

    @classmethod
    def splits(cls, neuron, sign, count=None):
        neuron = torch.as_tensor(neuron).to("cuda", torch.int32).contiguous()
        sign = torch.as_tensor(sign).to("cuda", torch.int8).contiguous()
        if count is not None:
            count = torch.as_tensor(count).to("cuda", torch.int32).contiguous()
        return cls(neuron.shape[1], count, neuron, sign)

    @classmethod
    def dense(cls, G, h, count=None):
        G, h = _f32(G), _f32(h)
        if count is not None:
            count = torch.as_tensor(count).to("cuda", torch.int32).contiguous()
        return cls(G.shape[1], count, None, None, G, h)

    def ref(self):
        return C.byref(self.struct)


def _cref(cons):
    return None if cons is None else cons.ref()


def constraint_order(root, lo, hi, cons, out=None, pid=None):
    """Constraint importance order of each subdomain over boxes lo/hi [B, n]
    (cv_constraint_order): returns int32 [B, kmax], position -> slot."""
    B, n = lo.shape
    order = out if out is not None else torch.empty(B, cons.kmax, dtype=torch.int32,
                                                    device="cuda")
    N.call("cv_constraint_order", _rh(root), _pid(pid), B, n, _cref(cons),
           _p(lo), _p(hi), _p(order), _stream())
    return order


def intermediate_bounds(net, root, lo, hi, l, u, infeasible=None, ws=None):
    """CROWN bounds of layers 2.. over each box, intersected with l, u in
    place (cv_intermediate_bounds)."""
    B = lo.shape[0]
    need = C.c_size_t()
    N.call("cv_intermediate_bounds_workspace", net.handle, B, C.byref(need))
    buf = (ws or Workspace()).get(need.value)
    N.call("cv_intermediate_bounds", net.handle, root.handle, B, _p(lo), _p(hi), _p(l), _p(u),
           _p(infeasible), _p(buf), need.value, _stream())
    return l, u


def branch_relu(root, l, u, weight, splits, lo, hi, kmax_out, pid=None):
    """ReLU branching (cv_branch_relu): returns (chosen [B], child splits
    (Constraints, 2B rows), lo2, hi2 [2B, n_in]); children 2b, 2b+1 belong
    to parent b's property."""
    B, n0 = lo.shape
    dev = "cuda"
    chosen = torch.empty(B, dtype=torch.int32, device=dev)
    neuron2 = torch.empty(2 * B, kmax_out, dtype=torch.int32, device=dev)
    sign2 = torch.empty(2 * B, kmax_out, dtype=torch.int8, device=dev)
    count2 = torch.empty(2 * B, dtype=torch.int32, device=dev)
    lo2 = torch.empty(2 * B, n0, device=dev)
    hi2 = torch.empty(2 * B, n0, device=dev)
    N.call("cv_branch_relu", root.handle, _pid(pid), B, _p(l), _p(u), _p(weight), _cref(splits),
           _p(lo),
           _p(hi), int(kmax_out), _p(chosen), _p(neuron2), _p(sign2), _p(count2), _p(lo2),
           _p(hi2), _stream())
    return chosen, Constraints(kmax_out, count2, neuron2, sign2), lo2, hi2


def branch_input(lo, hi, A):
    """Input branching (cv_branch_input): A [B, M, n]; returns (dim [B],
    lo2, hi2 [2B, n])."""
    B, n = lo.shape
    M = A.shape[1]
    dim = torch.empty(B, dtype=torch.int32, device="cuda")
    lo2 = torch.empty(2 * B, n, device="cuda")
    hi2 = torch.empty(2 * B, n, device="cuda")
    N.call("cv_branch_input", B, M, n, _p(lo), _p(hi), _p(A), _p(dim), _p(lo2), _p(hi2), _stream())
    return dim, lo2, hi2


class Workspace:
    """Grow-only device scratch buffer handed to the library."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        return self.buf


def clip_domains(root, lo, hi, cons, mode="parallel", infeasible=None, pid=None):
    """Relaxed clipping of boxes lo/hi [B, n] in place; returns the
    infeasible flags [B] (uint8)."""
    B, n = lo.shape
    if infeasible is None:
        infeasible = torch.empty(B, dtype=torch.uint8, device="cuda")
    m = N.CV_CLIP_SEQUENTIAL if mode == "sequential" else N.CV_CLIP_PARALLEL
    N.call("cv_clip_domains", _rh(root), _pid(pid), B, n, _cref(cons),
           _p(lo), _p(hi), _p(infeasible), m, _stream())
    return infeasible


def concretize_planes(root, lo, hi, splits=None, complete=False, passes=1, infeasible=None,
                      l=None, u=None, ws=None, topk=-1, weight=None, select=None, pid=None):
    """Bounds [B, n_hidden] of every hidden neuron over each box from the
    cached planes, then (complete) complete clipping of the unstable ones --
    all, or the top-k per layer by BaBSR score with ``weight``; returns
    (l, u, infeasible).  ``select`` (uint8 [B, n_hidden]) receives the mask."""
    B = lo.shape[0]
    nh = root.net.n_hidden
    l = torch.empty(B, nh, device="cuda") if l is None else l
    u = torch.empty(B, nh, device="cuda") if u is None else u
    if infeasible is None:
        infeasible = torch.zeros(B, dtype=torch.uint8, device="cuda")
    need = C.c_size_t()
    N.call("cv_concretize_planes_workspace", root.handle, B, int(bool(complete)), C.byref(need))
    buf = None
    if need.value:
        buf = (ws or Workspace()).get(need.value)
    N.call("cv_concretize_planes", root.handle, _pid(pid), B, _p(lo), _p(hi), _cref(splits),
           int(bool(complete)), int(passes), int(topk), _p(weight), _p(l), _p(u), _p(infeasible),
           _p(select), _p(buf), need.value, _stream())
    return l, u, infeasible


def concretize_planes_static(root, lo, hi, splits=None, complete=False, passes=1, infeasible=None,
                             l=None, u=None, topk=-1, weight=None, select=None, pid=None):
    """concretize_planes through the allocation-free entry point (scratch in
    the library's static per-device array; no workspace)."""
    B = lo.shape[0]
    nh = root.net.n_hidden
    l = torch.empty(B, nh, device="cuda") if l is None else l
    u = torch.empty(B, nh, device="cuda") if u is None else u
    if infeasible is None:
        infeasible = torch.zeros(B, dtype=torch.uint8, device="cuda")
    N.call("cv_concretize_planes_static", root.handle, _pid(pid), B, _p(lo), _p(hi),
           _cref(splits), int(bool(complete)), int(passes), int(topk), _p(weight), _p(l), _p(u),
           _p(infeasible), _p(select), _stream())
    return l, u, infeasible


def babsr_weights(net, root, C_, t, ws=None):
    """Weights of the neuron-selection score (cv_babsr_weights): [n_hidden]
    for a Root and C [M, n_out]; [P, n_hidden] for per-property C [P, M, n_out]."""
    M = C_.shape[-2]
    need = C.c_size_t()
    N.call("cv_babsr_weights_workspace", net.handle, M, C.byref(need))
    buf = (ws or Workspace()).get(need.value)
    w = torch.empty(*C_.shape[:-2], net.n_hidden, device="cuda")
    N.call("cv_babsr_weights", net.handle, root.handle, M, _p(C_), _p(t), _p(w), _p(buf),
           need.value, _stream())
    return w


def concretize(A, c, lo, hi, cons=None, passes=1, root=None, shared=False, want_ub=False,
               want_beta=False, infeasible=None, pid=None):
    """min (and optionally max) of A x + c over each box, with complete
    clipping against ``cons`` when given.  A: [B, P, n] or [P, n] (shared)."""
    B, n = lo.shape
    P = A.shape[-2]
    lb = torch.empty(B, P, device="cuda")
    ub = torch.empty(B, P, device="cuda") if want_ub else None
    beta = torch.empty(B, P, max(cons.kmax, 1), device="cuda") if (want_beta and cons) else None
    N.call("cv_concretize", _rh(root), _pid(pid), B, P, n, _p(A),
           int(bool(shared)), _p(c), _p(lo), _p(hi), _cref(cons), int(passes), _p(lb), _p(ub),
           _p(beta), _p(infeasible), _stream())
    return lb, ub, beta


def bound_propagate(net, root, C_, t, l, u, lo, hi, alpha=None, alpha_default=0.5,
                    infeasible=None, cons=None, passes=1, want_plane=False, ws=None, pid=None):
    """CROWN bound of the objective rows C y + t for every subdomain (with
    complete clipping when ``cons`` is given).  Returns lb [B, M] and, with
    ``want_plane``, the input plane (A [B, M, n_in], c [B, M])."""
    B = lo.shape[0]
    M = C_.shape[-2]
    lb = torch.empty(B, M, device="cuda")
    A = torch.empty(B, M, net.n_in, device="cuda") if want_plane else None
    c = torch.empty(B, M, device="cuda") if want_plane else None
    need = C.c_size_t()
    N.call("cv_bound_propagate_workspace", net.handle, root.P, B, M, C.byref(need))
    buf = (ws or Workspace()).get(need.value)
    N.call("cv_bound_propagate", net.handle, B, M, _p(C_), _p(t), _p(l), _p(u), _p(alpha),
           float(alpha_default), _p(lo), _p(hi), _p(infeasible), root.handle, _pid(pid),
           _cref(cons),
           int(passes), _p(lb), _p(A), _p(c), _p(buf), need.value, _stream())
    return (lb, A, c) if want_plane else lb


def alpha_step_into(net, root, C_, t, l, u, alpha, lo, hi, infeasible, cons, passes, adam_m,
                    adam_v, step, lr, lb, ws, beta1=0.9, beta2=0.999, eps=1e-8, pid=None,
                    alpha_init=-1.0, best=None):
    """alpha_step writing the bound into a given buffer lb [B, M] (and the
    running best into ``best``) with a workspace that is already large
    enough (no allocation: usable under stream capture)."""
    B = lo.shape[0]
    M = C_.shape[-2]
    need = C.c_size_t()
    N.call("cv_alpha_step_workspace", net.handle, root.P, B, M, C.byref(need))
    buf = ws.buf
    if buf is None or buf.numel() < need.value:
        raise RuntimeError("workspace too small for alpha_step_into; size it before capture")
    N.call("cv_alpha_step", net.handle, B, M, _p(C_), _p(t), _p(l), _p(u), _p(alpha),
           float(alpha_init), _p(lo), _p(hi), _p(infeasible), root.handle, _pid(pid), _cref(cons),
           int(passes), _p(adam_m), _p(adam_v), int(step), float(lr), float(beta1), float(beta2),
           float(eps), _p(lb), _p(best), None, _p(buf), need.value, _stream())
    return lb


def alpha_step(net, root, C_, t, l, u, alpha, lo, hi, infeasible=None, cons=None, passes=1,
               adam_m=None, adam_v=None, step=1, lr=0.0, beta1=0.9, beta2=0.999, eps=1e-8,
               want_grad=False, ws=None, pid=None, alpha_init=-1.0, best=None):
    """Bound at the current alpha [B, M, n_hidden] and its gradient, then
    (lr > 0) one Adam ascent step on alpha in place; ``best`` [B, M] (if
    given) becomes max(best, bound), the bound itself at step 1; at step 1
    an ``alpha_init`` in [0, 1] replaces alpha.  Returns (lb, grad)."""
    B = lo.shape[0]
    M = C_.shape[-2]
    lb = torch.empty(B, M, device="cuda")
    grad = torch.empty_like(alpha) if want_grad else None
    need = C.c_size_t()
    N.call("cv_alpha_step_workspace", net.handle, root.P, B, M, C.byref(need))
    buf = (ws or Workspace()).get(need.value)
    N.call("cv_alpha_step", net.handle, B, M, _p(C_), _p(t), _p(l), _p(u), _p(alpha),
           float(alpha_init), _p(lo), _p(hi), _p(infeasible), root.handle, _pid(pid), _cref(cons),
           int(passes), _p(adam_m), _p(adam_v), int(step), float(lr), float(beta1), float(beta2),
           float(eps), _p(lb), _p(best), _p(grad), _p(buf), need.value, _stream())
    return lb, grad
