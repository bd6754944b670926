"""CROWN backward bound propagation and the root pass that caches planes.

Network: z^(i) = W^(i) h^(i-1) + b^(i), h^(i) = ReLU(z^(i)) for the hidden
layers i = 1..L-1, h^(0) = x, output y = z^(L).  Objective rows C y + t
(specification matrix and threshold, appendix on Boolean properties).

ReLU relaxation (Lemma A.3, with the Planet upper line of the LP-relaxation
appendix): for neuron j with pre-activation bounds [l, u]
* l >= 0 (active):   slope 1, intercept 0
* u <= 0 (inactive): slope 0, intercept 0
* otherwise (unstable), chosen by the sign of the coefficient Psi_j that
  multiplies the neuron's output in the row being bounded:
    Psi_j >= 0: lower line  alpha_j * z   (alpha_j in [0, 1])
    Psi_j <  0: upper line  u/(u-l) * (z - l)
Plane recursion (appendix A.3): starting from Omega = C, c = t, each linear
layer adds Omega b to c and maps Omega -> Psi = Omega W; each ReLU maps
Psi -> Omega = Psi * slope and adds Psi * intercept to c.  At the input the
plane is A = Psi (= Omega W^(1)), so C y + t >= A x + c on the domain.

Readings taken:
* Lemma A.3 selects the relaxation by the sign of "W_j"; the sign of the
  propagated coefficient Psi_j of each objective row is used (as in the 2-D
  toy example, where the final-layer weights decide).  The lemma mixes
  l > 0 and l >= 0; l >= 0 is active, u <= 0 inactive, l < 0 < u unstable.
* The index garble in the Omega recursion is read as the standard top-down
  recursion above.
* The root pass (caching planes at initialisation) uses a fixed alpha for
  every unstable neuron, 0.5 by default.
* Conv layers are turned into their dense matrices with explicit loops.
"""
from dataclasses import dataclass
from typing import List

import numpy as np

from .box import f64, concretize_min, concretize_max


def conv_matrix(W, stride, pad, in_shape, out_shape):
    """Dense matrix [oc*ho*wo, ic*h*w] of a 2-D convolution (cross-
    correlation, zero padding), built with explicit loops over outputs and
    kernel taps; flattening order is (channel, row, column)."""
    W = f64(W)
    oc, ic, kh, kw = W.shape
    c, h, w = in_shape
    _, ho, wo = out_shape
    M = np.zeros((oc * ho * wo, c * h * w))
    for o in range(oc):
        for y in range(ho):
            for x in range(wo):
                r = (o * ho + y) * wo + x
                for i in range(ic):
                    for dy in range(kh):
                        yy = y * stride - pad + dy
                        if yy < 0 or yy >= h:
                            continue
                        for dx in range(kw):
                            xx = x * stride - pad + dx
                            if xx < 0 or xx >= w:
                                continue
                            M[r, (i * h + yy) * w + xx] += W[o, i, dy, dx]
    return M


def conv_bias(b, out_shape):
    oc, ho, wo = out_shape
    return np.repeat(f64(b), ho * wo)


def dense_layers(net):
    """[(W [out, in] float64, b [out] float64)] for every layer of ``net``
    (an object with ``.layers``, each having kind, W, b and for convs
    stride, pad, in_shape, out_shape)."""
    out = []
    for ly in net.layers:
        if ly.kind == "linear":
            out.append((f64(ly.W), f64(ly.b)))
        elif ly.kind == "conv":
            out.append((conv_matrix(ly.W, ly.stride, ly.pad, ly.in_shape, ly.out_shape),
                        conv_bias(ly.b, ly.out_shape)))
        else:
            raise ValueError(ly.kind)
    return out


def relu_relaxation(l, u, Psi, alpha):
    """Slopes and intercepts of the relaxation of ReLU neurons (Lemma A.3).
    l, u: [B, 1, n] (broadcast over rows), Psi: [B, M, n], alpha: scalar or
    [B, M, n].  Returns (slope, intercept, lower_mask) where lower_mask marks
    unstable entries that use the alpha line (the entries alpha acts on)."""
    active = l >= 0.0
    inactive = (u <= 0.0) & ~active
    unstable = ~active & ~inactive
    with np.errstate(divide="ignore", invalid="ignore"):
        s_up = u / (u - l)
        t_up = -u * l / (u - l)
    pos = Psi >= 0.0
    alpha = f64(alpha)
    slope = np.where(active, 1.0,
                     np.where(inactive, 0.0, np.where(pos, alpha, s_up)))
    icpt = np.where(unstable & ~pos, t_up, 0.0)
    lower_mask = unstable & pos
    return slope, icpt, lower_mask


def backward(layers, C, t, l_list, u_list, alpha=0.5, trace=False):
    """CROWN backward pass for a batch of subdomains.

    layers: list of (W, b) dense float64 pairs; C: [M, n_L]; t: [M];
    l_list/u_list: per hidden layer, [B, n_i]; alpha: a scalar or a list with
    one [B, M, n_i] array per hidden layer.
    Returns (A [B, M, n_0], c [B, M]); with ``trace`` also the list of Psi
    entering each hidden ReLU (top-down order reversed to layer order)."""
    L = len(layers)
    B = l_list[0].shape[0] if len(l_list) else 1
    C, t = f64(C), f64(t)
    M = C.shape[0]
    Omega = np.broadcast_to(C, (B, M, C.shape[1])).copy()
    c = np.broadcast_to(t, (B, M)).copy()
    psis = [None] * (L - 1)
    for i in range(L - 1, -1, -1):
        W, b = layers[i]
        c = c + Omega @ b
        Psi = Omega @ W
        if i == 0:
            A = Psi
            break
        l = f64(l_list[i - 1])[:, None, :]
        u = f64(u_list[i - 1])[:, None, :]
        a_i = alpha if np.isscalar(alpha) else alpha[i - 1]
        slope, icpt, _ = relu_relaxation(l, u, Psi, a_i)
        psis[i - 1] = Psi
        c = c + (Psi * icpt).sum(-1)
        Omega = Psi * slope
    if trace:
        return A, c, psis
    return A, c


@dataclass
class RootState:
    """Root bounds and cached planes of every hidden neuron (layer order).

    lower[i] = (A_lo [n_i, n_0], c_lo [n_i]) with z_i >= A_lo x + c_lo;
    upper[i] = (A_hi, c_hi) with z_i <= A_hi x + c_hi, for x in the root box;
    l[i], u[i]: [n_i] root pre-activation bounds."""

    lower: List[tuple]
    upper: List[tuple]
    l: List[np.ndarray]
    u: List[np.ndarray]

    def stacked(self):
        """All hidden neurons stacked in global order:
        (A_lo [N, n0], c_lo [N], A_hi [N, n0], c_hi [N], l [N], u [N])."""
        return (np.concatenate([p[0] for p in self.lower]),
                np.concatenate([p[1] for p in self.lower]),
                np.concatenate([p[0] for p in self.upper]),
                np.concatenate([p[1] for p in self.upper]),
                np.concatenate(self.l), np.concatenate(self.u))


def root_pass(layers, lo0, hi0, alpha0=0.5):
    """Intermediate bounds and planes at the root box (the initial bounding
    pass whose planes are cached, activation-BaB section and Alg. 5's
    Get_Constraints).  Layer 1's planes are W^(1), b^(1) exactly; layer i's
    lower plane is CROWN with objective I on z^(i) over the network cut after
    layer i, its upper plane the negation of CROWN with objective -I."""
    lo0, hi0 = f64(lo0)[None], f64(hi0)[None]
    lower, upper, ls, us = [], [], [], []
    W1, b1 = layers[0]
    lower.append((W1.copy(), b1.copy()))
    upper.append((W1.copy(), b1.copy()))
    ls.append(concretize_min(W1[None], b1[None], lo0, hi0)[0])
    us.append(concretize_max(W1[None], b1[None], lo0, hi0)[0])
    for i in range(2, len(layers)):
        n_i = layers[i - 1][0].shape[0]
        sub = layers[:i]
        lb_l = [x[None] for x in ls]
        lb_u = [x[None] for x in us]
        I = np.eye(n_i)
        A_lo, c_lo = backward(sub, I, np.zeros(n_i), lb_l, lb_u, alpha0)
        A_n, c_n = backward(sub, -I, np.zeros(n_i), lb_l, lb_u, alpha0)
        A_lo, c_lo, A_hi, c_hi = A_lo[0], c_lo[0], -A_n[0], -c_n[0]
        lower.append((A_lo, c_lo))
        upper.append((A_hi, c_hi))
        ls.append(concretize_min(A_lo[None], c_lo[None], lo0, hi0)[0])
        us.append(concretize_max(A_hi[None], c_hi[None], lo0, hi0)[0])
    return RootState(lower, upper, ls, us)
