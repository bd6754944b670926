"""Seeded synthetic inputs for the clip-and-verify hot path.

This module is shared by the GPU path, the CPU oracle, the tests and the
benchmark.  It only draws random numbers and arranges them into arrays: it
holds none of the bounding or clipping arithmetic.  Every array it returns is
float32 (or an integer type); a consumer that computes in float64 widens the
float32 values exactly.

Workload shapes follow the paper's settings where it states them: He-normal
ReLU networks, l-infinity input boxes (CIFAR radius 2/255 from the experiments
section), activation split constraints drawn as (layer, neuron, sign) triples,
and margin specifications ``e_y - e_j`` with a zero threshold (appendix on
specification matrices).  The paper's benchmark models and datasets are not
available; these synthetic inputs stand in for them.

Seeds: weights 0, box centres 1, splits 2, soundness samples 3, property
sizes 4 (each generator takes its seed explicitly).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

SEED_WEIGHTS = 0
SEED_CENTRES = 1
SEED_SPLITS = 2
SEED_SAMPLES = 3
SEED_SIZES = 4


@dataclass
class Layer:
    """One affine layer.  ``kind`` is ``"linear"`` (W: [out, in]) or
    ``"conv"`` (W: [oc, ic, kh, kw] with stride/pad and the input shape)."""

    kind: str
    W: np.ndarray
    b: np.ndarray
    stride: int = 1
    pad: int = 0
    in_shape: tuple = ()   # (C, H, W) for conv
    out_shape: tuple = ()  # (C, H, W) for conv

    @property
    def n_in(self) -> int:
        if self.kind == "linear":
            return int(self.W.shape[1])
        return int(np.prod(self.in_shape))

    @property
    def n_out(self) -> int:
        if self.kind == "linear":
            return int(self.W.shape[0])
        return int(np.prod(self.out_shape))


@dataclass
class Network:
    """A feed-forward ReLU network: ReLU after every layer but the last."""

    layers: List[Layer]

    @property
    def n_in(self) -> int:
        return self.layers[0].n_in

    @property
    def n_out(self) -> int:
        return self.layers[-1].n_out

    @property
    def hidden_sizes(self) -> List[int]:
        return [ly.n_out for ly in self.layers[:-1]]

    @property
    def hidden_offsets(self) -> List[int]:
        """Global index of the first neuron of each hidden layer."""
        off, acc = [], 0
        for n in self.hidden_sizes:
            off.append(acc)
            acc += n
        return off

    @property
    def n_hidden(self) -> int:
        return int(sum(self.hidden_sizes))


def he_mlp(widths: Sequence[int], seed: int = SEED_WEIGHTS,
           bias: str = "zero") -> Network:
    """ReLU MLP with He-normal weights N(0, 2/fan_in), drawn in layer order,
    row-major [out, in].  ``bias`` is ``"zero"`` or ``"uniform"``
    (U[-0.1, 0.1], a correctness-only variant exercising the bias path)."""
    rng = np.random.default_rng(seed)
    layers = []
    for n_in, n_out in zip(widths[:-1], widths[1:]):
        W = rng.normal(0.0, np.sqrt(2.0 / n_in), size=(n_out, n_in))
        layers.append(Layer("linear", W.astype(np.float32), np.zeros(n_out, np.float32)))
    if bias == "uniform":
        for ly in layers:
            ly.b = rng.uniform(-0.1, 0.1, size=ly.b.shape).astype(np.float32)
    return Network(layers)


def he_cnn(in_shape, convs, fcs, seed: int = SEED_WEIGHTS,
           bias: str = "zero") -> Network:
    """CNN: ``convs`` is a list of (out_ch, k, stride, pad); ``fcs`` a list of
    output widths of the linear layers after flattening (C, H, W order)."""
    rng = np.random.default_rng(seed)
    layers = []
    c, h, w = in_shape
    for oc, k, s, p in convs:
        fan_in = c * k * k
        W = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(oc, c, k, k))
        ho = (h + 2 * p - k) // s + 1
        wo = (w + 2 * p - k) // s + 1
        layers.append(Layer("conv", W.astype(np.float32), np.zeros(oc, np.float32),
                            stride=s, pad=p, in_shape=(c, h, w), out_shape=(oc, ho, wo)))
        c, h, w = oc, ho, wo
    n = c * h * w
    for n_out in fcs:
        W = rng.normal(0.0, np.sqrt(2.0 / n), size=(n_out, n))
        layers.append(Layer("linear", W.astype(np.float32), np.zeros(n_out, np.float32)))
        n = n_out
    if bias == "uniform":
        for ly in layers:
            ly.b = rng.uniform(-0.1, 0.1, size=ly.b.shape).astype(np.float32)
    return Network(layers)


def box_around(centre: np.ndarray, eps: float, clip: Optional[tuple] = None):
    """Input box [centre - eps, centre + eps], optionally intersected with
    [clip[0], clip[1]]; returned as float32 (lo, hi)."""
    c = np.asarray(centre, np.float64)
    lo, hi = c - eps, c + eps
    if clip is not None:
        lo = np.maximum(lo, clip[0])
        hi = np.minimum(hi, clip[1])
    return lo.astype(np.float32), hi.astype(np.float32)


def centres(n: int, count: int, low: float, high: float, seed: int = SEED_CENTRES):
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=(count, n))


def forward(net: Network, x: np.ndarray) -> np.ndarray:
    """Plain float64 forward pass (used to pick labels and to draw soundness
    samples).  ``x``: [S, n_in] -> [S, n_out]."""
    h = np.asarray(x, np.float64)
    for i, ly in enumerate(net.layers):
        h = affine(ly, h)
        if i < len(net.layers) - 1:
            h = np.maximum(h, 0.0)
    return h


def affine(ly: Layer, h: np.ndarray) -> np.ndarray:
    """Apply one layer to a batch of flat inputs [S, n_in] in float64."""
    W = ly.W.astype(np.float64)
    b = ly.b.astype(np.float64)
    if ly.kind == "linear":
        return h @ W.T + b
    c, hh, ww = ly.in_shape
    oc, ho, wo = ly.out_shape
    k = W.shape[2]
    S = h.shape[0]
    x = h.reshape(S, c, hh, ww)
    xp = np.zeros((S, c, hh + 2 * ly.pad, ww + 2 * ly.pad))
    xp[:, :, ly.pad:ly.pad + hh, ly.pad:ly.pad + ww] = x
    out = np.zeros((S, oc, ho, wo))
    for di in range(k):
        for dj in range(k):
            patch = xp[:, :, di:di + ly.stride * ho:ly.stride, dj:dj + ly.stride * wo:ly.stride]
            out += np.einsum("sihw,oi->sohw", patch, W[:, :, di, dj])
    out += b[None, :, None, None]
    return out.reshape(S, -1)


def pre_activations(net: Network, x: np.ndarray) -> np.ndarray:
    """Concatenated hidden pre-activations z^(1..L-1) at points x: [S, n_hidden]."""
    h = np.asarray(x, np.float64)
    zs = []
    for i, ly in enumerate(net.layers[:-1]):
        z = affine(ly, h)
        zs.append(z)
        h = np.maximum(z, 0.0)
    return np.concatenate(zs, axis=1) if zs else np.zeros((x.shape[0], 0))


def margin_spec(n_out: int, label: int):
    """Specification rows e_y - e_j for j != y, threshold 0 (float32)."""
    rows = []
    for j in range(n_out):
        if j != label:
            r = np.zeros(n_out)
            r[label], r[j] = 1.0, -1.0
            rows.append(r)
    C = np.asarray(rows, np.float32)
    return C, np.zeros(C.shape[0], np.float32)


def identity_spec(n_out: int):
    return np.eye(n_out, dtype=np.float32), np.zeros(n_out, np.float32)


@dataclass
class Splits:
    """Per-subdomain activation split lists, padded to ``kmax``.

    ``neuron``: [B, kmax] int32 global hidden-neuron index (-1 = unused slot),
    ``sign``:   [B, kmax] int8, +1 for the branch z >= 0, -1 for z <= 0,
    ``count``:  [B] int32 number of used slots (used slots come first)."""

    neuron: np.ndarray
    sign: np.ndarray
    count: np.ndarray

    @property
    def B(self) -> int:
        return int(self.neuron.shape[0])

    @property
    def kmax(self) -> int:
        return int(self.neuron.shape[1])


def draw_splits(B: int, counts: np.ndarray, candidates: np.ndarray,
                seed: int = SEED_SPLITS, kmax: Optional[int] = None) -> Splits:
    """For each subdomain b, ``counts[b]`` distinct neurons drawn uniformly
    from ``candidates`` (global indices), each with sign +-1 (p = 1/2)."""
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts, np.int32)
    if kmax is None:
        kmax = int(counts.max()) if B else 0
    kmax = max(int(kmax), 1)
    neuron = np.full((B, kmax), -1, np.int32)
    sign = np.zeros((B, kmax), np.int8)
    cand = np.asarray(candidates, np.int64)
    for b in range(B):
        k = int(counts[b])
        if k == 0:
            continue
        sel = rng.choice(cand.size, size=k, replace=False)
        neuron[b, :k] = cand[sel]
        sign[b, :k] = np.where(rng.random(k) < 0.5, 1, -1)
    return Splits(neuron, sign, counts.copy())


def splits_from_points(net: Network, x: np.ndarray, counts: np.ndarray,
                       candidates: np.ndarray, seed: int = SEED_SPLITS,
                       kmax: Optional[int] = None) -> Splits:
    """Split lists whose signs agree with the activation pattern of point
    x[b]: so x[b] is a feasible point of subdomain b (soundness tests)."""
    sp = draw_splits(x.shape[0], counts, candidates, seed, kmax)
    z = pre_activations(net, x)
    for b in range(sp.B):
        k = int(sp.count[b])
        idx = sp.neuron[b, :k]
        sp.sign[b, :k] = np.where(z[b, idx] >= 0.0, 1, -1)
    return sp


# ---------------------------------------------------------------- configs

@dataclass
class Workload:
    """One synthetic property: network, root box, specification and a batch
    of subdomains (boxes + split lists)."""

    name: str
    net: Network
    lo0: np.ndarray
    hi0: np.ndarray
    C: np.ndarray
    t: np.ndarray
    B: int
    split_counts: np.ndarray
    alpha0: float = 0.5
    extra: dict = field(default_factory=dict)


def tiny_mlp(B: int = 1024, seed: int = SEED_WEIGHTS) -> Workload:
    """ReLU MLP 5-50x6-5 (zero biases), box = centre U[-1,1]^5 +- 0.05,
    k ~ U{1..8} splits over all hidden neurons, objective = the 5 outputs."""
    net = he_mlp([5] + [50] * 6 + [5], seed)
    c = centres(5, 1, -1.0, 1.0)[0]
    lo, hi = box_around(c, 0.05)
    C, t = identity_spec(5)
    counts = np.random.default_rng(SEED_SIZES).integers(1, 9, size=B).astype(np.int32)
    return Workload("mlp5-50x6-5", net, lo, hi, C, t, B, counts)


def mnist_mlp(B: int = 16384, widths=(784,) + (256,) * 6 + (10,),
              k: int = 4, seed: int = SEED_WEIGHTS, name="mlp784-256x6-10") -> Workload:
    """ReLU MLP 784-256x6-10, centre U[0,1]^784, eps 0.02 clipped to [0,1],
    ``k`` splits per subdomain, 9 margin objectives (label = argmax f(centre))."""
    net = he_mlp(list(widths), seed)
    c = centres(widths[0], 1, 0.0, 1.0)[0]
    lo, hi = box_around(c, 0.02, clip=(0.0, 1.0))
    label = int(np.argmax(forward(net, c[None, :].astype(np.float32))[0]))
    C, t = margin_spec(widths[-1], label)
    counts = np.full(B, k, np.int32)
    return Workload(name, net, lo, hi, C, t, B, counts, extra={"label": label})


def alpha_mlp(B: int = 8192, seed: int = SEED_WEIGHTS) -> Workload:
    """ReLU MLP 784-1024x4-10, 6 splits per subdomain (slope optimisation)."""
    return mnist_mlp(B, (784,) + (1024,) * 4 + (10,), 6, seed, "mlp784-1024x4-10")


def cifar_cnn(B: int = 4096, seed: int = SEED_WEIGHTS, depth=(1, 12)) -> Workload:
    """CNN 3x32x32 -> conv 16 (4x4, stride 2, pad 1) -> conv 32 (4x4, stride 2,
    pad 1) -> linear 100 -> linear 10, He-normal, zero biases; one property:
    image centre U[0,1]^3072, eps 2/255 clipped to [0, 1], 9 margin rows;
    split depth per subdomain ~ U{depth[0]..depth[1]}."""
    net = he_cnn((3, 32, 32), [(16, 4, 2, 1), (32, 4, 2, 1)], [100, 10], seed)
    c = centres(3072, 1, 0.0, 1.0)[0]
    lo, hi = box_around(c, 2.0 / 255.0, clip=(0.0, 1.0))
    label = int(np.argmax(forward(net, c[None, :].astype(np.float32))[0]))
    C, t = margin_spec(10, label)
    counts = np.random.default_rng(SEED_SIZES).integers(depth[0], depth[1] + 1, size=B)
    return Workload("cnn3x32x32-c16-c32-100-10", net, lo, hi, C, t, B, counts.astype(np.int32),
                    extra={"label": label})


def ragged_cnn(B: int = 64, seed: int = SEED_WEIGHTS, depth=(1, 6)) -> Workload:
    """CNN 5x9x7 -> conv 6 (3x3, stride 1, pad 1) -> conv 17 (4x4, stride 3,
    pad 2) -> linear 12 -> linear 4, He-normal weights, uniform biases: channel
    counts that fill no channel block, stride 3, non-square maps; box = centre
    U[-1,1]^315 +- 0.05, the 4 outputs as objectives."""
    net = he_cnn((5, 9, 7), [(6, 3, 1, 1), (17, 4, 3, 2)], [12, 4], seed, bias="uniform")
    c = centres(315, 1, -1.0, 1.0)[0]
    lo, hi = box_around(c, 0.05)
    C, t = identity_spec(4)
    counts = np.random.default_rng(SEED_SIZES).integers(depth[0], depth[1] + 1, size=B)
    return Workload("cnn5x9x7-c6-c17-12-4", net, lo, hi, C, t, B, counts.astype(np.int32))


def wide_cnn(B: int = 32, seed: int = SEED_WEIGHTS, depth=(1, 6)) -> Workload:
    """CNN 4x24x24 -> conv 16 (3x3, stride 1, pad 1) -> conv 8 (4x4, stride 2,
    pad 1) -> linear 10 -> linear 3, uniform biases: the first conv's output
    (9216 values a row) is too long to stage in LDS; box = centre U[0,1]^2304
    +- 0.01, the 3 outputs as objectives."""
    net = he_cnn((4, 24, 24), [(16, 3, 1, 1), (8, 4, 2, 1)], [10, 3], seed, bias="uniform")
    c = centres(2304, 1, 0.0, 1.0)[0]
    lo, hi = box_around(c, 0.01)
    C, t = identity_spec(3)
    counts = np.random.default_rng(SEED_SIZES).integers(depth[0], depth[1] + 1, size=B)
    return Workload("cnn4x24x24-c16-c8-10-3", net, lo, hi, C, t, B, counts.astype(np.int32))


def edge_cnn(B: int = 48, seed: int = SEED_WEIGHTS, depth=(1, 6)) -> Workload:
    """Convolution edge cases: 3x7x7 -> conv 4 (1x1, stride 2, pad 0: in the
    transposed convolution the odd positions take no tap at all) -> conv 5
    (2x2, stride 2, pad 0: non-overlapping taps) -> conv 3 (3x3, stride 1,
    pad 2: the output grows) -> linear 6 -> linear 3, uniform biases; box =
    centre U[-1,1]^147 +- 0.05, the 3 outputs as objectives."""
    net = he_cnn((3, 7, 7), [(4, 1, 2, 0), (5, 2, 2, 0), (3, 3, 1, 2)], [6, 3], seed,
                 bias="uniform")
    c = centres(147, 1, -1.0, 1.0)[0]
    lo, hi = box_around(c, 0.05)
    C, t = identity_spec(3)
    counts = np.random.default_rng(SEED_SIZES).integers(depth[0], depth[1] + 1, size=B)
    return Workload("cnn3x7x7-c4k1s2-c5k2s2-c3k3p2-6-3", net, lo, hi, C, t, B,
                    counts.astype(np.int32))


@dataclass
class WorkloadSet:
    """Several properties over one network (own box centre, label and
    subdomain count each).  ``counts[p]`` subdomains of property p, grouped by
    property in order; ``split_counts`` [sum(counts)] split depth of each;
    ``member(p)`` is property p alone as a Workload."""

    name: str
    net: Network
    lo0s: List[np.ndarray]
    hi0s: List[np.ndarray]
    Cs: List[np.ndarray]
    ts: List[np.ndarray]
    counts: np.ndarray
    split_counts: np.ndarray
    alpha0: float = 0.5

    @property
    def P(self) -> int:
        return len(self.lo0s)

    @property
    def B(self) -> int:
        return int(self.counts.sum())

    def pid(self) -> np.ndarray:
        return np.repeat(np.arange(self.P, dtype=np.int32), self.counts)

    def member(self, p: int) -> Workload:
        start = int(self.counts[:p].sum())
        sc = self.split_counts[start:start + int(self.counts[p])]
        return Workload(f"{self.name}[{p}]", self.net, self.lo0s[p], self.hi0s[p], self.Cs[p],
                        self.ts[p], int(self.counts[p]), sc, self.alpha0)


def property_set(net: Network, n_in: int, centre_range, eps: float, clip, counts,
                 depth, name: str, seed_offset: int = 0) -> WorkloadSet:
    """Properties of one network: centre p ~ U(centre_range)^n_in (seed 1,
    the p-th draw), box centre +- eps (clipped to ``clip``), label = argmax
    of the network at the centre, margin rows; split depth of every
    subdomain ~ U{depth[0]..depth[1]} (seed 4)."""
    counts = np.asarray(counts, np.int64)
    P = counts.size
    cs = centres(n_in, P + seed_offset, centre_range[0], centre_range[1])[seed_offset:]
    lo0s, hi0s, Cs, ts = [], [], [], []
    for p in range(P):
        lo, hi = box_around(cs[p], eps, clip=clip)
        label = int(np.argmax(forward(net, cs[p][None, :].astype(np.float32))[0]))
        C, t = margin_spec(net.n_out, label)
        lo0s.append(lo)
        hi0s.append(hi)
        Cs.append(C)
        ts.append(t)
    rng = np.random.default_rng(SEED_SIZES)
    sc = rng.integers(depth[0], depth[1] + 1, size=int(counts.sum())).astype(np.int32)
    return WorkloadSet(name, net, lo0s, hi0s, Cs, ts, counts, sc)


def geometric_counts(P: int, p: float, cap: int, seed: int = SEED_SIZES) -> np.ndarray:
    """Subdomain count per property ~ Geometric(p) clipped to [1, cap]."""
    rng = np.random.default_rng(seed + 100)
    return np.clip(rng.geometric(p, size=P), 1, cap).astype(np.int64)


def cifar_cnn_set(P: int = 64, seed: int = SEED_WEIGHTS, counts=None) -> WorkloadSet:
    """The CNN of ``cifar_cnn`` with P properties (own image centre U[0,1]^3072
    and label, eps 2/255 clipped to [0,1]); subdomains per property ~
    Geometric(0.002) clipped to [1, 4096] unless ``counts`` is given; split
    depth ~ U{1..12}."""
    net = he_cnn((3, 32, 32), [(16, 4, 2, 1), (32, 4, 2, 1)], [100, 10], seed)
    if counts is None:
        counts = geometric_counts(P, 0.002, 4096)
    return property_set(net, 3072, (0.0, 1.0), 2.0 / 255.0, (0.0, 1.0), counts, (1, 12),
                        f"cnn3x32x32-c16-c32-100-10 x {len(counts)} properties")


def zipf_counts(P: int, s: float, total: int) -> np.ndarray:
    """Subdomain counts of P properties proportional to r^-s over the ranks
    r = 1..P (property p has rank p + 1), rounded by largest remainder to sum
    to ``total``, with at least 1 each."""
    w = np.arange(1, P + 1, dtype=np.float64) ** (-s)
    q = total * w / w.sum()
    base = np.maximum(np.floor(q).astype(np.int64), 1)
    left = total - int(base.sum())
    if left > 0:
        order = np.argsort(-(q - np.floor(q)), kind="stable")
        base[order[:left]] += 1
    elif left < 0:  # the minimum of 1 overshot: take from the largest counts
        order = np.argsort(-base, kind="stable")
        i = 0
        while left < 0:
            if base[order[i % P]] > 1:
                base[order[i % P]] -= 1
                left += 1
            i += 1
    return base


CONV64_CONVS = [(64, 3, 1, 1), (64, 3, 2, 1), (64, 3, 1, 1), (64, 3, 2, 1)]


def cifar_conv64_set(P: int = 256, total: int = 32768, seed: int = SEED_WEIGHTS,
                     counts=None) -> WorkloadSet:
    """CNN 3x32x32 -> four 64-channel 3x3 convolutions (strides 1, 2, 1, 2,
    pad 1) -> linear 512 -> linear 10, He-normal, zero biases; P properties
    (own image centre U[0,1]^3072 and label, eps 2/255 clipped to [0,1]);
    subdomain counts Zipf(1.2) over the properties summing to ``total``
    unless ``counts`` is given; split depth ~ U{1..12}."""
    net = he_cnn((3, 32, 32), CONV64_CONVS, [512, 10], seed)
    if counts is None:
        counts = zipf_counts(P, 1.2, total)
    return property_set(net, 3072, (0.0, 1.0), 2.0 / 255.0, (0.0, 1.0), counts, (1, 12),
                        f"cnn3x32x32-4xc64-512-10 x {len(counts)} properties")


def small_conv4_set(P: int = 3, B: int = 48, seed: int = SEED_WEIGHTS) -> WorkloadSet:
    """The layer pattern of ``cifar_conv64_set`` at a size the oracle bounds in
    seconds: 3x8x8 -> four 8-channel 3x3 convolutions (strides 1, 2, 1, 2,
    pad 1) -> linear 32 -> linear 10, uniform biases; eps 0.02 around U[0,1]
    centres; Zipf(1.2) counts summing to B; split depth ~ U{1..6}."""
    net = he_cnn((3, 8, 8), [(8, 3, 1, 1), (8, 3, 2, 1), (8, 3, 1, 1), (8, 3, 2, 1)], [32, 10],
                 seed, bias="uniform")
    return property_set(net, 192, (0.0, 1.0), 0.02, (0.0, 1.0), zipf_counts(P, 1.2, B), (1, 6),
                        f"cnn3x8x8-4xc8-32-10 x {P} properties")


def mnist_mlp_set(counts, seed: int = SEED_WEIGHTS, k: int = 4) -> WorkloadSet:
    """The 784-256x6-10 MLP with len(counts) properties (centre U[0,1]^784,
    eps 0.02 clipped to [0,1]), ``k`` splits per subdomain."""
    net = he_mlp([784] + [256] * 6 + [10], seed)
    return property_set(net, 784, (0.0, 1.0), 0.02, (0.0, 1.0), counts, (k, k),
                        f"mlp784-256x6-10 x {len(counts)} properties")


def random_boxes_and_constraints(B: int, n: int, k: int, seed: int, width=0.5,
                                 p_zero_coef=0.1, p_flat=0.05, slack=0.5, nnz=8):
    """Random boxes [B, n] and dense constraints G [B, k, n], h [B, k] with
    ragged counts.  Half of the constraint rows have only ``nnz`` nonzero
    coefficients (so that clipping and empty intersections stay frequent in
    high dimension), the rest are dense with a fraction of exact zeros; each
    passes near a random point of the box (``slack`` scales the offset); a
    fraction of coordinates has zero width (degenerate cases).  float32."""
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-1.0, 1.0, (B, n))
    hi = lo + rng.uniform(0.0, width, (B, n))
    flat = rng.random((B, n)) < p_flat
    hi[flat] = lo[flat]
    G = rng.normal(size=(B, k, n))
    G[rng.random((B, k, n)) < p_zero_coef] = 0.0
    sparse = rng.random((B, k)) < 0.5
    if n > nnz:
        keep = np.argsort(rng.random((B, k, n)), axis=-1) < nnz
        G = np.where(sparse[..., None] & ~keep, 0.0, G)
    xs = rng.uniform(lo, hi)
    scale = np.sqrt(np.where(sparse, min(n, nnz), n)) * width
    h = -np.einsum("bkn,bn->bk", G, xs) + rng.normal(0.0, 1.0, (B, k)) * slack * scale
    count = rng.integers(0, k + 1, B).astype(np.int32)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return f(lo), f(hi), f(G), f(h), count


def random_planes(B: int, P: int, n: int, seed: int):
    """Random objective planes A [B, P, n], c [B, P] (float32)."""
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(B, P, n))
    A[rng.random((B, P, n)) < 0.05] = 0.0
    c = rng.normal(size=(B, P)) * np.sqrt(n)
    return np.ascontiguousarray(A, np.float32), np.ascontiguousarray(c, np.float32)


def random_alpha(B: int, M: int, n_hidden: int, seed: int):
    """Slopes in [0, 1] for every (subdomain, objective row, hidden neuron)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.0, 1.0, (B, M, n_hidden)), np.float32)


def tie_problems(B: int, n: int, k: int, P: int, seed: int):
    """Boxes, constraints and objective rows arranged so that complete
    clipping after relaxed clipping meets ties (float32; values on coarse
    dyadic grids, so products of inputs are exact).

    Each constraint has one dominant coefficient (+-8 against normal(0, 1)
    entries rounded to 1/16), which makes relaxed clipping tighten that
    coordinate; 30 % of the subdomains repeat constraint 0 as constraint 1.
    Each objective row puts the first constraint's dominant coordinate's
    breakpoint -A_j / G_0j far out (64) and makes about a third of the other
    coordinates share one breakpoint (1/4, 1/2, 1 or 2) against constraint 0;
    the rest are normal(0, 1) rounded to 1/16.  Each constraint's hyperplane
    passes through the box corner where g.x is smallest, moved into the box
    by a fraction (0.2 to 0.9) of what the dominant coordinate spans.
    Returns lo, hi [B, n], G [B, k, n], h [B, k], count [B], A [B, P, n],
    c [B, P]."""
    rng = np.random.default_rng(seed)
    grid = lambda x, s: np.round(x * s) / s
    lo = grid(rng.uniform(-1.0, 0.5, (B, n)), 64)
    hi = lo + grid(rng.uniform(0.25, 1.0, (B, n)), 64)
    G = grid(rng.normal(0.0, 1.0, (B, k, n)), 16)
    G[rng.random((B, k, n)) < 0.1] = 0.0
    dom = rng.integers(0, n, (B, k))
    bi, ki = np.meshgrid(np.arange(B), np.arange(k), indexing="ij")
    G[bi, ki, dom] = 8.0 * rng.choice([-1.0, 1.0], (B, k))
    if k >= 2:
        dup = rng.random(B) < 0.3
        G[dup, 1] = G[dup, 0]
    corner = np.where(G > 0.0, lo[:, None, :], hi[:, None, :])
    span = 8.0 * (hi[bi, dom] - lo[bi, dom])
    h = -np.einsum("bkn,bkn->bk", G, corner) - rng.uniform(0.2, 0.9, (B, k)) * span
    if k >= 2:
        h[dup, 1] = h[dup, 0]
    A = grid(rng.normal(0.0, 1.0, (B, P, n)), 16)
    g0 = G[:, 0][:, None, :]
    tie_q = rng.choice([0.25, 0.5, 1.0, 2.0], (B, P))[..., None]
    tied = (rng.random((B, P, n)) < 0.33) & (g0 != 0.0)
    A = np.where(tied, -tie_q * g0, A)
    A[np.arange(B)[:, None], np.arange(P)[None, :], dom[:, 0][:, None]] = \
        -64.0 * G[np.arange(B), 0, dom[:, 0]][:, None]
    c = np.zeros((B, P))
    count = np.full(B, k, np.int32)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return f(lo), f(hi), f(G), f(h), count, f(A), f(c)
