"""Writes tests/golden/conv64_props0_255.npz: FP64 oracle results at full
size for the 3x32x32 CNN with four 64-channel 3x3 convolutions (strides 1,
2, 1, 2, pad 1) -> 512 -> 10, properties 0 and 255 of the 256-property set
(``workloads.cifar_conv64_set``), computed only with ``oracle/`` and the
seeded generators of ``paper_2512_11087_amd.workloads``.

    python tests/golden/make_conv64_golden.py      # about half an hour, ~40 GB

For each property: the root pass (appendix A.3 plane recursion with the
fixed slope 0.5; rows of the +-I objectives bounded in blocks by
``crown.backward``, row by row the same computation as ``crown.root_pass``),
then 8 subdomains whose splits are drawn from the property's root-unstable
neurons (depth U{1..12}, the configuration's recipe, seed 2 + p + 1000),
the plain pass (``pipeline.run``: relaxed clipping, re-concretization,
CROWN, complete clipping) and 10 slope iterations (``pipeline.alpha_opt``,
Adam lr 0.1 with the float32 hyperparameters, float32 slope state between
iterations).  Stored: the splits (inputs), the root bounds of a sample of
neurons, the clipped boxes' digests, the plain and slope-optimised bounds.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import box, crown, pipeline as opipe  # noqa: E402
from paper_2512_11087_amd import workloads as wl  # noqa: E402

PROPS = (0, 255)
N_SUB = 8
STEPS = 10
BLOCK = 2048
OUT = os.path.join(HERE, "conv64_props0_255.npz")
f32 = lambda x: float(np.float32(x))


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def root_pass_blocked(layers, lo0, hi0, alpha0=0.5):
    """crown.root_pass with the objective rows of each layer in blocks."""
    lo, hi = lo0.astype(np.float64)[None], hi0.astype(np.float64)[None]
    W1, b1 = layers[0]
    lower, upper = [(W1.copy(), b1.copy())], [(W1.copy(), b1.copy())]
    ls = [box.concretize_min(W1[None], b1[None], lo, hi)[0]]
    us = [box.concretize_max(W1[None], b1[None], lo, hi)[0]]
    for i in range(2, len(layers)):
        n_i = layers[i - 1][0].shape[0]
        sub = layers[:i]
        lb_l = [x[None] for x in ls]
        lb_u = [x[None] for x in us]
        A_lo = np.empty((n_i, W1.shape[1]))
        A_hi = np.empty((n_i, W1.shape[1]))
        c_lo = np.empty(n_i)
        c_hi = np.empty(n_i)
        for j0 in range(0, n_i, BLOCK):
            j1 = min(n_i, j0 + BLOCK)
            I = np.eye(n_i)[j0:j1]
            A, c = crown.backward(sub, I, np.zeros(j1 - j0), lb_l, lb_u, alpha0)
            A_lo[j0:j1], c_lo[j0:j1] = A[0], c[0]
            A, c = crown.backward(sub, -I, np.zeros(j1 - j0), lb_l, lb_u, alpha0)
            A_hi[j0:j1], c_hi[j0:j1] = -A[0], -c[0]
        lower.append((A_lo, c_lo))
        upper.append((A_hi, c_hi))
        ls.append(box.concretize_min(A_lo[None], c_lo[None], lo, hi)[0])
        us.append(box.concretize_max(A_hi[None], c_hi[None], lo, hi)[0])
        log(f"  root layer {i}: {n_i} neurons")
    return crown.RootState(lower, upper, ls, us)


def main():
    ws = wl.cifar_conv64_set(256)
    log("dense layers")
    layers = crown.dense_layers(ws.net)
    out = {"props": np.array(PROPS), "n_sub": N_SUB, "steps": STEPS,
           "script": "tests/golden/make_conv64_golden.py"}
    rng = np.random.default_rng(17)
    for p in PROPS:
        w = ws.member(p)
        log(f"property {p}: root pass")
        root = root_pass_blocked(layers, w.lo0, w.hi0, 0.5)
        A_lo, c_lo, A_hi, c_hi, l0, u0 = root.stacked()
        unst = np.nonzero((l0 < 0) & (u0 > 0))[0]
        depth = np.random.default_rng(wl.SEED_SIZES + 1000 + p).integers(1, 13, N_SUB)
        sp = wl.draw_splits(N_SUB, depth, unst, seed=wl.SEED_SPLITS + p + 1000, kmax=12)
        sample = np.sort(rng.choice(l0.size, 512, replace=False))
        log(f"property {p}: {unst.size} unstable; plain pass")
        lo = np.broadcast_to(w.lo0, (N_SUB, w.lo0.size)).astype(np.float64)
        hi = np.broadcast_to(w.hi0, (N_SUB, w.hi0.size)).astype(np.float64)
        ref = opipe.run(layers, root, w.C, w.t, lo, hi, sp.neuron, sp.sign, sp.count)
        fe = ~ref["infeasible"]
        log(f"property {p}: {int(fe.sum())} feasible; {STEPS} slope steps")
        best = np.full(ref["lb"].shape, np.nan)
        if fe.any():
            b, _, _ = opipe.alpha_opt(layers, w.C, w.t, opipe.split_layers(layers, ref["l"][fe]),
                                      opipe.split_layers(layers, ref["u"][fe]), ref["lo"][fe],
                                      ref["hi"][fe], ref["G"][fe], ref["h"][fe], ref["active"][fe],
                                      steps=STEPS, lr=f32(0.1), b1=f32(0.9), b2=f32(0.999),
                                      eps=f32(1e-8), state32=True)
            best[fe] = b
        out.update({
            f"p{p}_neuron": sp.neuron, f"p{p}_sign": sp.sign, f"p{p}_count": sp.count,
            f"p{p}_n_unstable": unst.size,
            f"p{p}_root_sample": sample, f"p{p}_root_l": l0[sample], f"p{p}_root_u": u0[sample],
            f"p{p}_infeasible": ref["infeasible"], f"p{p}_lb": ref["lb"],
            f"p{p}_best": best,
            f"p{p}_lo_sum": ref["lo"].sum(-1), f"p{p}_hi_sum": ref["hi"].sum(-1),
        })
        del root, A_lo, A_hi, ref
    np.savez_compressed(OUT, **out)
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
