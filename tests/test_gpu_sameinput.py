"""Same-input, directional parity of the backward pass (Lemma A.3), the final
concretization (Lemma A.2) and complete clipping of the final rows (Thm 3.1,
coordinate ascent), at full size.

The GPU's own intermediate bounds l, u (float32, the output of its
re-concretization step) are handed to the oracle as data, so the backward
pass is compared on identical inputs and the GPU bound must be within 1e-5
of the oracle's AND not above it beyond the oracle's own rounding
(1e-9 relative): the GPU subtracts a rigorous rounding bound, so a GPU bound
above the oracle's would be unsound.

* Final concretization alone (complete clipping off), over the GPU's box:
  the direct check of the fused concretization.
* With complete clipping: over the oracle's own clipped box and split
  halfspaces (its float64 relaxed clipping of the same splits).  The GPU's
  box contains the oracle's and its halfspaces are looser, so the GPU bound
  is again the smaller one; the oracle's box keeps the flat dual segments
  that relaxed clipping creates exactly flat, where the oracle's tie rule
  applies.
Samples: 256 subdomains of the 784-256x6 bench batch (16384 subdomains) and
64 of the CIFAR CNN batch (4096 subdomains).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import box, crown, pipeline as opipe  # noqa: E402
from paper_2512_11087_amd import api, pipeline as gpipe, workloads as wl  # noqa: E402
from helpers import OracleProp, assert_close, subset_splits  # noqa: E402

pytestmark = pytest.mark.gpu

REL = 1e-5
DIR = 1e-9


def H(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,make,n_sample", [
    ("mlp784-256x6-10", lambda: wl.mnist_mlp(B=16384), 256),
    ("cnn3x32x32", lambda: wl.cifar_cnn(4096), 64)])
def test_backward_concretize_and_clip_on_the_gpus_bounds(name, make, n_sample):
    w = make()
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts, op.unstable())
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig(complete_final=False))
    lb_plain = out["lb"].clone()
    inf = out["infeasible"].clone()
    lb_clip = api.bound_propagate(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], batch.lo,
                                  batch.hi, None, 0.5, inf, batch.cons(), 1, ws=prop.ws)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(31).choice(w.B, n_sample, replace=False))
    ref = op.run(subset_splits(sp, idx))
    fe = ~ref["infeasible"] & ~H(inf)[idx].astype(bool)
    assert fe.sum() >= n_sample // 2
    l, u = H(out["l"])[idx][fe].astype(np.float64), H(out["u"])[idx][fe].astype(np.float64)
    A, c = crown.backward(op.layers, w.C, w.t, opipe.split_layers(op.layers, l),
                          opipe.split_layers(op.layers, u), 0.5)
    # (a) backward + concretization over the GPU's box
    glo, ghi = H(batch.lo)[idx][fe], H(batch.hi)[idx][fe]
    olb0 = box.concretize_min(A, c, glo, ghi)
    g0 = H(lb_plain)[idx][fe]
    e0 = assert_close(g0, olb0, REL, f"{name}: bound without complete clipping")
    assert np.all(g0 <= olb0 + DIR * np.maximum(np.abs(olb0), 1.0)), "GPU bound above the oracle's"
    # (b) with complete clipping: the oracle's own box and halfspaces
    L, _, emp = opipe.final_clip(A, c, ref["G"][fe], ref["h"][fe], ref["active"][fe],
                                 ref["lo"][fe], ref["hi"][fe])
    olb = np.maximum(box.concretize_min(A, c, ref["lo"][fe], ref["hi"][fe]), L)
    g = H(lb_clip)[idx][fe]
    assert not emp.any() or np.isinf(g[emp]).all()
    keep = ~emp
    e1 = assert_close(g[keep], olb[keep], REL, f"{name}: bound with complete clipping")
    assert np.all(g[keep] <= olb[keep] + DIR * np.maximum(np.abs(olb[keep]), 1.0)), \
        "GPU clipped bound above the oracle's"
    gain = (olb[keep] - olb0[keep] > 1e-6).mean()
    print(f"{name}: {fe.sum()} subdomains; max rel err {e0:.2e} (no clip), {e1:.2e} (clip); "
          f"complete clipping raised {gain:.0%} of the rows")
    assert gain > 0.0
