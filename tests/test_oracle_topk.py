"""Pins the neuron-selection heuristic (BaBSR intercept score, heuristics
appendix): the score's closed form on hand values, its weights against the
backward coefficients that need no relaxation (the last hidden layer sees
C W_L exactly), the per-layer top-k with index tie-break, and that complete
clipping restricted to the selection stays sound and between plain
re-concretization and clipping every unstable neuron."""
import numpy as np

from oracle import crown, pipeline
from paper_2512_11087_amd import workloads as wl


def test_score_closed_form():
    l = np.array([[-1.0, 0.5, -2.0, -3.0]])
    u = np.array([[3.0, 2.0, -0.5, 1.0]])
    w = np.array([2.0, 7.0, 7.0, 0.0])
    sc = pipeline.babsr_scores(l, u, w)
    # unstable neuron 0: (1 * 3 / 4) * 2; stable ones and zero weight: 0
    assert np.allclose(sc, [[1.5, 0.0, 0.0, 0.0]])


def test_weights_of_last_hidden_layer_are_C_times_W():
    net = wl.he_mlp([4, 9, 7, 3], 5, bias="uniform")
    layers = crown.dense_layers(net)
    lo, hi = np.full(4, -0.5), np.full(4, 0.5)
    root = crown.root_pass(layers, lo, hi)
    C = np.array([[1.0, -1.0, 0.0], [0.0, 1.0, -1.0]])
    w = pipeline.babsr_weights(layers, C, np.zeros(2), root)
    W3 = layers[2][0]
    expect = np.maximum(0.0, -(C @ W3).mean(axis=0))
    assert w.shape == (16,)
    assert np.allclose(w[9:], expect, atol=1e-14)
    assert np.all(w >= 0.0)


def test_topk_per_layer_with_index_tie_break():
    l = np.array([[-1.0, -1.0, -1.0, -1.0, 1.0, -1.0, -1.0]])
    u = np.array([[1.0, 1.0, 1.0, 1.0, 2.0, 1.0, 1.0]])
    # icpt = 0.5 for every unstable neuron; the weights set the scores
    w = np.array([6.0, 10.0, 10.0, 2.0, 9.0, 4.0, 4.0])
    sizes = [5, 2]
    sel = pipeline.topk_select(l, u, w, sizes, 2)
    assert sel.tolist() == [[False, True, True, False, False, True, True]]
    sel = pipeline.topk_select(l, u, w, sizes, 3)
    assert sel.tolist() == [[True, True, True, False, False, True, True]]
    sel = pipeline.topk_select(l, u, w, sizes, 0)
    assert not sel.any()


def test_topk_clipping_is_sound_and_between_none_and_all():
    w = wl.tiny_mlp(64)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 1, bias="uniform")
    layers = crown.dense_layers(w.net)
    root = crown.root_pass(layers, w.lo0, w.hi0)
    wt = pipeline.babsr_weights(layers, w.C, w.t, root)
    rng = np.random.default_rng(wl.SEED_SAMPLES)
    anchors = rng.uniform(w.lo0, w.hi0, size=(64, 5))
    sp = wl.splits_from_points(w.net, anchors, w.split_counts[:64], np.arange(w.net.n_hidden))
    lo = np.broadcast_to(w.lo0, (64, 5)).astype(float)
    hi = np.broadcast_to(w.hi0, (64, 5)).astype(float)
    run = lambda cfg: pipeline.run(layers, root, w.C, w.t, lo, hi, sp.neuron, sp.sign, sp.count, cfg)
    none = run(pipeline.Config(complete_intermediate=False))
    allc = run(pipeline.Config(complete_intermediate=True))
    top = run(pipeline.Config(complete_intermediate=True, topk=5, babsr_weight=wt))
    big = run(pipeline.Config(complete_intermediate=True, topk=10 ** 6, babsr_weight=wt))
    assert not top["infeasible"].any()
    assert (top["select"].sum(-1) <= 5 * 6).all() and top["select"].any()
    # k larger than every layer = all unstable neurons
    assert np.array_equal(big["l"], allc["l"]) and np.array_equal(big["u"], allc["u"])
    # the selection only tightens, never more than clipping every neuron
    assert np.all(top["l"] >= none["l"] - 1e-12) and np.all(top["u"] <= none["u"] + 1e-12)
    assert np.all(top["l"] <= allc["l"] + 1e-12) and np.all(top["u"] >= allc["u"] - 1e-12)
    assert (top["l"] > none["l"] + 1e-9).any()
    x = rng.uniform(w.lo0, w.hi0, size=(2000, 5))
    z = wl.pre_activations(w.net, x)
    for b in range(64):
        k = sp.count[b]
        idx, sg = sp.neuron[b, :k], sp.sign[b, :k]
        feas = np.all(np.where(sg > 0, z[:, idx] >= 0, z[:, idx] <= 0), axis=1)
        assert np.all(z[feas] >= top["l"][b] - 1e-9) and np.all(z[feas] <= top["u"][b] + 1e-9)
