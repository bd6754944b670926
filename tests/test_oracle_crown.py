"""Pins the CROWN oracle (root pass, backward pass, pipeline, slope adjoint,
Adam) to facts fixed by the mathematics: sampled soundness, exactness on an
all-stable network, the conv matrix against an independent convolution,
per-step monotonicity, central finite differences, Adam's closed form."""
import numpy as np
import pytest

from oracle import box, crown, exact, pipeline
from paper_2512_11087_amd import workloads as wl


def small_net(seed, widths, bias="uniform"):
    return wl.he_mlp(widths, seed, bias=bias)


def test_all_stable_network_is_exact():
    # positive weights and a positive box: every neuron is active, the
    # network is affine on the box and CROWN is exact
    rng = np.random.default_rng(0)
    W1 = np.abs(rng.normal(size=(4, 3)))
    W2 = np.abs(rng.normal(size=(3, 4)))
    W3 = rng.normal(size=(2, 3))
    layers = [(W1, np.full(4, 0.1)), (W2, np.full(3, 0.2)), (W3, np.zeros(2))]
    lo, hi = np.full(3, 0.5), np.full(3, 1.5)
    root = crown.root_pass(layers, lo, hi)
    assert all(np.all(l >= 0) for l in root.l)
    A, c = crown.backward(layers, np.eye(2), np.zeros(2), [x[None] for x in root.l],
                          [x[None] for x in root.u], 0.5)
    lb = box.concretize_min(A, c, lo[None], hi[None])[0]
    Weff = W3 @ W2 @ W1
    beff = W3 @ (W2 @ np.full(4, 0.1) + np.full(3, 0.2))
    for m in range(2):
        assert lb[m] == pytest.approx(exact.box_corners_min(Weff[m], beff[m], lo, hi), abs=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_root_pass_and_crown_are_sound_on_samples(seed):
    net = small_net(seed, [4, 12, 12, 12, 3])
    layers = crown.dense_layers(net)
    rng = np.random.default_rng(seed)
    centre = rng.uniform(-1, 1, 4)
    lo, hi = wl.box_around(centre, 0.3)
    lo, hi = lo.astype(float), hi.astype(float)
    root = crown.root_pass(layers, lo, hi)
    x = rng.uniform(lo, hi, size=(100000, 4))
    z = wl.pre_activations(net, x)
    A_lo, c_lo, A_hi, c_hi, l0, u0 = root.stacked()
    assert np.all(z >= l0 - 1e-9) and np.all(z <= u0 + 1e-9)
    assert np.all(x @ A_lo.T + c_lo <= z + 1e-9)
    assert np.all(x @ A_hi.T + c_hi >= z - 1e-9)
    C, t = wl.identity_spec(3)
    A, c = crown.backward(layers, C, t, [v[None] for v in root.l], [v[None] for v in root.u], 0.5)
    y = wl.forward(net, x)
    assert np.all(x @ A[0].T + c[0] <= y + 1e-9)


def test_conv_matrix_matches_direct_convolution():
    net = wl.he_cnn((2, 6, 6), [(3, 4, 2, 1), (2, 3, 1, 1)], [4], seed=5, bias="uniform")
    layers = crown.dense_layers(net)
    x = np.random.default_rng(0).normal(size=(7, 72))
    h = x
    for i, (ly, (W, b)) in enumerate(zip(net.layers, layers)):
        assert np.allclose(h @ W.T + b, wl.affine(ly, h), atol=1e-12)
        h = np.maximum(wl.affine(ly, h), 0)


def tiny_setup(B=64, seed=0, bias="zero"):
    w = wl.tiny_mlp(B)
    if bias != "zero":
        w.net = wl.he_mlp([5] + [50] * 6 + [5], 0, bias=bias)
    layers = crown.dense_layers(w.net)
    root = crown.root_pass(layers, w.lo0, w.hi0, 0.5)
    return w, layers, root


@pytest.mark.parametrize("cfg", [pipeline.Config(),
                                 pipeline.Config(relaxed="sequential", complete_intermediate=True),
                                 pipeline.Config(split_fix=False, complete_final=False),
                                 pipeline.Config(relaxed="sequential", complete_intermediate=True,
                                                 order=True)])
def test_pipeline_sound_with_true_split_pattern(cfg):
    w, layers, root = tiny_setup(bias="uniform")
    rng = np.random.default_rng(wl.SEED_SAMPLES)
    B = 64
    lo0, hi0 = w.lo0.astype(float), w.hi0.astype(float)
    anchors = rng.uniform(lo0, hi0, size=(B, 5))
    sp = wl.splits_from_points(w.net, anchors, w.split_counts[:B], np.arange(w.net.n_hidden))
    lo = np.broadcast_to(lo0, (B, 5))
    hi = np.broadcast_to(hi0, (B, 5))
    out = pipeline.run(layers, root, w.C, w.t, lo, hi, sp.neuron, sp.sign, sp.count, cfg)
    # the anchor of every subdomain is feasible: nothing may be pruned
    assert not out["infeasible"].any()
    x = np.concatenate([anchors[:, None, :], rng.uniform(lo0, hi0, size=(B, 2000, 5))], axis=1)
    z = wl.pre_activations(w.net, x.reshape(-1, 5)).reshape(B, -1, w.net.n_hidden)
    y = wl.forward(w.net, x.reshape(-1, 5)).reshape(B, -1, 5)
    for b in range(B):
        k = sp.count[b]
        idx, sg = sp.neuron[b, :k], sp.sign[b, :k]
        feas = np.all(np.where(sg > 0, z[b][:, idx] >= 0, z[b][:, idx] <= 0), axis=1)
        xs, zs, ys = x[b][feas], z[b][feas], y[b][feas]
        assert feas[0]
        assert np.all(xs >= out["lo"][b] - 1e-12) and np.all(xs <= out["hi"][b] + 1e-12)
        assert np.all(zs >= out["l"][b] - 1e-9) and np.all(zs <= out["u"][b] + 1e-9)
        assert np.all(ys @ w.C.T + w.t >= out["lb"][b] - 1e-9)


def test_pipeline_monotone_per_step():
    w, layers, root = tiny_setup(B=256)
    cand = np.arange(w.net.n_hidden)
    sp = wl.draw_splits(w.B, w.split_counts, cand)
    lo = np.broadcast_to(w.lo0, (w.B, 5)).astype(float)
    hi = np.broadcast_to(w.hi0, (w.B, 5)).astype(float)
    out = pipeline.run(layers, root, w.C, w.t, lo, hi, sp.neuron, sp.sign, sp.count,
                       pipeline.Config(complete_intermediate=True))
    fe = ~out["infeasible"]
    assert np.all(out["lo"][fe] >= lo[fe]) and np.all(out["hi"][fe] <= hi[fe])
    _, _, _, _, l0, u0 = root.stacked()
    assert np.all(out["l_reconc"][fe] >= l0 - 1e-12) and np.all(out["u_reconc"][fe] <= u0 + 1e-12)
    assert np.all(out["l"][fe] >= out["l_reconc"][fe] - 1e-12)
    assert np.all(out["u"][fe] <= out["u_reconc"][fe] + 1e-12)
    assert np.all(out["lb"][fe] >= out["lb_unclipped"][fe] - 1e-12)
    assert np.all(np.isinf(out["lb"][~fe]))
    # tiny config has both infeasible and improved subdomains
    assert out["infeasible"].any() and (out["lb"][fe] > out["lb_unclipped"][fe] + 1e-9).any()


def test_alpha_gradient_matches_central_differences():
    w, layers, root = tiny_setup(B=16, bias="uniform")
    rng = np.random.default_rng(4)
    sp = wl.draw_splits(16, w.split_counts[:16], np.arange(w.net.n_hidden))
    lo = np.broadcast_to(w.lo0, (16, 5)).astype(float)
    hi = np.broadcast_to(w.hi0, (16, 5)).astype(float)
    out = pipeline.run(layers, root, w.C, w.t, lo, hi, sp.neuron, sp.sign, sp.count)
    fe = ~out["infeasible"]
    l_list = pipeline.split_layers(layers, out["l"][fe])
    u_list = pipeline.split_layers(layers, out["u"][fe])
    Bf = int(fe.sum())
    alpha = [rng.uniform(0.1, 0.9, size=(Bf, 5, 50)) for _ in range(6)]
    args = (w.C, w.t, l_list, u_list)
    G, h, act, lo2, hi2 = out["G"][fe], out["h"][fe], out["active"][fe], out["lo"][fe], out["hi"][fe]
    lb, grads, beta, emp = pipeline.bound_and_grad(layers, *args, alpha, lo2, hi2, G, h, act)
    hstep = 1e-4
    checked = 0
    for _ in range(60):
        kk = int(rng.integers(6))
        b, m, j = int(rng.integers(Bf)), int(rng.integers(5)), int(rng.integers(50))
        vals = []
        for d in (hstep, -hstep, hstep / 2, -hstep / 2):
            al = [a.copy() for a in alpha]
            al[kk][b, m, j] += d
            vals.append(pipeline.bound_and_grad(layers, *args, al, lo2, hi2, G, h, act)[0][b, m])
        fd = (vals[0] - vals[1]) / (2 * hstep)
        fd2 = (vals[2] - vals[3]) / hstep
        if not np.isfinite(fd) or abs(fd - fd2) > 1e-6 * max(1.0, abs(fd)):
            continue            # a kink lies within +-h: central differences are invalid there
        assert grads[kk][b, m, j] == pytest.approx(fd, rel=1e-5, abs=1e-7)
        checked += 1
    assert checked > 30
    assert sum(np.count_nonzero(g) for g in grads) > 0


def test_adam_closed_form_for_constant_gradient():
    # with a constant gradient g the bias-corrected step is lr*g/(|g|+eps):
    # the parameter moves by ~lr per step until it hits the [0, 1] clamp
    p = np.array([0.5, 0.5, 0.5])
    g = np.array([2.0, -3.0, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    for s in range(1, 4):
        p, m, v = pipeline.adam_ascent(p, g, m, v, s, 0.1)
        assert p[0] == pytest.approx(min(1.0, 0.5 + 0.1 * s), abs=1e-7)
        assert p[1] == pytest.approx(max(0.0, 0.5 - 0.1 * s), abs=1e-7)
        assert p[2] == 0.5


def test_alpha_opt_never_worse_than_plain():
    w, layers, root = tiny_setup(B=32, bias="uniform")
    sp = wl.draw_splits(32, w.split_counts[:32], np.arange(w.net.n_hidden))
    lo = np.broadcast_to(w.lo0, (32, 5)).astype(float)
    hi = np.broadcast_to(w.hi0, (32, 5)).astype(float)
    out = pipeline.run(layers, root, w.C, w.t, lo, hi, sp.neuron, sp.sign, sp.count)
    fe = ~out["infeasible"]
    l_list = pipeline.split_layers(layers, out["l"][fe])
    u_list = pipeline.split_layers(layers, out["u"][fe])
    best, hist, _ = pipeline.alpha_opt(layers, w.C, w.t, l_list, u_list, out["lo"][fe], out["hi"][fe],
                                       out["G"][fe], out["h"][fe], out["active"][fe], steps=8)
    assert np.allclose(hist[0], out["lb"][fe])          # first iterate = plain bound
    assert np.all(best >= out["lb"][fe] - 1e-12)
    assert (best > out["lb"][fe] + 1e-6).any()


def test_crown_intermediate_bounds_of_fresh_boxes():
    # the root box reproduces the root pass; sub-boxes get sound bounds that
    # are at least as tight as the re-concretized cached planes, and tighter
    # somewhere
    w, layers, root = tiny_setup(bias="uniform")
    _, _, _, _, l0, u0 = root.stacked()
    lo0 = w.lo0.astype(float)[None]
    hi0 = w.hi0.astype(float)[None]
    l, u = pipeline.reconcretize(root, lo0, hi0)
    l, u, _ = pipeline.fix_bounds(root, l, u, np.zeros((1, 0), int), np.zeros((1, 0), int),
                                  np.zeros(1, int), False)
    lc, uc = pipeline.crown_intermediate(layers, root, lo0, hi0, l, u)
    assert np.allclose(lc[0], l0, atol=1e-12) and np.allclose(uc[0], u0, atol=1e-12)
    rng = np.random.default_rng(7)
    B = 32
    a = rng.uniform(w.lo0, w.hi0, size=(B, 5))
    b = rng.uniform(w.lo0, w.hi0, size=(B, 5))
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    l, u = pipeline.reconcretize(root, lo, hi)
    l, u, _ = pipeline.fix_bounds(root, l, u, np.zeros((B, 0), int), np.zeros((B, 0), int),
                                  np.zeros(B, int), False)
    lc, uc = pipeline.crown_intermediate(layers, root, lo, hi, l, u)
    assert np.all(lc >= l) and np.all(uc <= u) and (lc > l + 1e-9).any()
    for bb in range(B):
        x = rng.uniform(lo[bb], hi[bb], size=(3000, 5))
        z = wl.pre_activations(w.net, x)
        assert np.all(z >= lc[bb] - 1e-9) and np.all(z <= uc[bb] + 1e-9)
