"""Parity of the HIP path (called through the C ABI) with the FP64 oracle on
the same seeded inputs, plus directional soundness checks.

Kernel-level tests feed both sides identical float32 inputs, so the GPU
result must equal the oracle's within the parity band AND lie on the safe
side of it (a clipped box never smaller, a lower bound never larger than the
exact value, up to the oracle's own float64 rounding).  Pipeline tests
compare the whole pass; their inputs to intermediate steps (cached planes,
intermediate bounds) are computed by each side independently.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import complete, crown, pipeline as opipe, relaxed  # noqa: E402
from paper_2512_11087_amd import api, pipeline as gpipe, workloads as wl  # noqa: E402
from helpers import ADAM, OracleProp, assert_close, subset_splits  # noqa: E402

pytestmark = pytest.mark.gpu

DIR = 1e-12   # slack for the oracle's own float64 rounding in directional checks


def T(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dtype)


def H(t):
    return t.detach().cpu().numpy()


def sync():
    torch.cuda.synchronize()


# ------------------------------------------------------------ relaxed clip

@pytest.mark.parametrize("n", [5, 37, 784])
@pytest.mark.parametrize("mode", ["parallel", "sequential"])
def test_clip_dense_matches_oracle_and_contains_it(n, mode):
    B, k = 300, 6
    lo, hi, G, h, count = wl.random_boxes_and_constraints(B, n, k, seed=20 + n)
    lo_t, hi_t = T(lo), T(hi)
    cons = api.Constraints.dense(G, h, count)
    inf = H(api.clip_domains(None, lo_t, hi_t, cons, mode))
    sync()
    act = np.arange(k)[None, :] < count[:, None]
    fn = relaxed.clip_parallel if mode == "parallel" else relaxed.clip_sequential
    olo, ohi, oinf = fn(G, h, lo, hi, act)
    assert np.array_equal(inf.astype(bool), oinf), "infeasible flags differ"
    assert 0 < oinf.sum() < B
    glo, ghi = H(lo_t).astype(np.float64), H(hi_t).astype(np.float64)
    fe = ~oinf
    scale = np.maximum(np.abs(olo[fe]), 1.0)
    assert np.all(glo[fe] <= olo[fe] + DIR * scale), "GPU lower bound tighter than exact"
    assert np.all(ghi[fe] >= ohi[fe] - DIR * np.maximum(np.abs(ohi[fe]), 1.0))
    assert_close(glo[fe], olo[fe], 1e-6, "lo")
    assert_close(ghi[fe], ohi[fe], 1e-6, "hi")
    assert (glo[fe] > lo[fe]).any() and (ghi[fe] < hi[fe]).any()   # something was clipped


# ------------------------------------------------- concretize / complete clip

@pytest.mark.parametrize("n", [5, 130, 784])
def test_concretize_and_complete_clip_match_oracle(n):
    B, P, k = 97, 3, 5
    lo, hi, G, h, count = wl.random_boxes_and_constraints(B, n, k, seed=40 + n, slack=0.2)
    A, c = wl.random_planes(B, P, n, seed=41 + n)
    lb, ub, _ = api.concretize(T(A), T(c), T(lo), T(hi), want_ub=True)
    cons = api.Constraints.dense(G, h, count)
    inf = torch.zeros(B, dtype=torch.uint8, device="cuda")
    lbc, _, beta = api.concretize(T(A), T(c), T(lo), T(hi), cons, want_beta=True, infeasible=inf)
    sync()
    from oracle import box
    olb = box.concretize_min(A, c, lo, hi)
    oub = box.concretize_max(A, c, lo, hi)
    sc = (np.abs(A) * np.maximum(np.abs(lo), np.abs(hi))[:, None, :]).sum(-1) + np.abs(c)
    assert np.all(H(lb) <= olb + DIR * sc) and np.all(H(ub) >= oub - DIR * sc)
    assert_close(H(lb), olb, 1e-6, "lb")
    assert_close(H(ub), oub, 1e-6, "ub")
    act = np.arange(k)[None, :] < count[:, None]
    rep = lambda x: np.repeat(x, P, axis=0)
    L, obeta, oinf = complete.coord_ascent(A.reshape(B * P, n), c.reshape(B * P), rep(G), rep(h),
                                           rep(lo), rep(hi), rep(act))
    L = np.maximum(L.reshape(B, P), olb)
    oinf = oinf.reshape(B, P).any(-1)
    assert np.array_equal(H(inf).astype(bool), oinf)
    fe = ~oinf
    g = H(lbc)
    assert np.all(np.isinf(g[oinf]))
    assert np.all(g[fe] <= L[fe] + DIR * sc[fe]), "complete clip above the exact dual value"
    assert_close(g[fe], L[fe], 1e-6, "complete clip")
    assert (L[fe] > olb[fe] + 1e-6).any()      # clipping tightened something
    # multipliers: where the oracle's is unique the GPU finds the same one
    gb = H(beta).reshape(B * P, k)
    ob = obeta
    keep = np.repeat(fe, P)
    assert_close(gb[keep], ob[keep], 1e-5, "beta")


def test_complete_clip_single_constraint_is_exact_lp():
    # one constraint: Thm 3.1 says the dual optimum equals the LP optimum
    from oracle import exact
    B, P, n, k = 40, 1, 6, 1
    lo, hi, G, h, _ = wl.random_boxes_and_constraints(B, n, k, seed=7, slack=0.3)
    A, c = wl.random_planes(B, P, n, seed=8)
    cons = api.Constraints.dense(G, h, np.ones(B, np.int32))
    lbc, _, _ = api.concretize(T(A), T(c), T(lo), T(hi), cons)
    g = H(lbc)[:, 0]
    for b in range(B):
        v = exact.lp_vertices(A[b, 0], c[b, 0], G[b], h[b], lo[b], hi[b])[0]
        if np.isinf(v):
            assert np.isinf(g[b])
        else:
            assert g[b] <= v + 1e-9 and g[b] == pytest.approx(v, rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("n", [784, 3072], ids=["wave-team", "workgroup-team"])
def test_complete_clip_search_with_skewed_breakpoints_and_weights(n):
    # the weighted-quantile search on inputs that interpolation serves badly:
    # breakpoints q_j = -a_j/g_j spread log-uniformly over 12 decades, weights
    # |g_j| (hi_j - lo_j) over 6 decades plus one weight far above the rest,
    # and the crossing placed at varying depths; every coordinate is a
    # candidate.  Thm 3.1: the bound at the exact quantile is the oracle's.
    B = 24
    rng = np.random.default_rng(2512)
    lo = np.full((B, n), -1.0, np.float32)
    hi = np.full((B, n), 1.0, np.float32)
    mag = (10.0 ** rng.uniform(-3, 3, (B, n))).astype(np.float32)
    mag[np.arange(B), rng.integers(0, n, B)] = 1e5          # one dominant weight
    g = (mag * rng.choice([-1.0, 1.0], (B, n))).astype(np.float32)
    q = 10.0 ** rng.uniform(-6, 6, (B, n))
    A = (-q * g).astype(np.float32)                          # opposite signs: all candidates
    depth = np.linspace(0.05, 0.95, B)                       # where the crossing falls
    h = (depth * np.abs(g.astype(np.float64)).sum(1)).astype(np.float32)
    c = np.zeros((B, 1), np.float32)
    cons = api.Constraints.dense(g[:, None, :], h[:, None], np.ones(B, np.int32))
    lbc, _, _ = api.concretize(T(A[:, None, :]), T(c), T(lo), T(hi), cons)
    L, beta, inf = complete.single_max(A, c[:, 0], g, h, lo, hi)
    assert not inf.any() and (beta > 0).all()                # every problem searches
    assert_close(H(lbc)[:, 0], L, 1e-5, "skewed search")
    assert np.all(H(lbc)[:, 0] <= L + 1e-6 * np.maximum(np.abs(L), 1.0))


# ---------------------------------------------------------------- root pass

@pytest.mark.parametrize("make", [lambda: wl.tiny_mlp(8), lambda: wl.mnist_mlp(8),
                                  lambda: wl.cifar_cnn(8), lambda: wl.ragged_cnn(8),
                                  lambda: wl.wide_cnn(8), lambda: wl.edge_cnn(8)],
                         ids=["mlp5-50x6-5", "mlp784-256x6-10", "cnn3x32x32", "cnn5x9x7",
                              "cnn4x24x24", "cnn3x7x7-edge"])
def test_root_pass_matches_oracle_and_is_sound(make):
    w = make()
    op = OracleProp(w)
    prop = gpipe.Property.from_workload(w)
    l0, u0 = prop.root.bounds()
    A_lo, c_lo, A_hi, c_hi = prop.root.planes()
    sync()
    assert_close(H(l0), op.l0, 1e-5, "root l")
    assert_close(H(u0), op.u0, 1e-5, "root u")
    oA_lo, oc_lo, oA_hi, oc_hi, _, _ = op.root.stacked()
    X = np.maximum(np.abs(w.lo0), np.abs(w.hi0)).astype(np.float64)
    rs = np.abs(oA_lo) @ X + np.abs(oc_lo) + 1.0
    assert np.all(np.abs(H(A_lo) - oA_lo) @ X <= 1e-5 * rs)
    assert np.all(np.abs(H(c_lo) - oc_lo) <= 1e-5 * rs)
    assert np.all(np.abs(H(c_hi) - oc_hi) <= 1e-5 * (np.abs(oA_hi) @ X + np.abs(oc_hi) + 1.0))
    assert prop.root.n_unstable == int(((op.l0 < 0) & (op.u0 > 0)).sum())
    # planes and bounds hold at sampled points of the root box
    rng = np.random.default_rng(wl.SEED_SAMPLES)
    x = rng.uniform(w.lo0, w.hi0, size=(4000, w.net.n_in))
    z = wl.pre_activations(w.net, x)
    assert np.all(z >= H(l0)) and np.all(z <= H(u0))
    assert np.all(x @ H(A_lo).astype(np.float64).T + H(c_lo) <= z + 1e-9 * np.abs(z).max())
    assert np.all(x @ H(A_hi).astype(np.float64).T + H(c_hi) >= z - 1e-9 * np.abs(z).max())


# ------------------------------------------------------------- whole pass

def run_both(w, sp, cfg_g, cfg_o, op=None):
    op = op or OracleProp(w)
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, cfg_g)
    sync()
    ref = op.run(sp, cfg=cfg_o)
    return prop, batch, out, ref, op


def compare_pass(out, batch, ref, op, rel=1e-5):
    """Whole pass, each side with its own intermediate steps: every result
    within ``rel`` of the oracle's, and the GPU's never the tighter one
    beyond the oracle's own rounding (its boxes contain the oracle's, its
    bounds are not above them)."""
    ginf = H(out["infeasible"]).astype(bool)
    oinf = ref["infeasible"]
    assert not (ginf & ~oinf).any(), "GPU pruned a subdomain the oracle keeps"
    assert (ginf == oinf).mean() > 0.999
    fe = ~oinf & ~ginf
    glo, ghi = H(batch.lo)[fe].astype(np.float64), H(batch.hi)[fe].astype(np.float64)
    assert np.all(glo <= ref["lo"][fe] + DIR * np.maximum(np.abs(ref["lo"][fe]), 1.0)), "box tighter"
    assert np.all(ghi >= ref["hi"][fe] - DIR * np.maximum(np.abs(ref["hi"][fe]), 1.0)), "box tighter"
    assert_close(glo, ref["lo"][fe], 1e-5, "clipped lo")
    assert_close(ghi, ref["hi"][fe], 1e-5, "clipped hi")
    unst = op.unstable()
    gl, gu = H(out["l"])[fe][:, unst], H(out["u"])[fe][:, unst]
    ol, ou = ref["l"][fe][:, unst], ref["u"][fe][:, unst]
    assert np.all(gl <= ol + 1e-9 * np.maximum(np.abs(ol), 1.0)), "intermediate l above the oracle's"
    assert np.all(gu >= ou - 1e-9 * np.maximum(np.abs(ou), 1.0)), "intermediate u below the oracle's"
    assert_close(gl, ol, rel, "l")
    assert_close(gu, ou, rel, "u")
    glb = H(out["lb"])
    assert np.all(np.isinf(glb[ginf]))
    olb = ref["lb"][fe]
    above = glb[fe] > olb + 1e-9 * np.maximum(np.abs(olb), 1.0)
    assert not above.any(), f"GPU bound above the oracle's on {above.sum()} rows"
    return assert_close(glb[fe], olb, rel, "lb")


@pytest.mark.parametrize("mode", ["parallel", "sequential"])
def test_pass_tiny_matches_oracle(mode):
    w = wl.tiny_mlp(1024)
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts, np.arange(w.net.n_hidden))
    cfg_g = gpipe.PassConfig(clip=mode, complete_intermediate=True)
    cfg_o = opipe.Config(relaxed=mode, complete_intermediate=True)
    prop, batch, out, ref, _ = run_both(w, sp, cfg_g, cfg_o, op)
    compare_pass(out, batch, ref, op)
    assert ref["infeasible"].any() and not ref["infeasible"].all()


def test_pass_mnist_matches_oracle():
    w = wl.mnist_mlp(B=517)            # ragged: not a multiple of any tile
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts, op.unstable())
    prop, batch, out, ref, _ = run_both(w, sp, gpipe.PassConfig(), opipe.Config(), op)
    compare_pass(out, batch, ref, op)


def test_pass_biased_net_matches_oracle():
    w = wl.tiny_mlp(256)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 0, bias="uniform")
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts[:256], np.arange(w.net.n_hidden))
    prop, batch, out, ref, _ = run_both(w, sp, gpipe.PassConfig(complete_intermediate=True),
                                        opipe.Config(complete_intermediate=True), op)
    compare_pass(out, batch, ref, op)


def test_pass_sound_on_sampled_points_of_each_subdomain():
    w = wl.tiny_mlp(256)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 1, bias="uniform")
    rng = np.random.default_rng(wl.SEED_SAMPLES)
    anchors = rng.uniform(w.lo0, w.hi0, size=(256, 5))
    sp = wl.splits_from_points(w.net, anchors, w.split_counts[:256], np.arange(w.net.n_hidden))
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig(complete_intermediate=True))
    sync()
    assert not H(out["infeasible"]).any()
    x = np.concatenate([anchors[:, None], rng.uniform(w.lo0, w.hi0, (256, 3000, 5))], 1)
    z = wl.pre_activations(w.net, x.reshape(-1, 5)).reshape(256, -1, w.net.n_hidden)
    y = wl.forward(w.net, x.reshape(-1, 5)).reshape(256, -1, 5) @ w.C.T.astype(np.float64) + w.t
    lo, hi, l, u, lb = H(batch.lo), H(batch.hi), H(out["l"]), H(out["u"]), H(out["lb"])
    for b in range(256):
        k = sp.count[b]
        idx, sg = sp.neuron[b, :k], sp.sign[b, :k]
        feas = np.all(np.where(sg > 0, z[b][:, idx] >= 0, z[b][:, idx] <= 0), axis=1)
        assert feas[0]
        assert np.all(x[b][feas] >= lo[b]) and np.all(x[b][feas] <= hi[b])
        assert np.all(z[b][feas] >= l[b]) and np.all(z[b][feas] <= u[b])
        assert np.all(y[b][feas] >= lb[b])


# ------------------------------------------------------------------ slopes

def test_alpha_gradient_matches_oracle():
    # the bound and its slope gradient at random slopes, with the GPU's own
    # intermediate bounds handed to the oracle as data (and the oracle's own
    # clipped box and halfspaces, see test_gpu_sameinput): every gradient
    # entry within 1e-5 of the largest of its row
    w = wl.tiny_mlp(64)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 2, bias="uniform")
    op = OracleProp(w)
    sp = wl.draw_splits(64, w.split_counts[:64], np.arange(w.net.n_hidden))
    prop, batch, out, ref, _ = run_both(w, sp, gpipe.PassConfig(), opipe.Config(), op)
    alpha = wl.random_alpha(64, 5, w.net.n_hidden, seed=9)
    a_t = T(alpha)
    lb, grad = api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], a_t,
                              batch.lo, batch.hi, out["infeasible"], batch.splits, want_grad=True,
                              ws=prop.ws)
    sync()
    fe = ~ref["infeasible"] & ~H(out["infeasible"]).astype(bool)
    al = [alpha[:, :, o:o + n].astype(np.float64) for o, n in
          zip(w.net.hidden_offsets, w.net.hidden_sizes)]
    l_list = opipe.split_layers(op.layers, H(out["l"]).astype(np.float64))
    u_list = opipe.split_layers(op.layers, H(out["u"]).astype(np.float64))
    olb, ograds, _, _ = opipe.bound_and_grad(op.layers, w.C, w.t, l_list, u_list, al, ref["lo"],
                                            ref["hi"], ref["G"], ref["h"], ref["active"])
    assert_close(H(lb)[fe], olb[fe], 1e-5, "alpha-step bound")
    assert np.all(H(lb)[fe] <= olb[fe] + 1e-9 * np.maximum(np.abs(olb[fe]), 1.0))
    og = np.concatenate(ograds, axis=2)[fe]
    gg = H(grad)[fe]
    scale = np.abs(og).max(axis=2, keepdims=True) + 1e-30
    bad = np.abs(gg - og) > 1e-5 * scale
    assert not bad.any(), f"{bad.sum()} gradient entries differ"
    assert (og != 0).sum() > 100


def test_alpha_opt_matches_oracle_and_improves():
    # six slope iterations on the tiny net: the oracle on the GPU's float32
    # intermediate bounds, with its slopes and moments carried as float32
    # between iterations (as through the library's interface), within 1e-5;
    # on its own float64 bounds as well here (no discrete choice flips)
    w = wl.tiny_mlp(48)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 3, bias="uniform")
    op = OracleProp(w)
    sp = wl.draw_splits(48, w.split_counts[:48], np.arange(w.net.n_hidden))
    prop, batch, out, ref, _ = run_both(w, sp, gpipe.PassConfig(), opipe.Config(), op)
    best, _ = gpipe.alpha_opt(prop, batch, out["l"], out["u"], out["infeasible"], steps=6, lr=0.1)
    sync()
    fe = ~ref["infeasible"] & ~H(out["infeasible"]).astype(bool)
    g = H(best)[fe]
    assert np.all(g >= H(out["lb"])[fe] - 1e-6 * np.maximum(np.abs(g), 1))
    assert (g > H(out["lb"])[fe] + 1e-4).any()
    for l, u in ((H(out["l"])[fe].astype(np.float64), H(out["u"])[fe].astype(np.float64)),
                 (ref["l"][fe], ref["u"][fe])):
        obest, _, _ = opipe.alpha_opt(op.layers, w.C, w.t, opipe.split_layers(op.layers, l),
                                      opipe.split_layers(op.layers, u), ref["lo"][fe], ref["hi"][fe],
                                      ref["G"][fe], ref["h"][fe], ref["active"][fe], steps=6,
                                      state32=True, **ADAM)
        assert_close(g, obest, 1e-5, "alpha-opt best bound")


# ---------------------------------------------- full size, bench configuration

def test_full_size_mnist_sampled_rows():
    w = wl.mnist_mlp(B=16384)
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts, op.unstable())
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig())
    sync()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(w.B, 48, replace=False))
    ref = op.run(subset_splits(sp, idx))
    glb = H(out["lb"])[idx]
    assert_close(glb, ref["lb"], 1e-5, "lb (sampled rows)")
    assert_close(H(batch.lo)[idx], ref["lo"], 1e-5, "lo (sampled rows)")
    # +inf rows are exactly the infeasible subdomains
    ginf = H(out["infeasible"]).astype(bool)
    assert np.array_equal(np.isinf(H(out["lb"])).any(-1), ginf)
    assert np.isfinite(H(out["lb"])[~ginf]).all()


# --------------------------------------------------------------- edge cases

def test_edge_cases_empty_and_degenerate_inputs():
    w = wl.tiny_mlp(4)
    prop = gpipe.Property.from_workload(w)
    op = OracleProp(w)
    # B = 0 is a no-op everywhere
    z = torch.empty(0, 5, device="cuda")
    cons0 = api.Constraints.splits(np.zeros((0, 1), np.int32), np.zeros((0, 1), np.int8))
    api.clip_domains(prop.root, z, z.clone(), cons0)
    # unused slots (count 0, index -1) are ignored; kmax = 0 gives the plain bound
    neuron = np.array([[-1, -1], [3, -1], [0, 1], [5, 7]], np.int32)
    sign = np.array([[1, 1], [-1, 1], [1, -1], [1, 1]], np.int8)
    count = np.array([0, 1, 2, 2], np.int32)
    sp = wl.Splits(neuron, sign, count)
    batch = gpipe.make_batch(prop, neuron, sign, count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig())
    ref = op.run(wl.Splits(np.where(neuron < 0, 0, neuron), sign, count))
    sync()
    compare_pass(out, batch, ref, op)
    # the subdomain without splits gets the root bound
    batch0 = gpipe.make_batch(prop, neuron[:1], sign[:1], count[:1])
    out0 = gpipe.plain_pass(prop, batch0, gpipe.PassConfig(clip="none", complete_final=False))
    sync()
    assert_close(H(out0["lb"]), ref["lb"][:1], 1e-5, "no-split bound")


def test_invalid_arguments_are_rejected_before_launch():
    w = wl.tiny_mlp(4)
    prop = gpipe.Property.from_workload(w)
    from paper_2512_11087_amd import _native as N
    with pytest.raises(N.CvError) as e:
        api.Root(prop.net, w.lo0, w.hi0, alpha0=1.5)
    assert e.value.status == -1
    lo, hi = prop.boxes(2)
    l = torch.zeros(2, prop.net.n_hidden, device="cuda")
    lb = torch.empty(2, 5, device="cuda")
    import ctypes as C
    st = N.lib().cv_bound_propagate(prop.net.handle, 2, 5, api._p(prop.C), api._p(prop.t),
                                    api._p(l), api._p(l), None, C.c_float(0.5), api._p(lo),
                                    api._p(hi), None, prop.root.handle, None, None, 1, api._p(lb),
                                    None, None, None, C.c_size_t(0), api._stream())
    assert st == -4   # workspace too small
    st = N.lib().cv_clip_domains(prop.root.handle, None, 2, 5, None, api._p(lo), api._p(hi), None, 7,
                                 api._stream())
    assert st == -1


def test_autograd_bound_matches_adjoint_and_fused_adam():
    w = wl.tiny_mlp(64)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 2, bias="uniform")
    op = OracleProp(w)
    sp = wl.draw_splits(64, w.split_counts[:64], np.arange(w.net.n_hidden))
    prop, batch, out, ref, _ = run_both(w, sp, gpipe.PassConfig(), opipe.Config(), op)
    alpha = T(wl.random_alpha(64, 5, w.net.n_hidden, seed=9)).requires_grad_(True)
    lb = gpipe.bound(prop, batch, out["l"], out["u"], alpha, out["infeasible"])
    wts = T(np.random.default_rng(3).uniform(0.5, 2.0, (64, 5)))
    fe = T(1.0 - H(out["infeasible"]).astype(np.float32))[:, None]
    (torch.where(fe > 0, lb, torch.zeros_like(lb)) * wts).sum().backward()
    _, g = api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], alpha.detach(),
                          batch.lo, batch.hi, out["infeasible"], batch.splits, want_grad=True,
                          ws=prop.ws)
    sync()
    m = H(fe).astype(bool)[:, 0]
    assert np.allclose(H(alpha.grad)[m], (H(wts)[:, :, None] * H(g))[m], rtol=1e-6, atol=0)
    assert np.count_nonzero(H(alpha.grad)) > 100
    # torch's Adam (ascent, clamp to [0, 1]) through the autograd bound follows
    # the Adam step fused into the adjoint kernel
    a1 = alpha.detach().clone().requires_grad_(True)
    a2 = alpha.detach().clone()
    mm, vv = torch.zeros_like(a2), torch.zeros_like(a2)
    opt = torch.optim.Adam([a1], lr=0.1, betas=(0.9, 0.999), eps=1e-8, maximize=True)
    for s in range(1, 4):
        opt.zero_grad()
        gpipe.bound(prop, batch, out["l"], out["u"], a1, out["infeasible"]).sum().backward()
        opt.step()
        with torch.no_grad():
            a1.clamp_(0.0, 1.0)
        api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], a2, batch.lo,
                       batch.hi, out["infeasible"], batch.splits, 1, mm, vv, s, 0.1, ws=prop.ws)
    sync()
    assert np.abs(H(a1) - H(a2))[m].max() < 1e-4


def test_alpha_step_keeps_the_best_bound_and_starts_from_alpha_init():
    # the running best and the step-1 start live in the library: slopes,
    # moments and best filled with NaN are never read at step 1, and the
    # results equal those of pre-filled buffers with the best taken outside
    w = wl.tiny_mlp(64)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 2, bias="uniform")
    sp = wl.draw_splits(64, w.split_counts[:64], np.arange(w.net.n_hidden))
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig())
    B, M, nh = 64, prop.M, prop.net.n_hidden
    a1 = torch.full((B, M, nh), 0.5, device="cuda")
    m1, v1 = torch.zeros_like(a1), torch.zeros_like(a1)
    nan = float("nan")
    a2, m2, v2 = (torch.full_like(a1, nan) for _ in range(3))
    best = torch.full((B, M), nan, device="cuda")
    lbs = []
    for s in range(1, 6):
        lb, _ = api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], a1,
                               batch.lo, batch.hi, out["infeasible"], batch.splits, 1, m1, v1, s,
                               0.1, ws=prop.ws)
        lbs.append(H(lb))
        api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], a2, batch.lo,
                       batch.hi, out["infeasible"], batch.splits, 1, m2, v2, s, 0.1, ws=prop.ws,
                       alpha_init=0.5 if s == 1 else -1.0, best=best)
    sync()
    ref = np.max(np.stack(lbs), axis=0)
    assert np.array_equal(H(best), ref)
    assert np.array_equal(H(a1), H(a2)) and np.array_equal(H(m1), H(m2))
    inf = H(out["infeasible"]).astype(bool)
    assert inf.any() and np.isinf(H(best)[inf]).all()
    assert np.isfinite(H(best)[~inf]).all()
    # a start value at a later step is refused before launch
    from paper_2512_11087_amd import _native as N
    with pytest.raises(N.CvError) as e:
        api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], a2, batch.lo,
                       batch.hi, out["infeasible"], batch.splits, 1, m2, v2, 2, 0.1, ws=prop.ws,
                       alpha_init=0.5)
    assert e.value.status == -1


# ---------------------------------------------------- constraint importance order

def test_constraint_order_matches_oracle():
    B, n, k = 300, 37, 8
    lo, hi, G, h, count = wl.random_boxes_and_constraints(B, n, k, seed=31)
    cons = api.Constraints.dense(G, h, count)
    order = H(api.constraint_order(None, T(lo), T(hi), cons))
    sync()
    act = np.arange(k)[None] < count[:, None]
    ref = opipe.constraint_order(G.astype(np.float64), h.astype(np.float64), act, lo, hi)
    assert np.array_equal(order, ref)


@pytest.mark.parametrize("make", [lambda: wl.tiny_mlp(1024), lambda: wl.mnist_mlp(B=517)],
                         ids=["mlp5-50x6-5", "mlp784-256x6-10"])
def test_pass_with_constraint_order_matches_oracle(make):
    w = make()
    op = OracleProp(w)
    cand = np.arange(w.net.n_hidden) if w.net.n_in == 5 else op.unstable()
    sp = wl.draw_splits(w.B, w.split_counts, cand)
    cfg_g = gpipe.PassConfig(clip="sequential", complete_intermediate=w.net.n_in == 5, order=True)
    cfg_o = opipe.Config(relaxed="sequential", complete_intermediate=w.net.n_in == 5, order=True)
    prop, batch, out, ref, _ = run_both(w, sp, cfg_g, cfg_o, op)
    assert np.array_equal(H(out["order1"])[~ref["infeasible"]], ref["order"][~ref["infeasible"]])
    compare_pass(out, batch, ref, op)
    # the slope steps follow the same order
    best, _ = gpipe.alpha_opt(prop, batch, out["l"], out["u"], out["infeasible"], steps=3, lr=0.1)
    sync()
    fe = ~ref["infeasible"] & ~H(out["infeasible"]).astype(bool)
    l_list = opipe.split_layers(op.layers, ref["l"][fe])
    u_list = opipe.split_layers(op.layers, ref["u"][fe])
    obest, _, _ = opipe.alpha_opt(op.layers, w.C, w.t, l_list, u_list, ref["lo"][fe], ref["hi"][fe],
                                  ref["G"][fe], ref["h"][fe], ref["active"][fe], steps=3, state32=True, **ADAM)
    assert_close(H(best)[fe], obest, 1e-5, "alpha-opt with order")


# ------------------------------------------------------- conv layers (CNN)

@pytest.mark.parametrize("kernels", ["auto", "tiled"])
@pytest.mark.parametrize("make", [lambda: wl.cifar_cnn(B=64), lambda: wl.ragged_cnn(B=64),
                                  lambda: wl.wide_cnn(B=32), lambda: wl.edge_cnn(B=64)],
                         ids=["cnn3x32x32", "cnn5x9x7", "cnn4x24x24", "cnn3x7x7-edge"])
def test_pass_cnn_matches_oracle(make, kernels, monkeypatch):
    # backward passes and the adjoint run direct (transposed) convolutions.
    # 3x32x32 -> conv16 4x4/2 -> conv32 4x4/2 -> 100 -> 10: 3072-dim input
    # boxes take the workgroup-per-row complete clipping.  5x9x7 -> conv6
    # 3x3/1 -> conv17 4x4/3 -> 12 -> 4: ragged channel blocks, stride 3.
    # 4x24x24 -> conv16 3x3/1 -> conv8 4x4/2 -> 10 -> 3: rows of 9216 values
    # (over 64 KiB) take the tiled kernels.  3x7x7 -> conv4 1x1/2 ->
    # conv5 2x2/2 -> conv3 3x3/1 pad 2 -> 6 -> 3: positions without taps,
    # non-overlapping taps, padding wider than half the kernel.  "tiled":
    # every conv layer on the tiled kernels (band staging; matrix cores from
    # 16 output channels), which otherwise run only where a row exceeds LDS.
    if kernels == "tiled":
        monkeypatch.setenv("CV_CONV_TILED", "1")
    w = make()
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts, op.unstable())
    prop, batch, out, ref, _ = run_both(w, sp, gpipe.PassConfig(clip="sequential", order=True),
                                        opipe.Config(relaxed="sequential", order=True), op)
    compare_pass(out, batch, ref, op)
    fe = ~ref["infeasible"]
    assert (ref["lb"][fe] > ref["lb_unclipped"][fe] + 1e-6).any()   # clipping acts
    best, _ = gpipe.alpha_opt(prop, batch, out["l"], out["u"], out["infeasible"], steps=2, lr=0.1)
    sync()
    idx = np.nonzero(fe)[0][:16]
    l_list = opipe.split_layers(op.layers, ref["l"][idx])
    u_list = opipe.split_layers(op.layers, ref["u"][idx])
    obest, _, _ = opipe.alpha_opt(op.layers, w.C, w.t, l_list, u_list, ref["lo"][idx],
                                  ref["hi"][idx], ref["G"][idx], ref["h"][idx], ref["active"][idx],
                                  steps=2, state32=True, **ADAM)
    assert_close(H(best)[idx], obest, 1e-5, "cnn alpha-opt")


# ------------------------------------- top-k intermediate neurons (BaBSR score)

@pytest.mark.parametrize("make", [lambda: wl.tiny_mlp(256), lambda: wl.mnist_mlp(B=64)],
                         ids=["mlp5-50x6-5", "mlp784-256x6-10"])
def test_topk_complete_clipping_matches_oracle(make):
    w = make()
    op = OracleProp(w)
    tiny = w.net.n_in == 5
    cand = np.arange(w.net.n_hidden) if tiny else op.unstable()
    sp = wl.draw_splits(w.B, w.split_counts, cand)
    k = 5 if tiny else 20
    prop = gpipe.Property.from_workload(w)
    gw = H(prop.babsr_weight())
    ow = opipe.babsr_weights(op.layers, w.C, w.t, op.root)
    assert_close(gw, ow, 1e-5, "babsr weights")
    assert (ow > 0).sum() > 10
    cfg_g = gpipe.PassConfig(complete_intermediate=True, topk=k)
    cfg_o = opipe.Config(complete_intermediate=True, topk=k, babsr_weight=ow)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, cfg_g)
    sync()
    ref = op.run(sp, cfg=cfg_o)
    fe = ~ref["infeasible"] & ~H(out["infeasible"]).astype(bool)
    gsel = H(out["select"]).astype(bool)[fe]
    osel = ref["select"][fe]
    assert (gsel != osel).sum() <= max(2, osel.sum() // 1000), "selection differs"
    assert osel.sum(-1).max() <= k * (len(w.net.layers) - 1) and osel.any()
    compare_pass(out, batch, ref, op)


# ---------------------------------------------------------- branch and bound

def test_branching_kernels_match_oracle():
    from oracle import bab as obab
    rng = np.random.default_rng(21)
    B, Nh, n0, k = 200, 300, 17, 6
    l = rng.normal(size=(B, Nh)).astype(np.float32)
    u = (l + rng.uniform(0, 2, (B, Nh))).astype(np.float32)
    u[:3] = np.abs(u[:3]) + 1.0
    l[:3] = np.abs(l[:3]) + 0.1          # rows with nothing unstable
    weight = rng.uniform(0, 1, Nh).astype(np.float32)
    weight[::7] = 0.0
    neuron = rng.integers(0, Nh, (B, k)).astype(np.int32)
    sign = rng.choice([-1, 1], (B, k)).astype(np.int8)
    count = rng.integers(0, k, B).astype(np.int32)
    lo = rng.uniform(-1, 0, (B, n0)).astype(np.float32)
    hi = (lo + rng.uniform(0, 1, (B, n0))).astype(np.float32)
    # cv_branch_relu reads n_hidden / n_in from the root: a net of matching sizes
    net = wl.he_mlp([n0, Nh, 3], 0)
    p2 = gpipe.Property(list(net.layers), lo[0], hi[0], np.eye(3, dtype=np.float32),
                        np.zeros(3, np.float32))
    cons = api.Constraints.splits(neuron, sign, count)
    chosen, ccons, lo2, hi2 = api.branch_relu(p2.root, T(l), T(u), T(weight), cons, T(lo), T(hi), k + 1)
    sync()
    ref = obab.branch_relu(l, u, weight, neuron, sign, count)
    assert np.array_equal(H(chosen), ref)
    n2, s2, c2, olo2, ohi2 = obab.children_relu(neuron, sign, count, lo, hi, ref)
    assert np.array_equal(H(ccons.count), c2)
    for r in range(2 * B):
        assert np.array_equal(H(ccons.neuron)[r, :c2[r]], n2[r, :c2[r]])
        assert np.array_equal(H(ccons.sign)[r, :c2[r]], s2[r, :c2[r]])
    assert np.array_equal(H(lo2), olo2) and np.array_equal(H(hi2), ohi2)
    A = rng.normal(size=(B, 2, n0)).astype(np.float32)
    dim, ilo2, ihi2 = api.branch_input(T(lo), T(hi), T(A))
    sync()
    rd = obab.branch_input(lo, hi, A)
    assert np.array_equal(H(dim), rd)
    rlo2, rhi2 = obab.children_input(lo, hi, rd)
    assert np.array_equal(H(ilo2), rlo2) and np.array_equal(H(ihi2), rhi2)


def _tiny_property(row, frac):
    """One output row of the tiny net, y_row >= thr, with thr = L + frac (m - L)
    where L is the root CROWN bound and m the minimum over 2e5 samples:
    0 < frac < 1 gives a true property the root bound cannot verify, frac > 1
    a false one (the sampled minimum violates it)."""
    w = wl.tiny_mlp(8)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 1, bias="uniform")
    x = np.random.default_rng(wl.SEED_SAMPLES).uniform(w.lo0, w.hi0, size=(200000, 5))
    m = wl.forward(w.net, x)[:, row].min()
    C = np.zeros((1, 5), np.float32)
    C[0, row] = 1.0
    prop = gpipe.Property(list(w.net.layers), w.lo0, w.hi0, C, np.zeros(1, np.float32))
    L = float(H(gpipe.plain_pass(prop, gpipe.Batch(*prop.boxes(1), None))["lb"])[0, 0])
    thr = L + frac * (m - L)
    prop = gpipe.Property(list(w.net.layers), w.lo0, w.hi0, C, np.array([-thr], np.float32))
    return w, prop, thr


@pytest.mark.parametrize("loop", ["activation", "input"])
def test_bab_verifies_a_true_property_and_never_a_false_one(loop):
    from paper_2512_11087_amd import bab
    run = bab.activation_bab if loop == "activation" else bab.input_bab
    w, prop, thr = _tiny_property(0, 0.3)
    base = gpipe.plain_pass(prop, gpipe.Batch(*prop.boxes(1), None))
    sync()
    assert float(H(base["lb"]).min()) <= 0.0, "root bound already verifies: not a BaB test"
    res = run(prop, batch=8192, max_iters=300)
    assert res.verified, res
    assert res.iterations >= 1 and res.visited > 1
    x = np.random.default_rng(99).uniform(w.lo0, w.hi0, size=(100000, 5))
    assert wl.forward(w.net, x)[:, 0].min() >= thr     # the verified claim holds at samples
    w, prop, thr = _tiny_property(0, 1.02)
    res = run(prop, batch=512, max_iters=15)
    assert not res.verified


def test_input_pass_matches_oracle():
    # fresh sub-boxes of the tiny net's root box with one dense plane constraint
    # each: relaxed clipping, CROWN intermediate bounds over the box, final bound
    # with complete clipping against the plane
    w = wl.tiny_mlp(8)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 1, bias="uniform")
    op = OracleProp(w)
    rng = np.random.default_rng(17)
    B = 96
    a = rng.uniform(w.lo0, w.hi0, size=(B, 5))
    b = rng.uniform(w.lo0, w.hi0, size=(B, 5))
    lo, hi = np.minimum(a, b).astype(np.float32), np.maximum(a, b).astype(np.float32)
    G = rng.normal(size=(B, 1, 5)).astype(np.float32)
    xs = rng.uniform(lo, hi)
    h = (-(G[:, 0] * xs).sum(-1, keepdims=True) + rng.normal(0, 0.05, (B, 1))).astype(np.float32)
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.Batch(T(lo), T(hi), api.Constraints.dense(G, h))
    out = gpipe.input_pass(prop, batch)
    sync()
    ref = opipe.run(op.layers, op.root, w.C, w.t, lo, hi, None, None, None,
                    opipe.Config(intermediate="crown"), dense=(G, h, np.ones((B, 1), bool)))
    compare_pass(out, batch, ref, op)
    assert ref["infeasible"].any() and (ref["lb"][~ref["infeasible"]] >
                                        ref["lb_unclipped"][~ref["infeasible"]] + 1e-6).any()


def test_step_graph_replays_match_eager():
    # the whole step (box reset, plain pass, slope iterations) captured once,
    # replayed several times with eager work in between: the eager step's
    # boxes, intermediate bounds, plain bound and best bound every time
    w = wl.mnist_mlp(B=160)
    prop = gpipe.Property.from_workload(w)
    l0, u0 = (H(x) for x in prop.root.bounds())
    cand = np.nonzero((l0 < 0) & (u0 > 0))[0]
    sp = wl.draw_splits(w.B, w.split_counts, cand)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    lo0, hi0 = batch.lo.clone(), batch.hi.clone()
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig())
    best_e, _ = gpipe.alpha_opt(prop, batch, out["l"], out["u"], out["infeasible"], steps=5,
                                lr=0.1)
    ref = [H(x).copy() for x in (batch.lo, batch.hi, out["l"], out["u"], out["lb"],
                                 out["infeasible"], best_e)]
    g = gpipe.StepGraph(prop, batch, lo0, hi0, steps=5, lr=0.1)
    for rep in range(3):
        o, best = g.run()
        sync()
        got = [H(x).copy() for x in (batch.lo, batch.hi, o["l"], o["u"], o["lb"], o["infeasible"],
                                     best)]
        for a, b, name in zip(ref, got, ("lo", "hi", "l", "u", "lb", "infeasible", "best")):
            assert np.array_equal(a, b), f"replay {rep}: {name}"
        # unrelated eager work between replays, on other buffers
        b2 = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
        gpipe.alpha_opt(prop, b2, out["l"], out["u"], out["infeasible"], steps=2, lr=0.3)
        sync()


def test_alpha_opt_graph_replays_match_eager():
    # the captured slope optimisation, replayed several times with eager work
    # in between, gives the eager result bit for bit every time
    w = wl.tiny_mlp(128)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 3, bias="uniform")
    sp = wl.draw_splits(128, w.split_counts[:128], np.arange(w.net.n_hidden))
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig())
    eager, alpha_e = gpipe.alpha_opt(prop, batch, out["l"], out["u"], out["infeasible"], steps=6,
                                     lr=0.1)
    eager = H(eager).copy()
    alpha_e = H(alpha_e).copy()
    g = gpipe.AlphaOptGraph(prop, batch, out["l"], out["u"], out["infeasible"], steps=6, lr=0.1)
    for rep in range(3):
        best = H(g.run()).copy()
        sync()
        assert np.array_equal(best, eager), f"replay {rep}"
        assert np.array_equal(H(g.alpha), alpha_e), f"replay {rep} alpha"
        # unrelated eager work between replays
        gpipe.plain_pass(prop, gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count),
                         gpipe.PassConfig())
        sync()
