"""The four-convolution CIFAR network (3x32x32 -> four 64-channel 3x3
convolutions -> 512 -> 10) batched over many properties: conv layers kept as
kernels only, roots that keep the planes of their unstable neurons only,
and batches bounded in chunks.

At the small size of the same layer pattern every subdomain is compared
with the oracle.  At full size the oracle's root pass is out of reach on the
CPU (its dense matrices alone pass 10 GB), so the full-size test pins the
root bounds of all layer-1 and sampled layer-2 neurons against the oracle,
checks that the unstable-only roots and the chunked schedule reproduce the
all-planes, one-call results bit for bit, and checks soundness at points of
the subdomains."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import box as obox, crown, pipeline as opipe  # noqa: E402
from paper_2512_11087_amd import api, pipeline as gpipe, workloads as wl  # noqa: E402
from helpers import ADAM, OracleProp, assert_close  # noqa: E402

pytestmark = pytest.mark.gpu


def T(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dtype)


def H(t):
    return t.detach().cpu().numpy()


def sync():
    torch.cuda.synchronize()


def _set_batch(ps, ws, sps, perm=None):
    lo, hi, pid = ps.boxes(ws.counts)
    neuron = np.concatenate([s.neuron for s in sps])
    sign = np.concatenate([s.sign for s in sps])
    count = np.concatenate([s.count for s in sps])
    if perm is None:
        perm = np.arange(ws.B)
    return gpipe.Batch(lo[T(perm, torch.int64)].contiguous(), hi[T(perm, torch.int64)].contiguous(),
                       api.Constraints.splits(neuron[perm], sign[perm], count[perm]),
                       pid=pid[T(perm, torch.int64)].contiguous())


def test_small_conv4_set_unstable_planes_match_oracle():
    # 3 properties, 48 subdomains (Zipf counts 28/12/8), interleaved; roots
    # keep the unstable neurons' planes only (splits are drawn over those)
    ws = wl.small_conv4_set()
    layers = list(ws.net.layers)
    ps = gpipe.PropertySet(layers, ws.lo0s, ws.hi0s, ws.Cs, ws.ts, planes="unstable")
    ops = [OracleProp(ws.member(p)) for p in range(ws.P)]
    k = int(ws.split_counts.max())
    sps = [wl.draw_splits(int(ws.counts[p]), ws.member(p).split_counts, ops[p].unstable(),
                          seed=40 + p, kmax=k) for p in range(ws.P)]
    perm = np.random.default_rng(5).permutation(ws.B)
    inv = np.argsort(perm)
    batch = _set_batch(ps, ws, sps, perm)
    # planes are not readable from an unstable-only root
    with pytest.raises(Exception):
        ps.roots[0].planes()
    out = gpipe.plain_pass(ps, batch, gpipe.PassConfig())
    best, _ = gpipe.alpha_opt(ps, batch, out["l"], out["u"], out["infeasible"], steps=3, lr=0.1)
    sync()
    ginf = H(out["infeasible"]).astype(bool)
    for p in range(ws.P):
        op, w = ops[p], ws.member(p)
        ref = op.run(sps[p])
        start = int(ws.counts[:p].sum())
        rows = inv[start:start + int(ws.counts[p])]
        assert not (ginf[rows] & ~ref["infeasible"]).any(), f"property {p}: GPU pruned a subdomain"
        fe = ~ref["infeasible"] & ~ginf[rows]
        assert_close(H(batch.lo)[rows][fe], ref["lo"][fe], 1e-5, f"lo of property {p}")
        assert_close(H(batch.hi)[rows][fe], ref["hi"][fe], 1e-5, f"hi of property {p}")
        un = op.unstable()
        assert_close(H(out["l"])[rows][fe][:, un], ref["l"][fe][:, un], 1e-5, f"l of {p}")
        assert_close(H(out["u"])[rows][fe][:, un], ref["u"][fe][:, un], 1e-5, f"u of {p}")
        assert_close(H(out["lb"])[rows][fe], ref["lb"][fe], 1e-5, f"lb of property {p}")
        idx = np.nonzero(fe)[0][:5]
        if idx.size == 0:
            continue
        l_list = opipe.split_layers(op.layers, ref["l"][idx])
        u_list = opipe.split_layers(op.layers, ref["u"][idx])
        obest, _, _ = opipe.alpha_opt(op.layers, w.C, w.t, l_list, u_list, ref["lo"][idx],
                                      ref["hi"][idx], ref["G"][idx], ref["h"][idx],
                                      ref["active"][idx], steps=3, state32=True, **ADAM)
        assert_close(H(best)[rows][idx], obest, 1e-5, f"alpha-opt of property {p}")

    # the same set with every plane kept, and the chunked schedule (chunks
    # of 7 subdomains, ragged tail): identical results
    ps_all = gpipe.PropertySet(layers, ws.lo0s, ws.hi0s, ws.Cs, ws.ts, planes="all", net=ps.net)
    b_all = _set_batch(ps_all, ws, sps, perm)
    o_all = gpipe.plain_pass(ps_all, b_all, gpipe.PassConfig())
    best_all, _ = gpipe.alpha_opt(ps_all, b_all, o_all["l"], o_all["u"], o_all["infeasible"],
                                  steps=3, lr=0.1)
    b_ch = _set_batch(ps, ws, sps, perm)
    res = gpipe.chunked_verify(ps, b_ch, 7, steps=3, lr=0.1)
    sync()
    assert np.array_equal(H(o_all["lb"]), H(out["lb"]))
    assert np.array_equal(H(best_all), H(best))
    assert np.array_equal(H(res["lb"]), H(out["lb"]))
    assert np.array_equal(H(res["best"]), H(best))
    assert np.array_equal(H(res["infeasible"]), H(out["infeasible"]))
    assert np.array_equal(H(b_ch.lo), H(batch.lo))


def test_unstable_planes_ignore_splits_of_stable_neurons():
    # a root that keeps only its unstable neurons' planes drops a split on a
    # root-stable neuron (no plane to clip with): the result is the oracle's
    # for the same subdomains without those splits (intermediate-bound fixes
    # of the split neuron still apply, as they need no plane)
    ws = wl.small_conv4_set(P=1, B=40)
    w = ws.member(0)
    op = OracleProp(w)
    prop = gpipe.Property(list(w.net.layers), w.lo0, w.hi0, w.C, w.t, planes="unstable")
    un = op.unstable()
    stable = np.setdiff1d(np.arange(w.net.n_hidden), un)
    sp = wl.draw_splits(w.B, np.minimum(w.split_counts, 4), un, seed=77, kmax=5)
    # append one stable-neuron split (with the sign of its fixed regime, so
    # the subdomain stays non-empty) to every subdomain
    rng = np.random.default_rng(78)
    for b in range(w.B):
        j = int(rng.choice(stable))
        k = int(sp.count[b])
        sp.neuron[b, k] = j
        sp.sign[b, k] = 1 if op.l0[j] >= 0 else -1
        sp.count[b] = k + 1
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig())
    sync()
    ref = op.run(sp)            # every split, the stable ones included
    keep = sp.neuron.copy()     # the same lists without the stable-neuron splits
    cnt = sp.count.copy()
    for b in range(w.B):
        k = int(cnt[b]) - 1
        keep[b, k] = -1
        cnt[b] = k
    ref_drop = op.run(wl.Splits(keep, sp.sign, cnt))
    fe = ~ref_drop["infeasible"]
    assert not (H(out["infeasible"]).astype(bool) & ~ref_drop["infeasible"]).any()
    assert_close(H(batch.lo)[fe], ref_drop["lo"][fe], 1e-5, "lo without the stable splits")
    assert_close(H(out["lb"])[fe], ref_drop["lb"][fe], 1e-5, "lb without the stable splits")
    # a stable neuron's split in its own regime clips nothing either way
    assert_close(ref["lb"][fe], ref_drop["lb"][fe], 1e-9, "oracle: the regime split is redundant")
    # and a root keeping every plane (which applies those splits) gives the
    # same GPU results bit for bit
    prop_all = gpipe.Property(list(w.net.layers), w.lo0, w.hi0, w.C, w.t, planes="all")
    b_all = gpipe.make_batch(prop_all, sp.neuron, sp.sign, sp.count)
    o_all = gpipe.plain_pass(prop_all, b_all, gpipe.PassConfig())
    sync()
    assert np.array_equal(H(o_all["lb"]), H(out["lb"]))
    assert np.array_equal(H(b_all.lo), H(batch.lo)) and np.array_equal(H(b_all.hi), H(batch.hi))
    assert np.array_equal(H(o_all["infeasible"]), H(out["infeasible"]))


def test_full_size_conv64_roots_chunks_and_soundness():
    ws = wl.cifar_conv64_set(256)
    net = ws.net
    sizes = net.hidden_sizes
    n1, n2 = sizes[0], sizes[1]
    assert sizes == [65536, 16384, 16384, 4096, 512] and net.n_hidden == 102912
    sel = [0, 255]                      # the largest and a smallest property
    n_pt, n_rand = 100, 1000            # property 0: 100 subdomains around points, 1000 random
    counts = [n_pt + n_rand, int(ws.counts[255])]
    lo0s, hi0s = [ws.lo0s[p] for p in sel], [ws.hi0s[p] for p in sel]
    Cs, ts = [ws.Cs[p] for p in sel], [ws.ts[p] for p in sel]
    ps = gpipe.PropertySet(list(net.layers), lo0s, hi0s, Cs, ts)   # auto: unstable planes
    sync()
    with pytest.raises(Exception):
        ps.roots[0].planes()
    # size limits: one call takes at most 2^31 / 102912 rows (2318 subdomains
    # of 9 rows); beyond, the workspace query and the call refuse (no launch)
    from paper_2512_11087_amd import _native as N
    import ctypes as C
    assert ps.net.max_batch(9) == (2 ** 31 - 1) // (9 * 102912)
    n = C.c_size_t()
    assert N.lib().cv_alpha_step_workspace(ps.net.handle, 2, 4096, 9, C.byref(n)) == -3
    assert N.lib().cv_bound_propagate_workspace(ps.net.handle, 2, 2318, 9, C.byref(n)) == 0
    # an unknown plane mode is refused
    h = C.c_void_p()
    assert N.lib().cv_root_create_ex(ps.net.handle, api._p(ps.roots[0].lo0), api._p(ps.roots[0].hi0),
                                     C.c_float(0.5), 7, None, C.byref(h)) == -1

    # root bounds: every layer-1 neuron and 24 layer-2 neurons of each
    # property against the oracle (layer 2: CROWN with objective e_j over
    # the first two layers, alpha 0.5, from the oracle's own layer-1 bounds)
    ly = net.layers
    W1 = crown.conv_matrix(ly[0].W, ly[0].stride, ly[0].pad, ly[0].in_shape, ly[0].out_shape)
    b1 = crown.conv_bias(ly[0].b, ly[0].out_shape)
    W2 = crown.conv_matrix(ly[1].W, ly[1].stride, ly[1].pad, ly[1].in_shape, ly[1].out_shape)
    b2 = crown.conv_bias(ly[1].b, ly[1].out_shape)
    rng = np.random.default_rng(17)
    for j, root in enumerate(ps.roots):
        l0, u0 = (H(x) for x in root.bounds())
        lo, hi = lo0s[j].astype(np.float64)[None], hi0s[j].astype(np.float64)[None]
        ol1 = obox.concretize_min(W1[None], b1[None], lo, hi)[0]
        ou1 = obox.concretize_max(W1[None], b1[None], lo, hi)[0]
        assert_close(l0[:n1], ol1, 1e-5, f"layer-1 lower bounds, property {sel[j]}")
        assert_close(u0[:n1], ou1, 1e-5, f"layer-1 upper bounds, property {sel[j]}")
        assert np.all(l0[:n1] <= ol1 + 1e-6 * np.maximum(1, abs(ol1)))
        js = np.sort(rng.choice(n2, 24, replace=False))
        cut = [(W1, b1), (W2[js], b2[js])]
        I = np.eye(js.size)
        A, c = crown.backward(cut, I, np.zeros(js.size), [ol1[None]], [ou1[None]], 0.5)
        An, cn = crown.backward(cut, -I, np.zeros(js.size), [ol1[None]], [ou1[None]], 0.5)
        ol2 = obox.concretize_min(A, c, lo, hi)[0]
        ou2 = -obox.concretize_min(An, cn, lo, hi)[0]
        assert_close(l0[n1 + js], ol2, 1e-5, f"layer-2 lower bounds, property {sel[j]}")
        assert_close(u0[n1 + js], ou2, 1e-5, f"layer-2 upper bounds, property {sel[j]}")
    del W1, W2

    # subdomains: property 0's first 100 around random points of its box
    # (the splits follow each point's activation pattern, so the point is
    # feasible), the rest random splits over each property's unstable neurons
    k = 12
    sps = []
    for j, root in enumerate(ps.roots):
        l0, u0 = (H(x) for x in root.bounds())
        cand = np.nonzero((l0 < 0) & (u0 > 0))[0]
        depth = rng.integers(1, k + 1, size=counts[j]).astype(np.int32)
        sp = wl.draw_splits(counts[j], depth, cand, seed=60 + j, kmax=k)
        if j == 0:
            x = rng.uniform(lo0s[0], hi0s[0], size=(n_pt, 3072)).astype(np.float32)
            spx = wl.splits_from_points(net, x, depth[:n_pt], cand, seed=70, kmax=k)
            sp.neuron[:n_pt], sp.sign[:n_pt], sp.count[:n_pt] = spx.neuron, spx.sign, spx.count
        sps.append(sp)
    two = wl.WorkloadSet("two", net, lo0s, hi0s, Cs, ts, np.asarray(counts), np.zeros(0))
    batch = _set_batch(ps, two, sps)
    res = gpipe.chunked_verify(ps, batch, 512, steps=10, lr=0.1)   # chunks 512, 512, 87
    sync()
    lb, best, inf = H(res["lb"]), H(res["best"]), H(res["infeasible"]).astype(bool)
    # soundness at the points: margin C f(x) + t >= bound
    fx = wl.forward(net, x)
    marg = fx @ Cs[0].astype(np.float64).T + ts[0].astype(np.float64)
    assert not inf[:n_pt].any(), "a subdomain with a feasible point was pruned"
    assert np.all(lb[:n_pt] <= marg + 1e-6), "plain bound above the margin at a feasible point"
    assert np.all(best[:n_pt] <= marg + 1e-6), "alpha bound above the margin at a feasible point"
    fe = ~inf
    assert np.all(best[fe] >= lb[fe]), "the slope iterations lost the plain bound"
    assert np.mean(best[fe] - lb[fe]) > 0.0

    # property 255 alone, every plane kept, one call: identical to its rows
    single = gpipe.PropertySet(list(net.layers), lo0s[1:], hi0s[1:], Cs[1:], ts[1:], planes="all",
                               net=ps.net)
    wsingle = wl.WorkloadSet("one", net, lo0s[1:], hi0s[1:], Cs[1:], ts[1:],
                             np.asarray(counts[1:]), np.zeros(0))
    b1_ = _set_batch(single, wsingle, sps[1:])
    o1 = gpipe.plain_pass(single, b1_, gpipe.PassConfig())
    best1, _ = gpipe.alpha_opt(single, b1_, o1["l"], o1["u"], o1["infeasible"], steps=10, lr=0.1)
    sync()
    rows = np.arange(counts[0], counts[0] + counts[1])
    assert np.array_equal(H(o1["lb"]), lb[rows])
    assert np.array_equal(H(best1), best[rows])
    assert np.array_equal(H(b1_.lo), H(batch.lo)[rows])
