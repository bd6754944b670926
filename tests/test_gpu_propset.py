"""Batching of several properties (a RootSet and a per-subdomain property
index): each subdomain's results must equal the oracle run of its own
property, whether the subdomains are grouped by property or interleaved,
and equal what the same calls give on each property alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import pipeline as opipe  # noqa: E402
from paper_2512_11087_amd import api, pipeline as gpipe, workloads as wl  # noqa: E402
from helpers import ADAM, OracleProp, assert_close  # noqa: E402

pytestmark = pytest.mark.gpu


def T(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dtype)


def H(t):
    return t.detach().cpu().numpy()


def sync():
    torch.cuda.synchronize()


def _setup(ws, order_seed=None, k=4):
    """GPU property set, oracle per property, split lists per property over
    its own root-unstable neurons; subdomains grouped by property, or
    permuted (order_seed)."""
    ps = gpipe.PropertySet(list(ws.net.layers), ws.lo0s, ws.hi0s, ws.Cs, ws.ts)
    ops = [OracleProp(ws.member(p)) for p in range(ws.P)]
    sps = [wl.draw_splits(int(ws.counts[p]), np.minimum(ws.member(p).split_counts, k),
                          ops[p].unstable(), seed=30 + p, kmax=k) for p in range(ws.P)]
    neuron = np.concatenate([s.neuron for s in sps])
    sign = np.concatenate([s.sign for s in sps])
    count = np.concatenate([s.count for s in sps])
    pid = ws.pid()
    lo = np.concatenate([np.broadcast_to(ws.lo0s[p], (int(ws.counts[p]), ws.net.n_in))
                         for p in range(ws.P)])
    hi = np.concatenate([np.broadcast_to(ws.hi0s[p], (int(ws.counts[p]), ws.net.n_in))
                         for p in range(ws.P)])
    perm = np.arange(ws.B)
    if order_seed is not None:
        perm = np.random.default_rng(order_seed).permutation(ws.B)
    batch = gpipe.Batch(T(lo[perm]), T(hi[perm]),
                        api.Constraints.splits(neuron[perm], sign[perm], count[perm]),
                        pid=T(pid[perm], torch.int32))
    return ps, ops, sps, perm, batch


def _rows_of(ws, perm, p):
    """Positions in the (permuted) batch of property p's subdomains, in the
    property's own order."""
    start = int(ws.counts[:p].sum())
    inv = np.argsort(perm)
    return inv[start:start + int(ws.counts[p])]


@pytest.mark.parametrize("order_seed", [None, 7], ids=["grouped", "interleaved"])
def test_property_set_pass_matches_oracle_per_property(order_seed):
    # 4 properties of uneven size; the first 64-row tile of the plane GEMM
    # holds 3 of them
    ws = wl.mnist_mlp_set([37, 1, 70, 12])
    ps, ops, sps, perm, batch = _setup(ws, order_seed)
    gw = H(ps.babsr_weight())
    cfg_g = gpipe.PassConfig(clip="sequential", order=True, complete_intermediate=True, topk=10)
    out = gpipe.plain_pass(ps, batch, cfg_g)
    best, _ = gpipe.alpha_opt(ps, batch, out["l"], out["u"], out["infeasible"], steps=3, lr=0.1)
    sync()
    ginf = H(out["infeasible"]).astype(bool)
    for p in range(ws.P):
        op, w = ops[p], ws.member(p)
        ow = opipe.babsr_weights(op.layers, w.C, w.t, op.root)
        assert_close(gw[p], ow, 1e-5, f"babsr weights of property {p}")
        cfg_o = opipe.Config(relaxed="sequential", order=True, complete_intermediate=True, topk=10,
                             babsr_weight=ow)
        ref = op.run(sps[p], cfg=cfg_o)
        rows = _rows_of(ws, perm, p)
        gi = ginf[rows]
        assert not (gi & ~ref["infeasible"]).any(), f"property {p}: GPU pruned a subdomain"
        fe = ~ref["infeasible"] & ~gi
        assert_close(H(batch.lo)[rows][fe], ref["lo"][fe], 1e-5, f"lo of property {p}")
        assert_close(H(batch.hi)[rows][fe], ref["hi"][fe], 1e-5, f"hi of property {p}")
        unst = op.unstable()
        assert_close(H(out["l"])[rows][fe][:, unst], ref["l"][fe][:, unst], 1e-5, f"l of {p}")
        assert_close(H(out["u"])[rows][fe][:, unst], ref["u"][fe][:, unst], 1e-5, f"u of {p}")
        assert_close(H(out["lb"])[rows][fe], ref["lb"][fe], 1e-5, f"lb of property {p}")
        # slope optimisation, on a few subdomains of the property
        idx = np.nonzero(fe)[0][:6]
        if idx.size == 0:
            continue
        l_list = opipe.split_layers(op.layers, ref["l"][idx])
        u_list = opipe.split_layers(op.layers, ref["u"][idx])
        obest, _, _ = opipe.alpha_opt(op.layers, w.C, w.t, l_list, u_list, ref["lo"][idx],
                                      ref["hi"][idx], ref["G"][idx], ref["h"][idx],
                                      ref["active"][idx], steps=3, state32=True, **ADAM)
        assert_close(H(best)[rows][idx], obest, 1e-5, f"alpha-opt of property {p}")


def test_property_set_equals_single_property_calls():
    # the same kernels on a set and on each property alone: identical results
    ws = wl.mnist_mlp_set([20, 45, 9])
    ps, ops, sps, perm, batch = _setup(ws, order_seed=3)
    out = gpipe.plain_pass(ps, batch, gpipe.PassConfig())
    lbs, _ = api.alpha_step(ps.net, ps.root, ps.C, ps.t, out["l"], out["u"],
                            torch.full((ws.B, ps.M, ps.net.n_hidden), 0.3, device="cuda"),
                            batch.lo, batch.hi, out["infeasible"], batch.cons(), want_grad=True,
                            ws=ps.ws, pid=batch.pid)
    sync()
    for p in range(ws.P):
        rows = _rows_of(ws, perm, p)
        single = gpipe.Property(list(ws.net.layers), ws.lo0s[p], ws.hi0s[p], ws.Cs[p], ws.ts[p])
        b1 = gpipe.make_batch(single, sps[p].neuron, sps[p].sign, sps[p].count)
        o1 = gpipe.plain_pass(single, b1, gpipe.PassConfig())
        l1, _ = api.alpha_step(single.net, single.root, single.C, single.t, o1["l"], o1["u"],
                               torch.full((len(rows), single.M, single.net.n_hidden), 0.3,
                                          device="cuda"),
                               b1.lo, b1.hi, o1["infeasible"], b1.cons(), want_grad=True,
                               ws=single.ws)
        sync()
        assert np.array_equal(H(out["lb"])[rows], H(o1["lb"])), f"plain bound of property {p}"
        assert np.array_equal(H(out["l"])[rows], H(o1["l"])), f"intermediate bounds of {p}"
        assert np.array_equal(H(batch.lo)[rows], H(b1.lo)), f"clipped boxes of {p}"
        assert np.array_equal(H(lbs)[rows], H(l1)), f"alpha-step bound of property {p}"
    # branching reads each subdomain's row of the per-property weights
    weight = ps.babsr_weight()
    chosen, ccons, _, _ = api.branch_relu(ps.root, out["l"], out["u"], weight, batch.splits,
                                          batch.lo, batch.hi, 8, pid=batch.pid)
    sync()
    for p in range(ws.P):
        rows = _rows_of(ws, perm, p)
        wp = weight[p].contiguous()
        c1, _, _, _ = api.branch_relu(ps.roots[p], out["l"][rows].contiguous(),
                                      out["u"][rows].contiguous(), wp,
                                      api.Constraints.splits(sps[p].neuron, sps[p].sign,
                                                             sps[p].count),
                                      batch.lo[rows].contiguous(), batch.hi[rows].contiguous(), 8)
        sync()
        assert np.array_equal(H(chosen)[rows], H(c1)), f"branching of property {p}"


def test_property_set_cnn_matches_oracle_per_property():
    # conv layers, 3 properties of the CIFAR CNN (complete clipping of the
    # 3072-dimensional final planes), interleaved
    ws = wl.cifar_cnn_set(counts=[9, 3, 14])
    ps, ops, sps, perm, batch = _setup(ws, order_seed=11, k=6)
    out = gpipe.plain_pass(ps, batch, gpipe.PassConfig())
    sync()
    ginf = H(out["infeasible"]).astype(bool)
    for p in range(ws.P):
        op = ops[p]
        ref = op.run(sps[p])
        rows = _rows_of(ws, perm, p)
        fe = ~ref["infeasible"] & ~ginf[rows]
        assert not (ginf[rows] & ~ref["infeasible"]).any()
        assert_close(H(out["lb"])[rows][fe], ref["lb"][fe], 1e-5, f"cnn lb of property {p}")


def test_set_of_one_property_equals_its_root():
    # a set of one takes the single-property launch paths (the host copy of
    # its table entry): the same results as the root alone
    ws = wl.mnist_mlp_set([23])
    ps, ops, sps, perm, batch = _setup(ws)
    out = gpipe.plain_pass(ps, batch, gpipe.PassConfig())
    best, _ = gpipe.alpha_opt(ps, batch, out["l"], out["u"], out["infeasible"], steps=2, lr=0.1)
    single = gpipe.Property(list(ws.net.layers), ws.lo0s[0], ws.hi0s[0], ws.Cs[0], ws.ts[0])
    b1 = gpipe.make_batch(single, sps[0].neuron, sps[0].sign, sps[0].count)
    o1 = gpipe.plain_pass(single, b1, gpipe.PassConfig())
    best1, _ = gpipe.alpha_opt(single, b1, o1["l"], o1["u"], o1["infeasible"], steps=2, lr=0.1)
    sync()
    assert ps.P == 1
    assert np.array_equal(H(out["lb"]), H(o1["lb"]))
    assert np.array_equal(H(out["l"]), H(o1["l"]))
    assert np.array_equal(H(best), H(best1))


def test_property_set_step_graph_replays_match_eager():
    # many properties through one captured graph: the whole step (box reset,
    # plain pass, slope iterations) over a 3-property set, replayed, equals
    # the eager step bit for bit
    ws = wl.mnist_mlp_set([30, 7, 19])
    ps, ops, sps, perm, batch = _setup(ws, order_seed=9)
    lo0, hi0 = batch.lo.clone(), batch.hi.clone()
    out = gpipe.plain_pass(ps, batch, gpipe.PassConfig())
    best_e, _ = gpipe.alpha_opt(ps, batch, out["l"], out["u"], out["infeasible"], steps=4, lr=0.1)
    ref = [H(x).copy() for x in (batch.lo, out["l"], out["lb"], best_e)]
    g = gpipe.StepGraph(ps, batch, lo0, hi0, steps=4, lr=0.1)
    for rep in range(2):
        o, best = g.run()
        sync()
        got = [H(x).copy() for x in (batch.lo, o["l"], o["lb"], best)]
        for a, b, name in zip(ref, got, ("lo", "l", "lb", "best")):
            assert np.array_equal(a, b), f"replay {rep}: {name}"


def test_rootset_rejects_single_root_queries():
    ws = wl.mnist_mlp_set([2, 2])
    ps = gpipe.PropertySet(list(ws.net.layers), ws.lo0s, ws.hi0s, ws.Cs, ws.ts)
    from paper_2512_11087_amd import _native as N
    import ctypes as C
    cnt = C.c_int()
    assert N.lib().cv_root_count(ps.root.handle, C.byref(cnt)) == 0 and cnt.value == 2
    assert N.lib().cv_root_unstable_count(ps.root.handle, C.byref(cnt)) == -1
    lo, hi, pid = ps.boxes([2, 2])
    l = torch.zeros(4, ps.net.n_hidden, device="cuda")
    with pytest.raises(N.CvError) as e:
        api.intermediate_bounds(ps.net, ps.root, lo, hi, l, l.clone())
    assert e.value.status == -3
    # a set of sets is refused
    arr = (C.c_void_p * 1)(ps.root.handle.value)
    out = C.c_void_p()
    assert N.lib().cv_rootset_create(arr, 1, C.byref(out)) == -1


def _tiny_set(specs):
    """Properties y_row >= thr of the tiny net over its root box, one per
    (row, frac): thr = L + frac (m - L), L the root CROWN bound of the row and
    m its minimum over 2e5 samples (frac < 1 true but not verified at the
    root, frac > 1 false)."""
    w = wl.tiny_mlp(8)
    w.net = wl.he_mlp([5] + [50] * 6 + [5], 1, bias="uniform")
    x = np.random.default_rng(wl.SEED_SAMPLES).uniform(w.lo0, w.hi0, size=(200000, 5))
    y = wl.forward(w.net, x)
    Cs, ts = [], []
    for row, frac in specs:
        C = np.zeros((1, 5), np.float32)
        C[0, row] = 1.0
        p1 = gpipe.Property(list(w.net.layers), w.lo0, w.hi0, C, np.zeros(1, np.float32))
        L = float(H(gpipe.plain_pass(p1, gpipe.Batch(*p1.boxes(1), None))["lb"])[0, 0])
        thr = L + frac * (y[:, row].min() - L)
        Cs.append(C)
        ts.append(np.array([-thr], np.float32))
    n = len(specs)
    return gpipe.PropertySet(list(w.net.layers), [w.lo0] * n, [w.hi0] * n, Cs, ts)


def test_activation_bab_over_a_property_set():
    from paper_2512_11087_amd import bab
    # two true properties (rows 0 and 2), bounded in one pool
    ps = _tiny_set([(0, 0.3), (2, 0.3)])
    res = bab.activation_bab(ps, batch=8192, max_iters=300)
    assert res.verified and res.per_property == [True, True], res
    assert res.iterations >= 1
    # a false property among true ones is never reported verified
    ps = _tiny_set([(0, 0.3), (0, 1.02), (2, 0.3)])
    res = bab.activation_bab(ps, batch=512, max_iters=12)
    assert not res.verified and res.per_property[1] is False, res
