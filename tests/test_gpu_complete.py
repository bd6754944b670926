"""Complete clipping on the GPU (Thm 3.1, coordinate ascent of eq. 4) where
the choice among maximisers matters, and over several passes.

* Ties: relaxed clipping followed by complete clipping with the same
  constraints (flat dual segments), duplicated constraints and tied
  breakpoints (``workloads.tie_problems``).  The kernel resolves a near-tie
  with its own tolerance, so its multipliers are judged on their own: the
  oracle takes them as data and checks, constraint by constraint in the
  kernel's order, that each one maximises its 1-D dual up to that tolerance
  and is the smallest such point, and that D at them is the kernel's bound.
  Separately the bound is compared with the oracle's own pipeline (float64
  relaxed clipping, then coordinate ascent with the oracle's float64 tie
  rule), which takes the decisions exact arithmetic takes.
* Several passes (passes = 2, 3) through cv_concretize (wave and workgroup
  teams), cv_concretize_planes (complete clipping of intermediate neurons)
  and cv_bound_propagate (final rows), against ``coord_ascent(passes=...)``.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import box, complete, pipeline as opipe, relaxed  # noqa: E402
from paper_2512_11087_amd import api, pipeline as gpipe, workloads as wl  # noqa: E402
from helpers import OracleProp, assert_close, check_multipliers  # noqa: E402

pytestmark = pytest.mark.gpu


def T(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dtype)


def H(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n", [200, 2000], ids=["wave-team", "workgroup-team"])
def test_ties_after_relaxed_clipping_take_valid_smallest_multipliers(n):
    B, P, k = 64, 3, 3
    lo, hi, G, h, count, A, c = wl.tie_problems(B, n, k, P, seed=71 + n)
    lo_t, hi_t = T(lo), T(hi)
    cons = api.Constraints.dense(G, h, count)
    inf = api.clip_domains(None, lo_t, hi_t, cons, "parallel")
    lb, _, beta = api.concretize(T(A), T(c), lo_t, hi_t, cons, want_beta=True, infeasible=inf)
    torch.cuda.synchronize()
    act = np.ones((B, k), bool)
    rep = lambda x: np.repeat(x, P, axis=0)
    # the oracle's own pipeline on the same float32 inputs
    olo, ohi, oinf0 = relaxed.clip_parallel(G, h, lo, hi, act)
    L, obeta, oinf1 = complete.coord_ascent(A.reshape(B * P, n), c.reshape(B * P), rep(G), rep(h),
                                            rep(olo), rep(ohi), rep(act))
    L = np.maximum(L.reshape(B, P), box.concretize_min(A, c, olo, ohi))
    oinf = oinf0 | oinf1.reshape(B, P).any(-1)
    ginf = H(inf).astype(bool)
    assert not (ginf & ~oinf).any(), "GPU pruned a subdomain the oracle keeps"
    fe = ~oinf & ~ginf
    assert fe.sum() >= B // 3
    g = H(lb)
    sc = (np.abs(A) * np.maximum(np.abs(lo), np.abs(hi))[:, None, :]).sum(-1) + np.abs(c) + 1.0
    assert np.all(g[fe] <= L[fe] + 1e-9 * sc[fe]), "complete clip above the oracle's bound"
    assert_close(g[fe], L[fe], 1e-5, "bound vs the oracle's pipeline")
    # the same candidates as the oracle (up to the float32 rounding of beta)
    gb = H(beta).reshape(B, P, k)[fe]
    ob = obeta.reshape(B, P, k)[fe]
    assert np.all(np.abs(gb - ob) <= 2.0 ** -21 * np.abs(ob) + 1e-30), "different multipliers"
    # the kernel's multipliers judged on the kernel's own (float32) box
    glo, ghi = H(lo_t), H(hi_t)
    stats = check_multipliers(A[fe].reshape(-1, n), c[fe].reshape(-1),
                              np.repeat(G[fe], P, 0), np.repeat(h[fe], P, 0),
                              np.repeat(glo[fe], P, 0), np.repeat(ghi[fe], P, 0),
                              gb.reshape(-1, k), g[fe].reshape(-1))
    # the inputs do make ties: flat segments at the chosen multiplier
    # (constraint 0) and duplicated constraints whose slope at 0+ is zero
    assert stats["flat"] >= 10 and stats["flat_at_zero"] >= 5, stats
    print(f"n={n}: {fe.sum()} feasible subdomains, {stats}")


@pytest.mark.parametrize("passes", [1, 2, 3])
@pytest.mark.parametrize("n", [5, 784, 3072], ids=["n5", "n784-wave", "n3072-workgroup"])
def test_concretize_passes_match_oracle(n, passes):
    B, P, k = 61, 3, 5
    lo, hi, G, h, count = wl.random_boxes_and_constraints(B, n, k, seed=90 + n, slack=0.2)
    A, c = wl.random_planes(B, P, n, seed=91 + n)
    cons = api.Constraints.dense(G, h, count)
    inf = torch.zeros(B, dtype=torch.uint8, device="cuda")
    lbc, _, beta = api.concretize(T(A), T(c), T(lo), T(hi), cons, passes=passes, want_beta=True,
                                  infeasible=inf)
    torch.cuda.synchronize()
    act = np.arange(k)[None, :] < count[:, None]
    rep = lambda x: np.repeat(x, P, axis=0)
    L, obeta, oinf = complete.coord_ascent(A.reshape(B * P, n), c.reshape(B * P), rep(G), rep(h),
                                           rep(lo), rep(hi), rep(act), passes=passes)
    olb = box.concretize_min(A, c, lo, hi)
    L = np.maximum(L.reshape(B, P), olb)
    oinf = oinf.reshape(B, P).any(-1)
    assert np.array_equal(H(inf).astype(bool), oinf)
    fe = ~oinf
    g = H(lbc)
    sc = (np.abs(A) * np.maximum(np.abs(lo), np.abs(hi))[:, None, :]).sum(-1) + np.abs(c)
    assert np.all(g[fe] <= L[fe] + 1e-9 * np.maximum(sc[fe], 1.0)), "above the oracle"
    assert_close(g[fe], L[fe], 1e-5, f"complete clip, {passes} passes")
    assert (L[fe] > olb[fe] + 1e-6).any()
    keep = np.repeat(fe, P)
    assert_close(H(beta).reshape(B * P, k)[keep], obeta[keep], 1e-5, "beta")
    if passes > 1:      # a later pass moved some multiplier
        L1, b1, _ = complete.coord_ascent(A.reshape(B * P, n), c.reshape(B * P), rep(G), rep(h),
                                          rep(lo), rep(hi), rep(act), passes=1)
        assert (np.abs(b1[keep] - obeta[keep]) > 1e-6).any()


@pytest.mark.parametrize("passes", [2, 3])
def test_pass_with_several_ca_passes_matches_oracle(passes):
    # complete clipping of intermediate neurons (cv_concretize_planes) and of
    # the final rows (cv_bound_propagate), both with `passes` passes
    from test_gpu_parity import compare_pass
    w = wl.tiny_mlp(512)
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts[:512], np.arange(w.net.n_hidden))
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig(complete_intermediate=True, passes=passes))
    torch.cuda.synchronize()
    ref = op.run(sp, cfg=opipe.Config(complete_intermediate=True, ca_passes=passes))
    compare_pass(out, batch, ref, op)
    one = op.run(sp, cfg=opipe.Config(complete_intermediate=True, ca_passes=1))
    fe = ~ref["infeasible"]
    assert (ref["lb"][fe] > one["lb"][fe] + 1e-7).any(), "more passes changed nothing"


def test_mnist_pass_with_two_ca_passes_matches_oracle():
    from test_gpu_parity import compare_pass
    w = wl.mnist_mlp(B=301)
    op = OracleProp(w)
    sp = wl.draw_splits(w.B, w.split_counts, op.unstable())
    prop = gpipe.Property.from_workload(w)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig(passes=2))
    torch.cuda.synchronize()
    ref = op.run(sp, cfg=opipe.Config(ca_passes=2))
    compare_pass(out, batch, ref, op)
