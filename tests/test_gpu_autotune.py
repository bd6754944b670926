"""Kernel variants (GEMM tiles, convolution staging depth and positions
per lane) and the autotuner that picks among them: every variant of every
layer must give bit-identical bounds, gradients and slope updates, so tuning
never changes a result."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2512_11087_amd import api, pipeline as gpipe, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


def H(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("make", [lambda: wl.mnist_mlp(B=96), lambda: wl.ragged_cnn(B=40),
                                  lambda: wl.small_conv4_set().member(0),
                                  lambda: wl.edge_cnn(B=40)],
                         ids=["mlp784-256x6-10", "cnn5x9x7", "cnn3x8x8-4xc8", "cnn3x7x7-edge"])
@pytest.mark.parametrize("kernels", ["auto", "tiled"])
def test_every_kernel_variant_gives_identical_results(make, kernels, monkeypatch):
    if kernels == "tiled":   # conv layers on the tiled kernels (no effect on the MLP)
        monkeypatch.setenv("CV_CONV_TILED", "1")
    w = make()
    prop = gpipe.Property.from_workload(w)
    l0, u0 = (H(x) for x in prop.root.bounds())
    cand = np.nonzero((l0 < 0) & (u0 > 0))[0]
    sp = wl.draw_splits(w.B, np.minimum(w.split_counts, 4), cand, kmax=4)
    batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
    out = gpipe.plain_pass(prop, batch, gpipe.PassConfig())
    shape = (w.B, prop.M, prop.net.n_hidden)

    def run():
        alpha = torch.full(shape, 0.4, device="cuda")
        m = torch.zeros_like(alpha)
        v = torch.zeros_like(alpha)
        lb, grad = api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"], alpha,
                                  batch.lo, batch.hi, out["infeasible"], batch.cons(), 1, m, v, 1,
                                  0.1, want_grad=True, ws=prop.ws)
        # a second step reads the slopes and Adam's moments (the GEMM
        # epilogue's form for the steps after the first)
        lb_s2, grad_s2 = api.alpha_step(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"],
                                        alpha, batch.lo, batch.hi, out["infeasible"], batch.cons(),
                                        1, m, v, 2, 0.1, want_grad=True, ws=prop.ws)
        lb2, A, c = api.bound_propagate(prop.net, prop.root, prop.C, prop.t, out["l"], out["u"],
                                        batch.lo, batch.hi, infeasible=out["infeasible"],
                                        cons=batch.cons(), want_plane=True, ws=prop.ws)
        torch.cuda.synchronize()
        return [H(x) for x in (lb, grad, lb_s2, grad_s2, alpha, m, v, lb2, A, c)]

    ref = run()
    assert np.isfinite(ref[0]).any()
    tuning = prop.net.tuning()
    assert tuning, "no tunable layer"
    tried = 0
    for (kind, layer), (v0, count) in tuning.items():
        assert v0 == 0
        for v in range(1, count):
            prop.net.set_tuning(kind, layer, v)
            got = run()
            for a, b in zip(ref, got):
                assert np.array_equal(a, b, equal_nan=True), (kind, layer, v)
            tried += 1
        prop.net.set_tuning(kind, layer, 0)
    assert tried >= 4
    with pytest.raises(Exception):
        prop.net.set_tuning("relax", 1, 0)        # layer 1 has no relax step
    t = prop.net.autotune(w.B, prop.M)
    assert all(0 <= v < c for v, c in t.values())
    for a, b in zip(ref, run()):
        assert np.array_equal(a, b, equal_nan=True)
