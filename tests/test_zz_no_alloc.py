"""The allocation-free entry point cv_concretize_planes_static (scratch in the
library's static per-device array) against cv_concretize_planes (caller
workspace): bit for bit on two calls in a row, the second with a smaller
batch, with and without complete clipping and top-k selection; and its size
limit, refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2512_11087_amd import _native as N, api, pipeline as gpipe, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


def H(t):
    return t.detach().cpu().numpy()


def test_static_scratch_variant_matches_the_workspace_variant():
    w = wl.mnist_mlp(B=1024)
    prop = gpipe.Property.from_workload(w)
    l0, u0 = (H(x) for x in prop.root.bounds())
    cand = np.nonzero((l0 < 0) & (u0 > 0))[0]
    sp = wl.draw_splits(w.B, w.split_counts, cand)
    weight = prop.babsr_weight()
    ws = api.Workspace()
    nh = prop.net.n_hidden
    for B in (1024, 333):                      # two calls in a row, the second smaller
        batch = gpipe.make_batch(prop, sp.neuron[:B], sp.sign[:B], sp.count[:B])
        api.clip_domains(prop.root, batch.lo, batch.hi, batch.splits)
        for complete, topk in ((True, -1), (True, 16), (False, -1)):
            outs = []
            for fn in ("workspace", "static"):
                inf = torch.zeros(B, dtype=torch.uint8, device="cuda")
                sel = torch.full((B, nh), 7, dtype=torch.uint8, device="cuda")
                kw = dict(infeasible=inf, topk=topk, weight=weight if topk >= 0 else None,
                          select=sel if topk >= 0 else None)
                if fn == "workspace":
                    l, u, inf = api.concretize_planes(prop.root, batch.lo, batch.hi, batch.splits,
                                                      complete, 1, ws=ws, **kw)
                else:
                    l, u, inf = api.concretize_planes_static(prop.root, batch.lo, batch.hi,
                                                             batch.splits, complete, 1, **kw)
                torch.cuda.synchronize()
                outs.append((H(l), H(u), H(inf), H(sel)))
            (l1, u1, i1, s1), (l2, u2, i2, s2) = outs
            tag = f"B={B} complete={complete} topk={topk}"
            assert np.array_equal(l1, l2) and np.array_equal(u1, u2), tag
            assert np.array_equal(i1, i2), tag
            if topk >= 0:
                assert np.array_equal(s1, s2) and (s1 == 1).any(), tag
            if complete:   # the clipping did tighten something (the scratch was used)
                l_plain, u_plain, _ = api.concretize_planes(prop.root, batch.lo, batch.hi,
                                                            batch.splits, False, 1)
                torch.cuda.synchronize()
                assert (l2 > H(l_plain)).any() or (u2 < H(u_plain)).any(), tag


def test_static_scratch_variant_refuses_a_batch_beyond_its_array():
    w = wl.mnist_mlp(B=4)
    prop = gpipe.Property.from_workload(w)
    lib = N.lib()
    need = C.c_size_t()
    B = 1
    while True:   # the smallest batch whose scratch exceeds the array
        assert lib.cv_concretize_planes_workspace(prop.root.handle, B, 1, C.byref(need)) == 0
        if need.value > (64 << 20):
            break
        B *= 2
    # refused before any pointer is read or anything enqueued
    st = lib.cv_concretize_planes_static(prop.root.handle, None, B, None, None, None, 1, 1, -1,
                                         None, None, None, None, None, api._stream())
    assert st == -4
    assert lib.cv_status_string(st) == b"workspace too small"
    # without complete clipping no scratch is needed, so any batch passes the
    # size check (and fails only on the missing pointers)
    st = lib.cv_concretize_planes_static(prop.root.handle, None, B, None, None, None, 0, 1, -1,
                                         None, None, None, None, None, api._stream())
    assert st == -1
