"""Full-size parity at the 3x32x32 CNN with four 64-channel convolutions
(102912 hidden neurons): properties 0 and 255 of the 256-property set
against FP64 oracle values computed by ``tests/golden/make_conv64_golden.py``
(only ``oracle/`` and the seeded generators; see that script for the
recipe).  Root bounds of 512 sampled neurons per property, then 8 subdomains
per property (the stored splits) bounded in one call of the property set:
the plain bound within 1e-5 and not above the oracle's, the clipped boxes,
and the best bound after 10 slope iterations against the oracle's own run
(its own float64 intermediate bounds: held to the band of the slope tests,
1e-4)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2512_11087_amd import pipeline as gpipe, workloads as wl  # noqa: E402
from helpers import assert_close  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "conv64_props0_255.npz")


def H(t):
    return t.detach().cpu().numpy()


def test_conv64_full_size_against_oracle_values():
    g = np.load(GOLDEN)
    props = [int(p) for p in g["props"]]
    ws = wl.cifar_conv64_set(256)
    ps = gpipe.PropertySet(list(ws.net.layers), [ws.lo0s[p] for p in props],
                           [ws.hi0s[p] for p in props], [ws.Cs[p] for p in props],
                           [ws.ts[p] for p in props])
    # root bounds of sampled neurons
    for j, p in enumerate(props):
        l0, u0 = (H(x) for x in ps.roots[j].bounds())
        s = g[f"p{p}_root_sample"]
        ol, ou = g[f"p{p}_root_l"], g[f"p{p}_root_u"]
        assert_close(l0[s], ol, 1e-5, f"root l, property {p}")
        assert_close(u0[s], ou, 1e-5, f"root u, property {p}")
        assert np.all(l0[s] <= ol + 1e-9 * np.maximum(np.abs(ol), 1.0))
        assert np.all(u0[s] >= ou - 1e-9 * np.maximum(np.abs(ou), 1.0))
        # the GPU's root-unstable set contains the oracle's (its bounds are outward)
        assert ps.roots[j].n_unstable >= int(g[f"p{p}_n_unstable"])
        assert ps.roots[j].n_unstable <= int(g[f"p{p}_n_unstable"]) + 8
    # the stored subdomains of both properties in one batch
    n = int(g["n_sub"])
    neuron = np.concatenate([g[f"p{p}_neuron"] for p in props])
    sign = np.concatenate([g[f"p{p}_sign"] for p in props])
    count = np.concatenate([g[f"p{p}_count"] for p in props])
    lo, hi, pid = ps.boxes([n] * len(props))
    batch = gpipe.make_batch(ps, neuron, sign, count, lo, hi, pid)
    res = gpipe.chunked_verify(ps, batch, 0, steps=int(g["steps"]), lr=0.1)
    torch.cuda.synchronize()
    lb, best, inf = H(res["lb"]), H(res["best"]), H(res["infeasible"]).astype(bool)
    olb = np.concatenate([g[f"p{p}_lb"] for p in props])
    obest = np.concatenate([g[f"p{p}_best"] for p in props])
    oinf = np.concatenate([g[f"p{p}_infeasible"] for p in props])
    assert np.array_equal(inf, oinf)
    fe = ~oinf
    assert fe.sum() >= n
    e0 = assert_close(lb[fe], olb[fe], 1e-5, "plain bound")
    assert np.all(lb[fe] <= olb[fe] + 1e-9 * np.maximum(np.abs(olb[fe]), 1.0)), "above the oracle"
    glo, ghi = H(batch.lo).astype(np.float64), H(batch.hi).astype(np.float64)
    olo = np.concatenate([g[f"p{p}_lo_sum"] for p in props])
    ohi = np.concatenate([g[f"p{p}_hi_sum"] for p in props])
    assert_close(glo.sum(-1)[fe], olo[fe], 1e-6, "clipped box (lo digest)")
    assert_close(ghi.sum(-1)[fe], ohi[fe], 1e-6, "clipped box (hi digest)")
    e1 = np.abs(best[fe] - obest[fe]) / np.maximum(np.abs(obest[fe]), 1.0)
    print(f"conv64 properties {props}: plain bound max rel err {e0:.2e}; after "
          f"{int(g['steps'])} slope steps max {e1.max():.2e}, median {np.median(e1):.2e}; "
          f"mean gain {np.mean(best[fe] - lb[fe]):.3f}")
    assert e1.max() <= 1e-4
    assert np.all(best[fe] >= lb[fe] - 1e-6 * np.maximum(np.abs(lb[fe]), 1.0))
