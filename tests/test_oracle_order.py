"""Pins the constraint importance order (heuristics appendix) to geometry:
the key is the Euclidean distance from the box centre to each constraint's
hyperplane, ascending; and checks that coordinate ascent in that order is
still a valid dual bound (below the exact LP optimum)."""
from fractions import Fraction

import numpy as np

from oracle import complete, exact, pipeline


def test_hand_example_order():
    # box [0, 2]^2, centre (1, 1)
    lo = np.array([[0.0, 0.0]])
    hi = np.array([[2.0, 2.0]])
    G = np.array([[[1.0, 0.0],      # x1 - 1.5 <= 0        distance 0.5
                   [1.0, 1.0],      # x1 + x2 - 5 <= 0     distance 3/sqrt(2)
                   [0.0, -1.0],     # -x2 + 0.9 <= 0       distance 0.1
                   [0.0, 0.0],      # no hyperplane: last
                   [3.0, 4.0]]])    # 3 x1 + 4 x2 - 7.5 <= 0: distance 0.1, after index 2
    h = np.array([[-1.5, -5.0, 0.9, -1.0, -7.5]])
    act = np.array([[True, True, True, True, True]])
    assert pipeline.constraint_order(G, h, act, lo, hi).tolist() == [[2, 4, 0, 1, 3]]
    # inactive slots go last, in list order
    act2 = np.array([[True, True, False, True, True]])
    assert pipeline.constraint_order(G, h, act2, lo, hi).tolist() == [[4, 0, 1, 2, 3]]


def test_order_follows_projection_distance():
    rng = np.random.default_rng(0)
    B, k, n = 40, 7, 6
    lo = rng.uniform(-1, 1, (B, n))
    hi = lo + rng.uniform(0, 1, (B, n))
    G = rng.normal(size=(B, k, n))
    h = rng.normal(size=(B, k)) * 2
    act = np.arange(k)[None] < rng.integers(1, k + 1, B)[:, None]
    order = pipeline.constraint_order(G, h, act, lo, hi)
    xc = 0.5 * (lo + hi)
    for b in range(B):
        dist = []
        for kk in order[b]:
            if not act[b, kk]:
                dist.append(np.inf)
                continue
            g = G[b, kk]
            # foot of the perpendicular from the centre onto g.x + h = 0
            xp = xc[b] - (g @ xc[b] + h[b, kk]) * g / (g @ g)
            assert abs(g @ xp + h[b, kk]) < 1e-9 * (1 + np.abs(g) @ np.abs(xp))
            # no sampled point of the hyperplane is closer than the foot
            v = rng.normal(size=(50, n))
            v -= np.outer(v @ g / (g @ g), g)
            assert np.all(np.linalg.norm(xp + v - xc[b], axis=1) >= np.linalg.norm(xp - xc[b]) - 1e-12)
            dist.append(np.linalg.norm(xp - xc[b]))
        dist = np.array(dist)
        assert np.all(np.diff(dist[np.isfinite(dist)]) >= -1e-12)
        assert sorted(order[b].tolist()) == list(range(k))


def test_ordered_coordinate_ascent_is_valid_and_can_differ():
    rng = np.random.default_rng(1)
    differ = 0
    for trial in range(60):
        n, k = 4, 3
        lo = rng.uniform(-1, 0, n)
        hi = rng.uniform(0, 1, n)
        a = rng.normal(size=n)
        G = rng.normal(size=(k, n))
        xs = rng.uniform(lo, hi)
        h = -(G @ xs) - rng.uniform(0.0, 0.3, k)     # xs is feasible
        act = np.ones((1, k), bool)
        order = pipeline.constraint_order(G[None], h[None], act, lo[None], hi[None])
        Go, ho, acto = pipeline.apply_order(order, G[None], h[None], act)
        L0, _, e0 = complete.coord_ascent(a[None], np.zeros(1), G[None], h[None], lo[None], hi[None], act)
        L1, _, e1 = complete.coord_ascent(a[None], np.zeros(1), Go, ho, lo[None], hi[None], acto)
        assert not e0[0] and not e1[0]
        lp = float(exact.lp_simplex(a, 0.0, G, h, lo, hi))
        assert L0[0] <= lp + 1e-9 and L1[0] <= lp + 1e-9
        differ += abs(L1[0] - L0[0]) > 1e-9
    assert differ > 0
