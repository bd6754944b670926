"""Pins the oracle to the worked 2-D toy example of the appendix (every value
the paper prints), in exact rational arithmetic where it matters."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import box, complete, crown, exact, relaxed

HERE = os.path.dirname(__file__)
G = json.load(open(os.path.join(HERE, "golden", "toy_2d.json")))
V = {k: v["value"] for k, v in G["values"].items()}
W1 = np.array(G["network"]["W1"], float)
b1 = np.array(G["network"]["b1"], float)
w2 = np.array([G["network"]["w2"]], float)
lo = np.array(G["box"]["lo"], float)
hi = np.array(G["box"]["hi"], float)
LAYERS = [(W1, b1), (w2, np.zeros(1))]


def fr(s):
    return float(Fraction(s))


def test_prebounds():
    l = box.concretize_min(W1[None], b1[None], lo[None], hi[None])[0]
    u = box.concretize_max(W1[None], b1[None], lo[None], hi[None])[0]
    assert list(l) == [fr(s) for s in V["z_lower"]]
    assert list(u) == [fr(s) for s in V["z_upper"]]
    # the centre/radius form of the paper agrees
    xh = np.array(G["box"]["centre"], float)
    eps = np.array(G["box"]["radius"], float)
    assert np.allclose(W1 @ xh - np.abs(W1) @ eps + b1, l)


def test_crown_bound_alpha_one():
    root = crown.root_pass(LAYERS, lo, hi, alpha0=1.0)
    A, c = crown.backward(LAYERS, np.eye(1), np.zeros(1), [root.l[0][None]], [root.u[0][None]], 1.0)
    lb = box.concretize_min(A, c, lo[None], hi[None])[0, 0]
    assert lb == pytest.approx(fr(V["crown_lb"]), abs=1e-14)


def test_relaxed_clip_values():
    nl, nh, inf = relaxed.clip_single_literal(W1[0], b1[0], lo, hi)
    assert not inf
    assert nh[0] == pytest.approx(fr(V["x_clip"][0]))
    assert nl[1] == pytest.approx(fr(V["x_clip"][1]))
    assert np.allclose(nl, [fr(s) for s in V["clipped_lo"]])
    assert np.allclose(nh, [fr(s) for s in V["clipped_hi"]])
    pl, ph, pinf = relaxed.clip_parallel(W1[None, :1], b1[None, :1], lo[None], hi[None])
    assert np.allclose(pl[0], nl) and np.allclose(ph[0], nh) and not pinf[0]


def test_reconcretized_bounds_and_bound_after_clipping():
    nl = np.array([fr(s) for s in V["clipped_lo"]])
    nh = np.array([fr(s) for s in V["clipped_hi"]])
    l = box.concretize_min(W1[None], b1[None], nl[None], nh[None])
    u = box.concretize_max(W1[None], b1[None], nl[None], nh[None])
    assert np.allclose(l[0], [fr(s) for s in V["z_lower_rc"]])
    assert np.allclose(u[0], [fr(s) for s in V["z_upper_rc"]])
    A, c = crown.backward(LAYERS, np.eye(1), np.zeros(1), [l], [u], 1.0)
    assert box.concretize_min(A, c, nl[None], nh[None])[0, 0] == pytest.approx(fr(V["crown_lb_rc"]))


def test_complete_clip_upper_z2():
    # max z2 s.t. z1 <= 0  ==  -min(-z2)
    L, beta = complete.single_enum(-W1[1], -b1[1], W1[0], b1[0], lo, hi)
    assert -L == pytest.approx(fr(V["z2_upper_cc"]))
    assert beta == pytest.approx(fr(V["beta_star_z2"]))
    Ls, bs, inf = complete.single_max(-W1[1][None], -b1[1:2], W1[0][None], b1[0:1], lo[None], hi[None])
    assert -Ls[0] == pytest.approx(fr(V["z2_upper_cc"])) and bs[0] == pytest.approx(5.0)
    assert exact.lp_simplex(-W1[1], -b1[1], W1[0:1], b1[0:1], lo, hi) == -Fraction(V["z2_upper_cc"])


def test_complete_clip_upper_z1():
    L, _ = complete.single_enum(-W1[0], -b1[0], W1[0], b1[0], lo, hi)
    assert -L == pytest.approx(fr(V["z1_upper_cc"]), abs=1e-12)


def test_dual_subgradients_per_segment():
    # slopes of the convex dual printed in the paper are the negated slopes of
    # the concave dual D(beta) of min(-z2); measure them on each segment.
    d = lambda b: float(complete.dual_value(-W1[1], -b1[1], W1[0], b1[0], lo, hi, np.float64(b)))
    pts = [(0.0, 1.0 / 7.0), (1.0 / 7.0, 5.0), (5.0, 7.0)]
    slopes = [-(d(b - 1e-3) - d(a + 1e-3)) / (b - a - 2e-3) for a, b in pts]
    assert np.allclose(slopes, [fr(s) for s in V["subgradients_z2"]], atol=1e-9)
