"""Pins the clipping oracle (relaxed and complete) to the exact LP optimum,
computed by vertex enumeration and by a rational simplex, and to the
closed-form and knapsack restatements, on small random problems with the
degenerate cases the method has (zero coefficients, zero-width coordinates,
tied breakpoints, redundant and infeasible constraints)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import box, complete, exact, relaxed


def rand_problem(rng, n, m, degenerate=True):
    lo = rng.uniform(-1, 1, n)
    hi = lo + rng.uniform(0.05, 1.5, n)
    a = rng.normal(size=n)
    G = rng.normal(size=(m, n))
    xs = rng.uniform(lo, hi)            # keep most constraints feasible
    h = -(G @ xs) + rng.normal(0, 0.7, m)
    if degenerate:
        if rng.random() < 0.3:
            G[rng.integers(m), rng.integers(n)] = 0.0
        if rng.random() < 0.2:
            j = rng.integers(n)
            hi[j] = lo[j]
        if rng.random() < 0.2 and n >= 2:   # tied breakpoints
            G[0, 1] = G[0, 0]
            a[1] = a[0]
        if rng.random() < 0.1:
            a[rng.integers(n)] = 0.0
    return a, 0.3, G, h, lo, hi


def test_concretize_is_corner_minimum():
    rng = np.random.default_rng(10)
    for _ in range(40):
        n = rng.integers(1, 8)
        a = rng.normal(size=n)
        lo = rng.uniform(-2, 1, n)
        hi = lo + rng.uniform(0, 2, n)
        v = box.concretize_min(a[None], np.array([0.7]), lo, hi)[0]
        assert v == pytest.approx(exact.box_corners_min(a, 0.7, lo, hi), abs=1e-12)
        assert box.concretize_min_centre(a[None], np.array([0.7]), lo, hi)[0] == pytest.approx(v, abs=1e-12)
        vmax = box.concretize_max(a[None], np.array([0.7]), lo, hi)[0]
        assert vmax == pytest.approx(-exact.box_corners_min(-a, -0.7, lo, hi), abs=1e-12)


def test_shared_matmul_form_equals_elementwise_form():
    rng = np.random.default_rng(11)
    A = rng.normal(size=(7, 9))
    c = rng.normal(size=7)
    lo = rng.uniform(-1, 0, (5, 9))
    hi = lo + rng.uniform(0, 1, (5, 9))
    assert np.allclose(box.concretize_min_shared(A, c, lo, hi),
                       box.concretize_min(A[None], c[None], lo, hi), atol=1e-12)
    assert np.allclose(box.concretize_max_shared(A, c, lo, hi),
                       box.concretize_max(A[None], c[None], lo, hi), atol=1e-12)


def test_relaxed_single_literal_equals_fast_and_is_the_exact_lp_box():
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(60):
        n = int(rng.integers(1, 6))
        a, c, G, h, lo, hi = rand_problem(rng, n, 1)
        nl, nh, inf = relaxed.clip_single_literal(G[0], h[0], lo, hi)
        pl, ph, pinf = relaxed.clip_parallel(G[None], h[None], lo[None], hi[None])
        assert inf == bool(pinf[0])
        lp_empty = exact.lp_vertices(np.zeros(n), 0.0, G, h, lo, hi)[0] == np.inf
        assert inf == lp_empty
        if inf:
            continue
        assert np.allclose(nl, pl[0], atol=1e-12) and np.allclose(nh, ph[0], atol=1e-12)
        # Thm 3.2: the clipped box is the tightest box around box ∩ halfspace
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            xmin = exact.lp_vertices(e, 0.0, G, h, lo, hi)[0]
            xmax = -exact.lp_vertices(-e, 0.0, G, h, lo, hi)[0]
            assert nl[i] == pytest.approx(xmin, abs=1e-9)
            assert nh[i] == pytest.approx(xmax, abs=1e-9)
        checked += 1
    assert checked > 30


def test_parallel_is_intersection_and_sequential_is_tighter_but_sound():
    rng = np.random.default_rng(13)
    for _ in range(40):
        n = int(rng.integers(2, 6))
        m = int(rng.integers(2, 4))
        a, c, G, h, lo, hi = rand_problem(rng, n, m)
        pl, ph, pinf = relaxed.clip_parallel(G[None], h[None], lo[None], hi[None])
        sl, sh, sinf = relaxed.clip_sequential(G[None], h[None], lo[None], hi[None])
        single = [relaxed.clip_single_literal(G[k], h[k], lo, hi) for k in range(m)]
        if any(s[2] for s in single):
            assert pinf[0] and sinf[0]
            continue
        inter_lo = np.max([s[0] for s in single], axis=0)
        inter_hi = np.min([s[1] for s in single], axis=0)
        assert np.allclose(pl[0], inter_lo) and np.allclose(ph[0], inter_hi)
        feasible = exact.lp_vertices(np.zeros(n), 0.0, G, h, lo, hi)[0] != np.inf
        if not feasible:
            continue
        assert not sinf[0]
        assert np.all(sl[0] >= pl[0] - 1e-12) and np.all(sh[0] <= ph[0] + 1e-12)
        for i in range(n):     # the sequential box still contains box ∩ all constraints
            e = np.zeros(n)
            e[i] = 1.0
            assert sl[0][i] <= exact.lp_vertices(e, 0.0, G, h, lo, hi)[0] + 1e-9
            assert sh[0][i] >= -exact.lp_vertices(-e, 0.0, G, h, lo, hi)[0] - 1e-9


def test_sequential_clipping_depends_on_order():
    # order dependency theorem: the sequential box depends on the permutation
    # (2 constraints, box [0,3]x[0,1]); the parallel box does not.
    G = np.array([[-1.0, 3.0], [0.0, -3.0]])
    h = np.array([1.0, 1.0])
    lo = np.array([0.0, 0.0])
    hi = np.array([3.0, 1.0])
    a = relaxed.clip_sequential(G[None], h[None], lo[None], hi[None])
    b = relaxed.clip_sequential(G[None, ::-1], h[None, ::-1], lo[None], hi[None])
    assert np.allclose(a[0], [[1.0, 1.0 / 3.0]]) and np.allclose(b[0], [[2.0, 1.0 / 3.0]])
    assert np.allclose(a[1], b[1])
    pa = relaxed.clip_parallel(G[None], h[None], lo[None], hi[None])
    pb = relaxed.clip_parallel(G[None, ::-1], h[None, ::-1], lo[None], hi[None])
    assert np.allclose(pa[0], pb[0]) and np.allclose(pa[1], pb[1])
    # both orders still contain box ∩ constraints = [2, 3] x [1/3, 2/3]
    for i in range(2):
        e = np.eye(2)[i]
        xmin = exact.lp_vertices(e, 0.0, G, h, lo, hi)[0]
        xmax = -exact.lp_vertices(-e, 0.0, G, h, lo, hi)[0]
        for box_ in (a, b):
            assert box_[0][0, i] <= xmin + 1e-12 and box_[1][0, i] >= xmax - 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_single_constraint_solvers_agree_with_exact_lp(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(25):
        n = int(rng.integers(1, 6))
        a, c, G, h, lo, hi = rand_problem(rng, n, 1)
        Le, be = complete.single_enum(a, c, G[0], h[0], lo, hi)
        Ls, bs, infs = complete.single_max(a[None], np.array([c]), G, h, lo[None], hi[None])
        Lk, infk = complete.knapsack_greedy(a, c, G[0], h[0], lo, hi)
        Lv = exact.lp_vertices(a, c, G, h, lo, hi)[0]
        if Lv == np.inf:
            assert Le == np.inf and Ls[0] == np.inf and infk and infs[0]
            continue
        assert Le == pytest.approx(Lv, abs=1e-9)
        assert Ls[0] == pytest.approx(Lv, abs=1e-9)
        assert Lk == pytest.approx(Lv, abs=1e-9)
        assert bs[0] == pytest.approx(be, abs=1e-9)      # smallest maximiser


def test_single_constraint_exact_rational():
    rng = np.random.default_rng(7)
    for _ in range(8):
        n = int(rng.integers(2, 5))
        a, c, G, h, lo, hi = rand_problem(rng, n, 1, degenerate=False)
        Lx = exact.lp_simplex(a, c, G, h, lo, hi)
        Lv = exact.lp_vertices(a, c, G, h, lo, hi, exact=True)[0]
        if Lx == np.inf:
            assert Lv == np.inf
            continue
        assert Lx == Lv
        Le, _ = complete.single_enum(a, c, G[0], h[0], lo, hi)
        assert Le == pytest.approx(float(Lx), abs=1e-12)


def test_redundant_constraint_gives_zero_multiplier():
    lo, hi = np.zeros(3), np.ones(3)
    a = np.array([1.0, -2.0, 0.5])
    G = np.array([[1.0, 1.0, 1.0]])
    h = np.array([-5.0])           # max over the box is -2 <= 0: redundant
    L, beta, inf = complete.single_max(a[None], np.array([0.0]), G, h, lo[None], hi[None])
    assert beta[0] == 0.0 and not inf[0]
    assert L[0] == pytest.approx(box.concretize_min(a[None], np.array([0.0]), lo, hi)[0])


def test_coordinate_ascent_is_a_valid_and_useful_dual_bound():
    rng = np.random.default_rng(14)
    for _ in range(40):
        n = int(rng.integers(2, 6))
        m = int(rng.integers(1, 4))
        a, c, G, h, lo, hi = rand_problem(rng, n, m)
        L, beta, inf = complete.coord_ascent(a[None], np.array([c]), G[None], h[None], lo[None], hi[None])
        Lp = exact.lp_vertices(a, c, G, h, lo, hi)[0]
        if inf[0]:
            assert Lp == np.inf
            continue
        if Lp == np.inf:
            continue               # jointly empty but every single constraint feasible
        assert L[0] <= Lp + 1e-9                             # weak duality
        L1 = exact.lp_vertices(a, c, G[:1], h[:1], lo, hi)[0]
        assert L[0] >= L1 - 1e-9                             # first step is exact
        if m == 1:
            assert L[0] == pytest.approx(Lp, abs=1e-9)
        L2, _, _ = complete.coord_ascent(a[None], np.array([c]), G[None], h[None], lo[None], hi[None], passes=3)
        assert L2[0] >= L[0] - 1e-9                          # ascent
        assert L2[0] <= Lp + 1e-9
        assert np.all(beta >= 0.0)


def test_coordinate_ascent_is_exact_for_disjoint_constraints():
    # constraints on disjoint coordinate sets: the dual separates into one
    # concave function per multiplier, so one pass of exact 1-D maximisations
    # reaches the dual optimum, which equals the LP optimum (strong duality)
    rng = np.random.default_rng(11)
    for trial in range(12):
        n, k = 9, 3
        lo = rng.uniform(-1, 0, n)
        hi = rng.uniform(0, 1, n)
        a = rng.normal(size=n)
        perm = rng.permutation(n)
        G = np.zeros((k, n))
        for q, part in enumerate(np.array_split(perm, k)):
            G[q, part] = rng.normal(size=part.size)
        xs = rng.uniform(lo, hi)
        h = -(G @ xs) - rng.uniform(0.0, 0.2, k)
        act = np.ones((1, k), bool)
        L, _, emp = complete.coord_ascent(a[None], np.zeros(1), G[None], h[None], lo[None], hi[None], act)
        assert not emp[0]
        lp = exact.lp_simplex(a, 0.0, G, h, lo, hi)
        assert L[0] == pytest.approx(float(lp), abs=1e-9)
