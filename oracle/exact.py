"""Exact checkers for tiny problems (n <= ~10), independent of the dual-based
solvers they are used to pin.

* ``lp_vertices``: the optimum of  min a.x + c  over
  {lo <= x <= hi, G x + h <= 0}  by enumerating vertices.  A vertex of a box
  cut by m halfspaces has some set S of tight halfspaces (|S| <= n) and at
  least n - |S| coordinates at a box bound; every such combination is solved
  as a small linear system.  Fraction (rational) arithmetic is optional.
* ``lp_simplex``: the same LP by a two-phase tableau simplex with Bland's
  rule, in exact rational arithmetic.
* ``box_corners_min``: brute force over the 2^n corners of a box (Lemma A.2
  check).

Both LP routines return +inf for an empty feasible set.
"""
from fractions import Fraction
from itertools import combinations, product

import numpy as np


def box_corners_min(a, c, lo, hi):
    best = np.inf
    for bits in product((0, 1), repeat=len(a)):
        x = np.where(np.array(bits) == 1, hi, lo)
        best = min(best, float(np.dot(a, x) + c))
    return best


def _solve(M, r):
    """Gaussian elimination with exact pivoting on a list-of-lists matrix of
    Fractions (or floats).  Returns the solution or None if singular."""
    n = len(M)
    A = [row[:] + [r[i]] for i, row in enumerate(M)]
    for col in range(n):
        piv = None
        best = 0
        for i in range(col, n):
            v = abs(A[i][col])
            if v > best:
                best, piv = v, i
        if piv is None or best == 0 or (not isinstance(best, Fraction) and best < 1e-12):
            return None
        A[col], A[piv] = A[piv], A[col]
        for i in range(n):
            if i != col and A[i][col] != 0:
                f = A[i][col] / A[col][col]
                A[i] = [x - f * y for x, y in zip(A[i], A[col])]
    return [A[i][n] / A[i][i] for i in range(n)]


def lp_vertices(a, c, G, h, lo, hi, exact=False, tol=1e-9):
    """min a.x + c over the box cut by G x + h <= 0 by vertex enumeration.
    Returns (value, argmin) (value +inf, None if empty)."""
    conv = (lambda v: Fraction(float(v))) if exact else float
    a = [conv(v) for v in np.ravel(a)]
    lo = [conv(v) for v in np.ravel(lo)]
    hi = [conv(v) for v in np.ravel(hi)]
    G = [[conv(v) for v in row] for row in np.atleast_2d(G)] if np.size(G) else []
    h = [conv(v) for v in np.ravel(h)] if np.size(h) else []
    c = conv(c)
    n, m = len(a), len(G)
    zero = Fraction(0) if exact else 0.0
    slack = zero if exact else tol
    best, arg = None, None
    for s in range(0, min(m, n) + 1):
        for S in combinations(range(m), s):
            for free in combinations(range(n), s):
                fixed = [i for i in range(n) if i not in free]
                for bits in product((0, 1), repeat=len(fixed)):
                    x = [None] * n
                    for i, bt in zip(fixed, bits):
                        x[i] = hi[i] if bt else lo[i]
                    if s:
                        Msys = [[G[k][i] for i in free] for k in S]
                        rhs = [-h[k] - sum(G[k][i] * x[i] for i in fixed) for k in S]
                        sol = _solve(Msys, rhs)
                        if sol is None:
                            continue
                        for i, v in zip(free, sol):
                            x[i] = v
                    ok = all(lo[i] - slack <= x[i] <= hi[i] + slack for i in range(n))
                    ok = ok and all(sum(G[k][i] * x[i] for i in range(n)) + h[k] <= slack
                                    for k in range(m))
                    if not ok:
                        continue
                    val = sum(a[i] * x[i] for i in range(n)) + c
                    if best is None or val < best:
                        best, arg = val, x
    if best is None:
        return np.inf, None
    return best, arg


def lp_simplex(a, c, G, h, lo, hi):
    """min a.x + c over {lo <= x <= hi, G x + h <= 0} by a two-phase tableau
    simplex (Bland's rule) in exact rational arithmetic.  Substitutes
    y = x - lo >= 0; rows are y_i <= hi_i - lo_i and G y <= -h - G lo."""
    F = lambda v: Fraction(float(v))
    a = [F(v) for v in np.ravel(a)]
    lo = [F(v) for v in np.ravel(lo)]
    hi = [F(v) for v in np.ravel(hi)]
    Gm = [[F(v) for v in row] for row in np.atleast_2d(G)] if np.size(G) else []
    hv = [F(v) for v in np.ravel(h)] if np.size(h) else []
    n = len(a)
    rows, rhs = [], []
    for i in range(n):
        r = [Fraction(0)] * n
        r[i] = Fraction(1)
        rows.append(r)
        rhs.append(hi[i] - lo[i])
    for k in range(len(Gm)):
        rows.append(Gm[k][:])
        rhs.append(-hv[k] - sum(Gm[k][i] * lo[i] for i in range(n)))
    m = len(rows)
    # equality form: rows y + slack = rhs; negative rhs rows are negated and
    # receive an artificial variable.
    nv = n + m
    T, basis, art = [], [], []
    for i in range(m):
        coef = rows[i] + [Fraction(1) if j == i else Fraction(0) for j in range(m)]
        b = rhs[i]
        if b < 0:
            coef = [-x for x in coef]
            b = -b
            art.append(i)
        T.append(coef + [b])
    na = len(art)
    for idx, i in enumerate(art):
        for r in range(m):
            T[r].insert(nv + idx, Fraction(1) if r == i else Fraction(0))
    for i in range(m):
        basis.append(nv + art.index(i) if i in art else n + i)
    width = nv + na

    def pivot(r, col):
        p = T[r][col]
        T[r] = [x / p for x in T[r]]
        for i in range(m):
            if i != r and T[i][col] != 0:
                f = T[i][col]
                T[i] = [x - f * y for x, y in zip(T[i], T[r])]
        basis[r] = col

    def run(cost, allowed):
        while True:
            # reduced costs
            red = []
            for j in range(width):
                if not allowed(j):
                    red.append(Fraction(0))
                    continue
                z = sum(cost[basis[i]] * T[i][j] for i in range(m))
                red.append(cost[j] - z)
            enter = next((j for j in range(width) if allowed(j) and red[j] < 0), None)
            if enter is None:
                return True
            ratios = [(T[i][-1] / T[i][enter], basis[i], i) for i in range(m) if T[i][enter] > 0]
            if not ratios:
                return False  # unbounded (cannot happen on a box)
            best = min(r[0] for r in ratios)
            leave = min((r for r in ratios if r[0] == best), key=lambda r: r[1])[2]
            pivot(leave, enter)

    if na:
        cost1 = [Fraction(0)] * nv + [Fraction(1)] * na
        run(cost1, lambda j: True)
        phase1 = sum(T[i][-1] for i in range(m) if basis[i] >= nv)
        if phase1 > 0:
            return np.inf
        # drive artificial variables out of the basis
        for i in range(m):
            if basis[i] >= nv:
                col = next((j for j in range(nv) if T[i][j] != 0), None)
                if col is not None:
                    pivot(i, col)
    cost2 = a + [Fraction(0)] * (m + na)
    run(cost2, lambda j: j < nv)
    y = [Fraction(0)] * nv
    for i in range(m):
        if basis[i] < nv:
            y[basis[i]] = T[i][-1]
    return sum(a[i] * (y[i] + lo[i]) for i in range(n)) + F(c)
