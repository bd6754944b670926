"""Concretization over an axis-aligned box (Lemma A.2; eq. 1 of the
preliminaries).

For v in R^n and the box X = {lo <= x <= hi} (centre xh = (lo+hi)/2, radius
eps = (hi-lo)/2):  min_X v.x = v.xh - |v|.eps  and  max_X v.x = v.xh + |v|.eps.
The oracle evaluates the algebraically identical endpoint form
sum_j min(v_j lo_j, v_j hi_j), which avoids forming the centre and radius.
All arithmetic is float64.
"""
import numpy as np


def f64(a):
    return np.asarray(a, dtype=np.float64)


def concretize_min(A, c, lo, hi):
    """min over the box of A x + c, row-wise.

    A: [..., P, n], c: [..., P], lo/hi: [..., n] (broadcast against A's
    leading dims).  Returns [..., P].  Lemma A.2 (minimisation line)."""
    A, c, lo, hi = f64(A), f64(c), f64(lo), f64(hi)
    lo_ = lo[..., None, :]
    hi_ = hi[..., None, :]
    return np.minimum(A * lo_, A * hi_).sum(axis=-1) + c


def concretize_max(A, c, lo, hi):
    """max over the box of A x + c (Lemma A.2, maximisation line)."""
    A, c, lo, hi = f64(A), f64(c), f64(lo), f64(hi)
    lo_ = lo[..., None, :]
    hi_ = hi[..., None, :]
    return np.maximum(A * lo_, A * hi_).sum(axis=-1) + c


def concretize_min_centre(A, c, lo, hi):
    """The centre/radius form printed in the paper, v.xh - |v|.eps + c; kept
    to pin the endpoint form against it."""
    A, c, lo, hi = f64(A), f64(c), f64(lo), f64(hi)
    xh = (lo + hi) / 2.0
    eps = (hi - lo) / 2.0
    return (A * xh[..., None, :]).sum(-1) - (np.abs(A) * eps[..., None, :]).sum(-1) + c


def concretize_min_shared(A, c, lo, hi):
    """Same minimum for planes shared by a batch of boxes, written with
    matrix products: lo A+^T + hi A-^T + c.  A: [P, n], c: [P],
    lo/hi: [B, n] -> [B, P]."""
    A, c, lo, hi = f64(A), f64(c), f64(lo), f64(hi)
    return lo @ np.maximum(A, 0.0).T + hi @ np.minimum(A, 0.0).T + c


def concretize_max_shared(A, c, lo, hi):
    """max over each box of A x + c for shared planes: hi A+^T + lo A-^T + c."""
    A, c, lo, hi = f64(A), f64(c), f64(lo), f64(hi)
    return hi @ np.maximum(A, 0.0).T + lo @ np.minimum(A, 0.0).T + c
