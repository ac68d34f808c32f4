"""Conical-product Gauss rules on the reference simplex (oracle).

The paper does not state its quadrature.  The reading used here: the
collapsed-coordinate (Duffy) map of the unit simplex onto the unit cube,
with a Gauss-Jacobi rule in each collapsed direction (weight (1-s)^a) and
Gauss-Legendre in the last one.  ``n`` points per direction integrate every
polynomial of total degree <= 2n-1 exactly.

Reference simplices: segment [0,1]; triangle (0,0),(1,0),(0,1); tetrahedron
(0,0,0),(1,0,0),(0,1,0),(0,0,1).  Point order: first collapsed coordinate
outermost, each 1D point set ascending.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi


def gauss_jacobi_01(n: int, a: int):
    """n-point rule on [0,1] for the weight (1-s)^a (library Golub-Welsch)."""
    x, w = roots_jacobi(n, a, 0)          # weight (1-x)^a (1+x)^0 on [-1,1]
    s = 0.5 * (1.0 + x)
    ws = w * 0.5 ** (a + 1)
    order = np.argsort(s)
    return s[order], ws[order]


def simplex_rule(dim: int, n: int):
    """Points (nq, dim) and weights (nq,) on the reference simplex; the
    weights sum to its measure (1, 1/2, 1/6)."""
    if dim == 1:
        s, w = gauss_jacobi_01(n, 0)
        return s[:, None], w
    if dim == 2:
        s, ws = gauss_jacobi_01(n, 1)
        t, wt = gauss_jacobi_01(n, 0)
        pts, wts = [], []
        for i in range(n):
            for j in range(n):
                pts.append((s[i], t[j] * (1.0 - s[i])))
                wts.append(ws[i] * wt[j])
        return np.array(pts), np.array(wts)
    if dim == 3:
        s, ws = gauss_jacobi_01(n, 2)
        t, wt = gauss_jacobi_01(n, 1)
        r, wr = gauss_jacobi_01(n, 0)
        pts, wts = [], []
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    pts.append((s[i], t[j] * (1.0 - s[i]), r[k] * (1.0 - s[i]) * (1.0 - t[j])))
                    wts.append(ws[i] * wt[j] * wr[k])
        return np.array(pts), np.array(wts)
    raise ValueError(dim)


def volume_rule(dim: int, order: int):
    """Element rule: n = order points per direction (exact to degree 2*order-1,
    enough for the P^k stiffness integrand of degree 2(k-1))."""
    return simplex_rule(dim, order)


def face_rule(dim: int, order: int):
    """Interface rule on the (dim-1)-simplex: n = order+1 points per direction
    (exact to degree 2*order+1, enough for the penalty integrand of degree
    2k).  Weights are normalised to sum to one, so that they multiply the
    physical face measure."""
    pts, w = simplex_rule(dim - 1, order + 1)
    return pts, w / w.sum()
