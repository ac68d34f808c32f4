"""Lagrange P1/P2 bases on simplices in barycentric coordinates (oracle).

Both spaces of the method use these (Sec. "Computational framework"): the
discontinuous displacement space uses P^k on each bulk simplex; the
continuous pressure space uses P^k on each interface simplex.

Local node order: the simplex vertices in the order given, then (P2) one
node per edge at its midpoint, edges listed as
  segment      (0,1)
  triangle     (0,1), (1,2), (2,0)
  tetrahedron  (0,1), (1,2), (2,0), (0,3), (1,3), (2,3)
Basis: P1 phi_a = lam_a; P2 vertex phi_a = lam_a(2 lam_a - 1), edge
phi_ab = 4 lam_a lam_b.
"""
from __future__ import annotations

import numpy as np

EDGES = {
    1: [(0, 1)],
    2: [(0, 1), (1, 2), (2, 0)],
    3: [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)],
}


def n_nodes(dim: int, order: int) -> int:
    return dim + 1 if order == 1 else dim + 1 + len(EDGES[dim])


def node_keys(vertices, dim: int, order: int):
    """Global identity of each local node of a simplex with global vertex
    ids ``vertices``: ('v', id) or ('e', lo, hi)."""
    keys = [("v", int(v)) for v in vertices]
    if order == 2:
        for a, b in EDGES[dim]:
            lo, hi = sorted((int(vertices[a]), int(vertices[b])))
            keys.append(("e", lo, hi))
    return keys


def phi(lam: np.ndarray, dim: int, order: int) -> np.ndarray:
    """lam (..., dim+1) -> basis values (..., n_nodes)."""
    if order == 1:
        return lam.copy()
    cols = [lam[..., a] * (2.0 * lam[..., a] - 1.0) for a in range(dim + 1)]
    cols += [4.0 * lam[..., a] * lam[..., b] for a, b in EDGES[dim]]
    return np.stack(cols, axis=-1)


def dphi_dlam(lam: np.ndarray, dim: int, order: int) -> np.ndarray:
    """Partial derivatives wrt each barycentric coordinate:
    (..., n_nodes, dim+1)."""
    shp = lam.shape[:-1]
    nn = n_nodes(dim, order)
    out = np.zeros(shp + (nn, dim + 1))
    if order == 1:
        for a in range(dim + 1):
            out[..., a, a] = 1.0
        return out
    for a in range(dim + 1):
        out[..., a, a] = 4.0 * lam[..., a] - 1.0
    for k, (a, b) in enumerate(EDGES[dim]):
        out[..., dim + 1 + k, a] = 4.0 * lam[..., b]
        out[..., dim + 1 + k, b] = 4.0 * lam[..., a]
    return out


def ref_to_bary(xi: np.ndarray) -> np.ndarray:
    """Reference coordinates (..., dim) -> barycentric (..., dim+1) with
    lam_0 = 1 - sum(xi), lam_k = xi_{k-1}."""
    return np.concatenate([1.0 - xi.sum(axis=-1, keepdims=True), xi], axis=-1)


def node_bary(dim: int, order: int) -> np.ndarray:
    """Barycentric coordinates of the local nodes (n_nodes, dim+1)."""
    pts = [np.eye(dim + 1)[a] for a in range(dim + 1)]
    if order == 2:
        for a, b in EDGES[dim]:
            pts.append(0.5 * (np.eye(dim + 1)[a] + np.eye(dim + 1)[b]))
    return np.array(pts)
