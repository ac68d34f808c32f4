"""Mesh topology, geometry and interface elements (oracle).

Follows Sec. "Computational framework": bulk simplices carry independent
(discontinuous) P^k displacement nodes; an interface element sits on every
interior face (the internal boundary of the partition); the pressure lives
on the continuous P^k skeleton of the interface elements where the fluid
flag beta is set.  Opening w = [[u]] . n_Gamma with [[.]] = (.)^+ - (.)^- and
n_Gamma the normal of the "-" side (eq. displacementJump).

Readings where the paper is silent:
  * the "-" element of an interior face is the one with the lower element id
    and n_Gamma is its outward unit normal (``flip_labels`` swaps the roles,
    used by the label-invariance test);
  * mesh size of a face h_f = min(|e+|, |e-|) / |f|;
  * a displacement node is clamped (strong Dirichlet, u = ubar) when it lies
    on a boundary facet whose vertices are all flagged;
  * pressure unknowns exist only on nodes of faces with beta = 1, ordered:
    vertex nodes by vertex id, then edge-midpoint nodes by (lo, hi) vertex id.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import quadrature, shapes


class Mesh:
    def __init__(self, dim: int, order: int, xyz: np.ndarray, elem: np.ndarray,
                 dirichlet_vert: Optional[np.ndarray] = None, flip_labels: bool = False):
        self.dim, self.order = int(dim), int(order)
        d = self.dim
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.elem = np.asarray(elem, dtype=np.int64)
        self.ne = self.elem.shape[0]
        self.nn = shapes.n_nodes(d, order)
        self.bu = self.nn * d
        self.n_u = self.ne * self.bu

        # ---- element geometry: x = X0 + J xi -------------------------------
        X = self.xyz[self.elem]                                  # (ne, d+1, d)
        self.J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
        self.detJ = np.linalg.det(self.J)
        self.vol = np.abs(self.detJ) / math.factorial(d)
        Jinv = np.linalg.inv(self.J)
        gl = np.zeros((self.ne, d + 1, d))
        gl[:, 1:, :] = Jinv                                      # grad lam_k = row k-1 of J^-1
        gl[:, 0, :] = -Jinv.sum(axis=1)
        self.grad_lam = gl

        # ---- faces ----------------------------------------------------------
        owners: Dict[Tuple[int, ...], List[Tuple[int, int]]] = {}
        for e in range(self.ne):
            ev = self.elem[e]
            for lf in range(d + 1):
                key = tuple(sorted(int(ev[c]) for c in range(d + 1) if c != lf))
                owners.setdefault(key, []).append((e, lf))
        interior, boundary = [], []
        for key, lst in owners.items():
            if len(lst) == 2:
                interior.append(key)
            elif len(lst) == 1:
                boundary.append(key)
            else:
                raise ValueError("non-manifold face")
        interior.sort()
        boundary.sort()
        self.face_keys = interior
        self.face_index = {k: i for i, k in enumerate(interior)}
        self.nf = len(interior)
        fv = np.array(interior, dtype=np.int64).reshape(self.nf, d)
        self.face_vert = fv
        em = np.empty(self.nf, dtype=np.int64)
        ep = np.empty(self.nf, dtype=np.int64)
        for i, key in enumerate(interior):
            (a, _), (b, _) = owners[key]
            lo, hi = min(a, b), max(a, b)
            em[i], ep[i] = (hi, lo) if flip_labels else (lo, hi)
        self.face_em, self.face_ep = em, ep
        # local position of each face vertex inside each element
        pos_m = np.empty((self.nf, d), dtype=np.int64)
        pos_p = np.empty((self.nf, d), dtype=np.int64)
        opp_m = np.empty(self.nf, dtype=np.int64)
        for i in range(self.nf):
            lm = list(self.elem[em[i]])
            lp = list(self.elem[ep[i]])
            for k in range(d):
                pos_m[i, k] = lm.index(fv[i, k])
                pos_p[i, k] = lp.index(fv[i, k])
            opp_m[i] = [c for c in range(d + 1) if c not in pos_m[i]][0]
        self.face_pos_m, self.face_pos_p = pos_m, pos_p
        self.face_local_m = opp_m

        # ---- face geometry ---------------------------------------------------
        V = self.xyz[fv]                                         # (nf, d, d)
        Jf = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))  # (nf, d, d-1)
        if d == 2:
            t = Jf[:, :, 0]
            nraw = np.stack([t[:, 1], -t[:, 0]], axis=1)
            area = np.linalg.norm(nraw, axis=1)
        else:
            nraw = np.cross(Jf[:, :, 0], Jf[:, :, 1])
            area = 0.5 * np.linalg.norm(nraw, axis=1)
        xopp = self.xyz[self.elem[em, opp_m]]
        sgn = np.where(np.einsum("fi,fi->f", nraw, xopp - V[:, 0, :]) > 0.0, -1.0, 1.0)
        self.normal = nraw * (sgn / np.linalg.norm(nraw, axis=1))[:, None]
        self.area = area
        self.hf = np.minimum(self.vol[em], self.vol[ep]) / area
        Gf = np.einsum("fia,fib->fab", Jf, Jf)
        self.face_Ginv = np.linalg.inv(Gf)

        # ---- face quadrature, mapped into both elements ----------------------
        fq, fw = quadrature.face_rule(d, order)
        self.fq_pts, self.fq_w = fq, fw
        self.nq = len(fw)
        mu = shapes.ref_to_bary(fq)                               # (nq, d)
        self.fq_mu = mu
        lam_m = np.zeros((self.nf, self.nq, d + 1))
        lam_p = np.zeros((self.nf, self.nq, d + 1))
        fi = np.arange(self.nf)[:, None]
        qi = np.arange(self.nq)[None, :]
        for k in range(d):
            # the face vertex k sits at local vertex pos[f, k] of the element
            lam_m[fi, qi, pos_m[:, k][:, None]] = mu[None, :, k]
            lam_p[fi, qi, pos_p[:, k][:, None]] = mu[None, :, k]
        self.face_lam_m, self.face_lam_p = lam_m, lam_p
        # pressure (skeleton) shape functions on the face simplex
        self.nnf = shapes.n_nodes(d - 1, order)
        self.eta = shapes.phi(mu, d - 1, order)                   # (nq, nnf)
        dmu_dst = np.vstack([-np.ones((1, d - 1)), np.eye(d - 1)])  # (d, d-1)
        self.deta_dst = np.einsum("qkm,ms->qks", shapes.dphi_dlam(mu, d - 1, order), dmu_dst)

        # ---- volume quadrature ----------------------------------------------
        vq, vw = quadrature.volume_rule(d, order)
        self.vq_pts, self.vq_w = vq, vw

        # ---- Dirichlet node copies ---------------------------------------------
        if dirichlet_vert is None:
            dirichlet_vert = np.zeros(len(self.xyz), dtype=np.uint8)
        dv = np.asarray(dirichlet_vert).astype(bool)
        cv, ce = set(), set()
        for key in boundary:
            if all(dv[v] for v in key):
                cv.update(key)
                for a, b in shapes.EDGES[d - 1]:
                    ce.add(tuple(sorted((key[a], key[b]))))
        clamp = np.zeros((self.ne, self.nn), dtype=bool)
        for e in range(self.ne):
            for a, k in enumerate(shapes.node_keys(self.elem[e], d, order)):
                clamp[e, a] = (k[1] in cv) if k[0] == "v" else ((k[1], k[2]) in ce)
        self.clamped_node = clamp
        self.clamped_dof = np.repeat(clamp.reshape(-1), d)       # (n_u,)

    # ------------------------------------------------------------------------
    def dof(self, e, a, i):
        return (e * self.nn + a) * self.dim + i

    def face_of(self, key) -> int:
        return self.face_index[tuple(sorted(int(v) for v in key))]

    def node_xyz(self) -> np.ndarray:
        """Physical coordinates of every element node copy (ne, nn, d)."""
        nb = shapes.node_bary(self.dim, self.order)               # (nn, d+1)
        return np.einsum("ak,ekd->ead", nb, self.xyz[self.elem])


class Interfaces:
    """Interface state: per-qp activation state (0 intact/DG, 1 cohesive law,
    2 traction-free) and the per-face fluid flag beta, plus the active
    pressure-node numbering they induce."""

    def __init__(self, mesh: Mesh, crack_faces=None, crack_state=None, crack_beta=None,
                 qp_state: Optional[np.ndarray] = None, beta: Optional[np.ndarray] = None):
        m = mesh
        self.mesh = m
        if qp_state is None:
            qp_state = np.zeros((m.nf, m.nq), dtype=np.uint8)
            beta = np.zeros(m.nf, dtype=np.uint8)
            if crack_faces is not None:
                for key, st, bt in zip(np.asarray(crack_faces), np.asarray(crack_state),
                                       np.asarray(crack_beta)):
                    f = m.face_of(key)
                    qp_state[f, :] = st
                    beta[f] = bt
        self.qp_state = np.asarray(qp_state, dtype=np.uint8)
        self.beta = np.asarray(beta, dtype=np.uint8)
        # active skeleton pressure nodes
        keys = set()
        face_nodes = {}
        for f in np.nonzero(self.beta)[0]:
            ks = shapes.node_keys(m.face_vert[f], m.dim - 1, m.order)
            face_nodes[int(f)] = ks
            keys.update(ks)
        vk = sorted(k for k in keys if k[0] == "v")
        ek = sorted(k for k in keys if k[0] == "e")
        self.p_keys = vk + ek
        self.p_index = {k: i for i, k in enumerate(self.p_keys)}
        self.n_p = len(self.p_keys)
        self.active_faces = np.array(sorted(face_nodes), dtype=np.int64)
        self.face_pnodes = np.array([[self.p_index[k] for k in face_nodes[int(f)]]
                                     for f in self.active_faces], dtype=np.int64).reshape(
                                         len(self.active_faces), m.nnf)

    def p_node_of_vertex(self, v: int) -> int:
        return self.p_index[("v", int(v))]
