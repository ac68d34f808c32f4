"""Residual and consistent Jacobian of the fully-discrete coupled system
(oracle).

The discrete equations are eq. (discreteElastoStatics) and
eq. (discreteLubrication) of Sec. "Computational framework"; their
linearisation is the 2x2 block system eq. (fully-coupled-fully-discrete)
[[A, B], [C, D]] [U; P] = [E; F], whose blocks the paper lists in a passage
excluded from the published text.  Here the Jacobian is the exact derivative
of the residual written below (checked against finite differences by the
tests); the paper's printed cohesive tangent t'.n [[phi_j]].[[phi_i]] is
replaced by the derivative of the normal-only law, T'(w) (n.[[phi_j]])(n.[[phi_i]]).

Residual, for a displacement test function v (one DG node copy, one
component) and an active pressure node i:

  R_u(v) = sum_e int_e C eps(u) : eps(v)
         + sum_faces int_f [ (1-alpha)( <C eps(u)> n + (b/h) Chat(n) [[u]] )
                             + alpha T(w) n - beta p n ] . [[v]]
  R_p(i) = s_p { sum_{faces, beta=1} int_f [ K(w) grad_G p . grad_G eta_i
                                            + (w - w_old)/dt eta_i ]
                 - sum_sources Q0 eta_i(x_src) }

with Chat(n) = G I + (lambda + G) n (x) n, which equals the paper's
stabilisation [[v]] (x) n : C : [[u]] (x) n; K(w) = max(w,0)^3 / (12 mu)
(cubic law of eq. lubrication, clamped at w = 0 where the equation
degenerates); s_p the fluid-row scale (a reading of the paper's remark on
scaling the fluid equations, see ``newton.fluid_scale``).

Interface law (eq. tsl, extended where the paper is silent):
  state 1 (cohesive): T = sigma_c (1 - w/delta_c) for 0 <= w <= delta_c,
                      T = 0 for w > delta_c, T = sigma_c + k_c w for w < 0
  state 2 (pre-crack, traction free): T = 0 for w >= 0, T = k_c w for w < 0
  k_c = (b/h_f)(lambda + 2G) (contact penalty: the normal stiffness of the DG
  stabilisation, so a closing rigid motion meets the force it meets on an
  intact face), delta_c = 2 G_c / sigma_c.
alpha = 1 at integration points with state >= 1.
Unloading (optional history w_max per face point, the largest opening a
cohesive point has reached at the end of a load step; the paper cites the
Camacho-Ortiz law for eq. tsl and prints only its loading envelope; the
reading here is that law's irreversible linear unloading to the origin):
in state 1, with w_m = max(w_max, 0) > 0 and w < w_m, T = (T_env(w_m)/w_m) w
for 0 <= w < w_m and T = k_c w for w < 0 (the secant reaches zero at w = 0);
from w >= w_m on the envelope applies again.

Clamped displacement copies get the row R = u - ubar with an identity
Jacobian row.  Plane strain in 2D.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import shapes
from .mesh import Interfaces, Mesh


@dataclasses.dataclass
class Params:
    E: float
    nu: float
    sigma_c: float
    G_c: float
    mu: float
    dt: float
    b_stab: float = 10.0

    @property
    def lame(self):
        lam = self.E * self.nu / ((1.0 + self.nu) * (1.0 - 2.0 * self.nu))
        G = self.E / (2.0 * (1.0 + self.nu))
        return lam, G

    @property
    def delta_c(self):
        # G_c = sigma_c delta_c / 2 (Sec. "Governing equations", after eq. tsl)
        return 2.0 * self.G_c / self.sigma_c


def traction_law(state, w, sigma_c, delta_c, kc, w_max=None):
    """Normal cohesive traction T(w) and dT/dw for interface state 1 or 2.

    Follows eq. (tsl) on 0 <= w <= delta_c; see the module docstring for the
    branches outside it and for the unloading branch of a state-1 point
    whose history w_max exceeds its opening (readings).  ``w >= 0`` selects
    the softening / free branch at w = 0."""
    T = np.zeros_like(w)
    dT = np.zeros_like(w)
    neg = w < 0.0
    s1 = state == 1
    s2 = state == 2
    soft = s1 & ~neg & (w <= delta_c)
    T[soft] = sigma_c * (1.0 - w[soft] / delta_c)
    dT[soft] = -sigma_c / delta_c
    c1 = s1 & neg
    T[c1] = sigma_c + kc[c1] * w[c1]
    dT[c1] = kc[c1]
    c2 = s2 & neg
    T[c2] = kc[c2] * w[c2]
    dT[c2] = kc[c2]
    if w_max is not None:
        wm = np.maximum(w_max, 0.0)
        un = s1 & (wm > 0.0) & (w < wm)
        if np.any(un):
            # secant slope T_env(w_m) / w_m of the point's envelope value at w_m
            k_s = np.where(wm <= delta_c, sigma_c * (1.0 - wm / delta_c), 0.0) / np.where(un, wm, 1.0)
            op = un & ~neg
            T[op] = k_s[op] * w[op]
            dT[op] = k_s[op]
            cl = un & neg
            T[cl] = kc[cl] * w[cl]
            dT[cl] = kc[cl]
    return T, dT


def conductivity(w, mu):
    """Cubic-law conductivity K(w) = max(w,0)^3/(12 mu) and dK/dw (eq. lubrication)."""
    wp = np.maximum(w, 0.0)
    return wp ** 3 / (12.0 * mu), 3.0 * wp ** 2 / (12.0 * mu)


def _stress(grad_u, lam, G):
    """sigma = lambda tr(eps) I + 2 G eps with eps = sym(grad u); grad_u[..., i, x]."""
    eps = 0.5 * (grad_u + np.swapaxes(grad_u, -1, -2))
    tr = np.trace(eps, axis1=-2, axis2=-1)
    d = grad_u.shape[-1]
    return lam * tr[..., None, None] * np.eye(d) + 2.0 * G * eps


@dataclasses.dataclass
class System:
    """Assembled residual and Jacobian blocks.

    R_u (n_u,), R_p (n_p,);
    A_diag (ne, bu, bu): diagonal element blocks (after Dirichlet rows);
    A_mp / A_pm (nf, bu, bu): block (row e-, col e+) / (row e+, col e-) of each
    interior face; B (n_u x n_p), C (n_p x n_u), D (n_p x n_p) sparse.
    """
    R_u: np.ndarray
    R_p: np.ndarray
    A_diag: Optional[np.ndarray] = None
    A_mp: Optional[np.ndarray] = None
    A_pm: Optional[np.ndarray] = None
    B: Optional[sp.csr_matrix] = None
    C: Optional[sp.csr_matrix] = None
    D: Optional[sp.csr_matrix] = None

    @property
    def R(self):
        return np.concatenate([self.R_u, self.R_p])


def assemble(mesh: Mesh, itf: Interfaces, prm: Params, u: np.ndarray, p: np.ndarray,
             w_old: np.ndarray, s_p: float, src_pnode, src_q0, ubar: Optional[np.ndarray] = None,
             jacobian: bool = True, faces: Optional[np.ndarray] = None,
             elements: Optional[np.ndarray] = None, face_chunk: int = 4096,
             w_max: Optional[np.ndarray] = None) -> System:
    """Residual (and Jacobian) at the state (u, p).

    u: (n_u,) element-major DG displacement copies, index (e*nn + a)*d + i
    p: (n_p,) pressure at the active skeleton nodes
    w_old: (nf, nq) opening of the previous load step at face points
    w_max: optional (nf, nq) unloading history of the cohesive points (None:
        the loading envelope only)
    faces: optional subset of interior faces to include (default all); used
        to evaluate selected element rows.
    elements: optional subset of elements whose bulk term is included
        (default all; the others get a zero bulk term).
    """
    m = mesh
    d, nn, bu = m.dim, m.nn, m.bu
    lam, G = prm.lame
    ue = u.reshape(m.ne, nn, d)
    n_p = itf.n_p

    # ---------------- bulk term: sum_e int_e C eps(u) : eps(v) ------------------
    E = np.arange(m.ne) if elements is None else np.asarray(elements, dtype=np.int64)
    lq = shapes.ref_to_bary(m.vq_pts)
    dphi = shapes.dphi_dlam(lq, d, m.order)                     # (nqv, nn, d+1)
    gphi = np.einsum("qak,ekx->eqax", dphi, m.grad_lam[E])       # (nE, nqv, nn, d)
    wdet = m.vq_w[None, :] * np.abs(m.detJ[E])[:, None]         # (nE, nqv)
    grad_u = np.einsum("eai,eqax->eqix", ue[E], gphi)
    sig = _stress(grad_u, lam, G)
    R_u = np.zeros((m.ne, nn, d))
    R_u[E] = np.einsum("eq,eqix,eqax->eai", wdet, sig, gphi)
    R_u = R_u.reshape(-1)
    if jacobian:
        eye = np.eye(d)
        K = (lam * np.einsum("eq,eqai,eqbj->eaibj", wdet, gphi, gphi)
             + G * np.einsum("eq,eqax,eqbx,ij->eaibj", wdet, gphi, gphi, eye)
             + G * np.einsum("eq,eqaj,eqbi->eaibj", wdet, gphi, gphi))
        A_diag = np.zeros((m.ne, bu, bu))
        A_diag[E] = K.reshape(len(E), bu, bu)
        A_mp = np.zeros((m.nf, bu, bu))
        A_pm = np.zeros((m.nf, bu, bu))
    R_p = np.zeros(n_p)

    # pressure nodes of each face (only faces with beta = 1 have them)
    face_slot = -np.ones(m.nf, dtype=np.int64)
    face_slot[itf.active_faces] = np.arange(len(itf.active_faces))
    Bt, Ct, Dt = [], [], []       # (rows, cols, vals) triplets

    all_faces = np.arange(m.nf) if faces is None else np.asarray(faces)
    Ru3 = R_u.reshape(m.ne, nn, d)
    for c0 in range(0, len(all_faces), face_chunk):
        F = all_faces[c0:c0 + face_chunk]
        em, ep = m.face_em[F], m.face_ep[F]
        n = m.normal[F]                                          # (F, d)
        W = m.fq_w[None, :] * m.area[F][:, None]                 # (F, nq)
        bh = prm.b_stab / m.hf[F]                                # (F,)
        st = m_state = itf.qp_state[F]                           # (F, nq)
        alpha = (m_state > 0).astype(np.float64)
        beta = itf.beta[F].astype(np.float64)
        side = {}
        for name, e_s, lam_s, sg in (("m", em, m.face_lam_m[F], -1.0),
                                     ("p", ep, m.face_lam_p[F], +1.0)):
            ph = shapes.phi(lam_s, d, m.order)                   # (F, nq, nn)
            dph = shapes.dphi_dlam(lam_s, d, m.order)            # (F, nq, nn, d+1)
            gph = np.einsum("fqak,fkx->fqax", dph, m.grad_lam[e_s])
            us = ue[e_s]                                         # (F, nn, d)
            U = np.einsum("fqa,fai->fqi", ph, us)
            gU = np.einsum("fai,fqax->fqix", us, gph)
            side[name] = (e_s, ph, gph, U, _stress(gU, lam, G), sg)
        jump = side["p"][3] - side["m"][3]                       # [[u]] = u+ - u-
        w = np.einsum("fqi,fi->fq", jump, n)
        avg_sn = 0.5 * np.einsum("fqix,fx->fqi", side["m"][4] + side["p"][4], n)
        Chat = G * np.eye(d)[None] + (lam + G) * np.einsum("fi,fj->fij", n, n)
        kc = np.repeat((bh * (lam + 2.0 * G))[:, None], m.nq, axis=1)
        T, dT = traction_law(st, w, prm.sigma_c, prm.delta_c, kc,
                             None if w_max is None else w_max[F])
        # pressure at the face points (beta faces only)
        slot = face_slot[F]
        act = slot >= 0
        ph_p = np.zeros((len(F), m.nq))
        if np.any(act):
            pn = itf.face_pnodes[slot[act]]                      # (Fa, nnf)
            ph_p[act] = np.einsum("qk,fk->fq", m.eta, p[pn])
        tau = ((1.0 - alpha)[..., None] * (avg_sn + bh[:, None, None]
                                           * np.einsum("fij,fqj->fqi", Chat, jump))
               + (alpha * T)[..., None] * n[:, None, :]
               - (beta[:, None] * ph_p)[..., None] * n[:, None, :])
        for name in ("m", "p"):
            e_s, ph, _, _, _, sg = side[name]
            contrib = sg * np.einsum("fq,fqa,fqi->fai", W, ph, tau)
            np.add.at(Ru3, e_s, contrib)

        if jacobian:
            X = {}
            for name in ("m", "p"):
                e_t, ph, gph, _, _, sg = side[name]
                gn = np.einsum("fqbx,fx->fqb", gph, n)
                cons = 0.5 * (lam * np.einsum("fqbj,fi->fqbji", gph, n)
                              + G * np.einsum("fqbi,fj->fqbji", gph, n)
                              + G * np.einsum("fqb,ij->fqbji", gn, np.eye(d)))
                pen = sg * bh[:, None, None, None, None] * np.einsum(
                    "fqb,fij->fqbji", ph, Chat)
                coh = sg * np.einsum("fq,fqb,fi,fj->fqbji", dT, ph, n, n)
                X[name] = ((1.0 - alpha)[:, :, None, None, None] * (cons + pen)
                           + alpha[:, :, None, None, None] * coh)
            blk = {}
            for s_name in ("m", "p"):
                _, ph_s, _, _, _, sg_s = side[s_name]
                for t_name in ("m", "p"):
                    blk[s_name + t_name] = sg_s * np.einsum(
                        "fq,fqa,fqbji->faibj", W, ph_s, X[t_name]).reshape(len(F), bu, bu)
            np.add.at(A_diag, em, blk["mm"])
            np.add.at(A_diag, ep, blk["pp"])
            A_mp[F] = blk["mp"]
            A_pm[F] = blk["pm"]

        if not np.any(act):
            continue
        # ---------------- fluid terms on faces with beta = 1 -------------------
        Fa = np.nonzero(act)[0]
        pn = itf.face_pnodes[slot[Fa]]                           # (Fa, nnf)
        Gi = m.face_Ginv[F[Fa]]                                  # (Fa, d-1, d-1)
        gp = np.einsum("qks,fk->fqs", m.deta_dst, p[pn])         # grad_st p_h
        gp_geta = np.einsum("fqs,fst,qkt->fqk", gp, Gi, m.deta_dst)
        geta_geta = np.einsum("qls,fst,qkt->fqlk", m.deta_dst, Gi, m.deta_dst)
        wa = w[Fa]
        Kw, dK = conductivity(wa, prm.mu)
        Wa = W[Fa]
        wo = w_old[F[Fa]]
        rp = s_p * np.einsum("fq,fqk->fk", Wa, Kw[..., None] * gp_geta
                             + ((wa - wo) / prm.dt)[..., None] * m.eta[None])
        np.add.at(R_p, pn, rp)
        if jacobian:
            na = n[Fa]
            for name in ("m", "p"):
                e_s, ph, _, _, _, sg = side[name]
                phs = ph[Fa]
                # B: d tau / d p_k = -beta eta_k n ; tested by sg phi_a
                bv = -sg * np.einsum("fq,fqa,qk,fi->faik", Wa, phs, m.eta, na)
                rows = ((e_s[Fa][:, None, None] * nn + np.arange(nn)[None, :, None]) * d
                        + np.arange(d)[None, None, :])           # (Fa, nn, d)
                rr = np.broadcast_to(rows[..., None], bv.shape)
                cc = np.broadcast_to(pn[:, None, None, :], bv.shape)
                Bt.append((rr.ravel(), cc.ravel(), bv.ravel()))
                # C: d R_p,k / d u  (trial on side sg)
                cv = s_p * sg * np.einsum("fq,fqk,fqb,fj->fkbj", Wa,
                                          dK[..., None] * gp_geta + m.eta[None] / prm.dt,
                                          phs, na)
                rr = np.broadcast_to(pn[:, :, None, None], cv.shape)
                cc = np.broadcast_to(rows[:, None, :, :], cv.shape)
                Ct.append((rr.ravel(), cc.ravel(), cv.ravel()))
            dv = s_p * np.einsum("fq,fqlk->fkl", Wa, Kw[..., None, None] * geta_geta)
            rr = np.broadcast_to(pn[:, :, None], dv.shape)
            cc = np.broadcast_to(pn[:, None, :], dv.shape)
            Dt.append((rr.ravel(), cc.ravel(), dv.ravel()))

    for node, q0 in zip(src_pnode, src_q0):
        R_p[node] -= s_p * q0
    R_u = Ru3.reshape(-1)

    # ---------------- strong Dirichlet rows ------------------------------------
    cl = m.clamped_dof
    ub = np.zeros(m.n_u) if ubar is None else ubar
    R_u = R_u.copy()
    R_u[cl] = u[cl] - ub[cl]
    sysm = System(R_u=R_u, R_p=R_p)
    if not jacobian:
        return sysm
    clb = cl.reshape(m.ne, bu)
    for e, r in zip(*np.nonzero(clb)):
        A_diag[e, r, :] = 0.0
        A_diag[e, r, r] = 1.0
    rows_m = clb[m.face_em]                                      # (nf, bu)
    rows_p = clb[m.face_ep]
    A_mp[rows_m] = 0.0
    A_pm[rows_p] = 0.0

    def coo(tr, shape):
        if not tr:
            return sp.csr_matrix(shape)
        r = np.concatenate([t[0] for t in tr]); c = np.concatenate([t[1] for t in tr])
        v = np.concatenate([t[2] for t in tr])
        return sp.coo_matrix((v, (r, c)), shape=shape).tocsr()

    Bm = coo(Bt, (m.n_u, n_p))
    if n_p:   # Dirichlet rows of B are zero
        row_of = np.repeat(np.arange(m.n_u), np.diff(Bm.indptr))
        Bm.data[cl[row_of]] = 0.0
        Bm.eliminate_zeros()
    sysm.A_diag, sysm.A_mp, sysm.A_pm = A_diag, A_mp, A_pm
    sysm.B = Bm
    sysm.C = coo(Ct, (n_p, m.n_u))
    sysm.D = coo(Dt, (n_p, n_p))
    return sysm


def bsr_A(mesh: Mesh, sysm: System) -> sp.bsr_matrix:
    """The displacement block A as a block-sparse matrix (element blocks)."""
    m = mesh
    rows = np.concatenate([np.arange(m.ne), m.face_em, m.face_ep])
    cols = np.concatenate([np.arange(m.ne), m.face_ep, m.face_em])
    data = np.concatenate([sysm.A_diag, sysm.A_mp, sysm.A_pm])
    order = np.lexsort((cols, rows))
    indptr = np.zeros(m.ne + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    return sp.bsr_matrix((data[order], cols[order], indptr), shape=(m.n_u, m.n_u))


def full_matrix(mesh: Mesh, sysm: System) -> sp.csr_matrix:
    """J = [[A, B], [C, D]] as one sparse matrix."""
    A = bsr_A(mesh, sysm).tocsr()
    return sp.bmat([[A, sysm.B], [sysm.C, sysm.D]], format="csr")
