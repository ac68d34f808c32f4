"""Fracture and fluid activation at the end of a load step (oracle; test
infrastructure, imported only by tests, smoke checks and the benchmark's CPU
baseline).

Sec. "Governing equations" / discretisation: the factor alpha switches an
interface integration point from the DG terms to the traction-separation law
once the traction the DG method exchanges there reaches sigma_c
(eq. fractureActivation, irreversible: the maximum over the history), and the
binary fluid field beta switches a face to the fluid domain once its opening
exceeds the threshold (eq. fluidActivation with the threshold delta_c);
beta is only changed at the end of a time step (Sec. "Computational
framework").

Readings (the paper prints both criteria only in its unpublished text):
  * the DG traction at an intact point is the numerical flux of the
    consistency and stabilisation terms, t = {sigma(u)} n + (b/h_f) Chat(n) [[u]],
    and its normal part t.n is compared with sigma_c;
  * the check runs on the converged state of a load step; an activated point
    becomes state 1 (cohesive) with beta unchanged;
  * a face becomes a fluid face when the opening at any of its points
    exceeds delta_c, and only faces already cohesive or traction-free there
    (state >= 1 at every point) are eligible (the fluid enters open cracks).
"""
from __future__ import annotations

import numpy as np

from . import shapes
from .assemble import _stress
from .newton import Case, opening


def dg_normal_traction(case: Case, u: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """t.n = n.{sigma(u)} n + (b/h_f)(lambda + 2G) [[u]].n at every face point
    (nf, nq); the stabilisation's normal part is n.Chat(n)[[u]] =
    (lambda + 2G) w since Chat(n) n = (lambda + 2G) n."""
    m, prm = case.mesh, case.prm
    d = m.dim
    lam, G = prm.lame
    ue = u.reshape(m.ne, m.nn, d)
    out = np.empty((m.nf, m.nq))
    w = opening(m, u)
    for c0 in range(0, m.nf, chunk):
        F = np.arange(c0, min(c0 + chunk, m.nf))
        n = m.normal[F]
        sn = np.zeros((len(F), m.nq, d))
        for e_s, lam_s in ((m.face_em[F], m.face_lam_m[F]), (m.face_ep[F], m.face_lam_p[F])):
            dph = shapes.dphi_dlam(lam_s, d, m.order)                  # (F, nq, nn, d+1)
            gph = np.einsum("fqak,fkx->fqax", dph, m.grad_lam[e_s])    # (F, nq, nn, d)
            gU = np.einsum("fai,fqax->fqix", ue[e_s], gph)
            sn += 0.5 * np.einsum("fqix,fx->fqi", _stress(gU, lam, G), n)
        tn = np.einsum("fqi,fi->fq", sn, n)
        out[F] = tn + (prm.b_stab / m.hf[F])[:, None] * (lam + 2.0 * G) * w[F]
    return out


def detect(case: Case, u: np.ndarray):
    """New (qp_state, beta) after the activation checks at displacement u, and
    the counts of newly activated points and faces."""
    itf, prm = case.itf, case.prm
    qp = itf.qp_state.copy()
    beta = itf.beta.copy()
    tn = dg_normal_traction(case, u)
    new_alpha = (qp == 0) & (tn > prm.sigma_c)
    qp[new_alpha] = 1
    w = opening(case.mesh, u)
    eligible = (beta == 0) & np.all(qp >= 1, axis=1)
    new_beta = eligible & np.any(w > prm.delta_c, axis=1)
    beta[new_beta] = 1
    return qp, beta, int(new_alpha.sum()), int(new_beta.sum())


def rebuild(case: Case, qp_state: np.ndarray, beta: np.ndarray) -> Case:
    """The same mesh, material and injection with new interface states (the
    pressure unknowns follow beta)."""
    from .mesh import Interfaces
    itf = Interfaces(case.mesh, qp_state=qp_state, beta=beta)
    src_v = [case.itf.p_keys[i][1] for i in case.src_pnode]
    src = np.array([itf.p_node_of_vertex(v) for v in src_v], dtype=np.int64)
    return Case(case.mesh, itf, case.prm, src, case.src_q0)


def carry_pressure(old: Case, p: np.ndarray, new: Case) -> np.ndarray:
    """Pressure on the new pressure nodes: kept where a node existed; a new
    node (the crack front's) starts at the lowest existing pressure (a
    reading: the paper does not say how the fluid enters a new face)."""
    index = old.itf.p_index
    low = float(p.min()) if p.size else 0.0
    return np.array([p[index[k]] if k in index else low for k in new.itf.p_keys])


def run(case: Case, steps: int, predictor: bool = True, **kw):
    """Load steps with activation: each converged load step ends with
    w^n <- w(u), then the activation checks; when states change the case is
    rebuilt with them, the pressure carried over and the fluid-row scale
    recomputed from the state (the next load step starts there).  Returns
    [(case, state, NewtonStats, points activated, faces made fluid)]."""
    from .newton import State, end_load_step, fluid_scale, initial_state, newton_solve
    state = initial_state(case, predictor=predictor)
    out = []
    for _ in range(steps):
        state, ns = newton_solve(case, state, **kw)
        if not ns.converged:
            out.append((case, state, ns, 0, 0))
            break
        state = end_load_step(case, state)
        qp, beta, na, nb = detect(case, state.u)
        if na or nb:
            new = rebuild(case, qp, beta)
            p = carry_pressure(case, state.p, new)
            state = State(state.u, p, state.w_old, fluid_scale(new, state.w_old, state.u), state.w_max)
            case = new
        out.append((case, state, ns, na, nb))
    return out
