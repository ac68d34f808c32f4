"""Newton-Raphson on the monolithic system and the given-length load-step
driver (oracle).

Sec. "Computational framework": the linearised system is solved at every
nonlinear iteration, starting from the previous time step's fields;
convergence is judged on the Euclidean norms of the relative increments of
both nodal arrays; the fluid flag beta is only updated at the end of a time
step.  In the given-crack-length mode of Sec. "Verification of the
fully-coupled algorithm" neither alpha nor beta changes, and the previous
opening w^n enters eq. (discreteLubrication) as a fixed source.

Readings (the paper gives no values):
  * tolerance 1e-10 on ||dU|| <= tol ||U|| and ||dP|| <= tol ||P|| (an
    absolute test when the norm is zero), at most 25 iterations;
  * first step starts from u = 0 and p = sigma_c on every active node;
  * optional cut-off p <= p_v -> p_v after each update (off by default);
  * fluid-row scale s_p (see ``fluid_scale``).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import shapes
from .assemble import Params, assemble
from .mesh import Interfaces, Mesh
from .solve import BlockJacobi, Operator, SolveStats, dense_solve, gmres, gmres_ir


@dataclasses.dataclass
class Case:
    mesh: Mesh
    itf: Interfaces
    prm: Params
    src_pnode: np.ndarray
    src_q0: np.ndarray

    @classmethod
    def from_problem(cls, prob, flip_labels: bool = False, b_stab: float = 10.0):
        mesh = Mesh(prob.dim, prob.order, prob.xyz, prob.elem, prob.dirichlet_vert,
                    flip_labels=flip_labels)
        itf = Interfaces(mesh, prob.crack_faces, prob.crack_state, prob.crack_beta)
        mt = prob.material
        prm = Params(mt.E, mt.nu, mt.sigma_c, mt.G_c, mt.mu, mt.dt, b_stab)
        src = np.array([itf.p_node_of_vertex(v) for v in prob.src_vert], dtype=np.int64)
        return cls(mesh, itf, prm, src, np.asarray(prob.src_q0, dtype=np.float64))


@dataclasses.dataclass
class State:
    u: np.ndarray          # (n_u,)
    p: np.ndarray          # (n_p,)
    w_old: np.ndarray      # (nf, nq)
    s_p: float
    w_max: Optional[np.ndarray] = None   # (nf, nq) unloading history, or None (envelope only)


def opening(mesh: Mesh, u: np.ndarray) -> np.ndarray:
    """w = [[u]] . n at every interior-face integration point (nf, nq)
    (eq. displacementJump)."""
    m = mesh
    ue = u.reshape(m.ne, m.nn, m.dim)
    um = np.einsum("fqa,fai->fqi", shapes.phi(m.face_lam_m, m.dim, m.order), ue[m.face_em])
    up = np.einsum("fqa,fai->fqi", shapes.phi(m.face_lam_p, m.dim, m.order), ue[m.face_ep])
    return np.einsum("fqi,fi->fq", up - um, m.normal)


def fluid_scale(case: Case, w_old: np.ndarray, u: Optional[np.ndarray] = None) -> float:
    """Fluid-row scale s_p = 12 mu (L / w_ref)^3.

    A reading of the paper's (unpublished) remark on bringing the fluid
    equations to the units of the solid ones with c^n = 12 mu (L/max w^n)^3:
    L is the largest bounding-box extent of the mesh and w_ref is the
    largest opening of the state a load step starts from, over the fluid
    faces' points: the larger of w^n and, when the start displacement u is
    given, its own opening w(u) (the elastic predictor opens the crack
    before w^n does at the first load step), floored at 0.01 delta_c so that
    it is defined for a closed crack.  Fixed for a load step."""
    m, itf = case.mesh, case.itf
    L = float(np.max(m.xyz.max(axis=0) - m.xyz.min(axis=0)))
    fa = itf.active_faces
    wmax = float(np.max(w_old[fa])) if len(fa) else 0.0
    if u is not None and len(fa):
        wmax = max(wmax, float(np.max(opening(m, u)[fa])))
    w_ref = max(wmax, 0.01 * case.prm.delta_c)
    return 12.0 * case.prm.mu * (L / w_ref) ** 3


def initial_state(case: Case, predictor: bool = False) -> State:
    """Start of the load sequence: w_old = 0 and either u = 0, p = sigma_c,
    or (predictor) the uniform-pressure elastic state: with the pressure held
    at 1 on every node the displacement equations give u1 (direct sparse
    solve), V1 = crack volume of u1 on the fluid faces, p0 = sum(Q0) dt / V1,
    u = p0 u1, p = p0.  The paper starts its given-length test from uniform
    pressure and opening; the predictor is the elastically compatible form
    of such a start (a reading)."""
    m = case.mesh
    w0 = np.zeros((m.nf, m.nq))
    st = State(u=np.zeros(m.n_u), p=np.full(case.itf.n_p, case.prm.sigma_c), w_old=w0,
               s_p=fluid_scale(case, w0))
    q = float(np.sum(case.src_q0))
    if not predictor or case.itf.n_p == 0 or q <= 0.0:
        return st
    import scipy.sparse.linalg as spla
    from .assemble import bsr_A
    S = assemble(m, case.itf, case.prm, np.zeros(m.n_u), np.ones(case.itf.n_p), w0, st.s_p,
                 case.src_pnode, case.src_q0)
    u1 = spla.spsolve(bsr_A(m, S).tocsc(), -S.R_u)
    fa = case.itf.active_faces
    V1 = float(np.sum(m.fq_w[None, :] * m.area[fa][:, None] * opening(m, u1)[fa]))
    p0 = q * case.prm.dt / V1
    u0 = p0 * u1
    return State(u=u0, p=np.full(case.itf.n_p, p0), w_old=w0, s_p=fluid_scale(case, w0, u0))


@dataclasses.dataclass
class NewtonStats:
    iterations: int = 0
    converged: bool = False
    linear_iterations: int = 0
    ir_steps: int = 0
    max_true_relres: float = 0.0
    du_rel: list = dataclasses.field(default_factory=list)
    dp_rel: list = dataclasses.field(default_factory=list)
    res_norm: list = dataclasses.field(default_factory=list)


def linear_solve(case: Case, sysm, solver: str, m: int, rtol: float, maxit: int,
                 rtol_inner: float = 1e-2):
    b = -sysm.R
    if solver == "dense":
        return dense_solve(case.mesh, sysm, b), SolveStats(converged=True, true_relres=0.0)
    op = Operator(case.mesh, sysm)
    if solver == "gmres":
        return gmres(op, b, BlockJacobi(case.mesh, sysm), m=m, rtol=rtol, maxit=maxit)
    if solver == "ir":
        op32 = Operator(case.mesh, sysm, dtype=np.float32)
        pc32 = BlockJacobi(case.mesh, sysm, dtype=np.float32)
        return gmres_ir(op, op32, pc32, b, m=m, rtol=rtol, rtol_inner=rtol_inner,
                        maxit=maxit)
    raise ValueError(solver)


def newton_solve(case: Case, state: State, solver: str = "gmres", tol: float = 1e-10,
                 maxit: int = 25, m: int = 60, rtol: float = 1e-10, lin_maxit: int = 20000,
                 cutoff: Optional[float] = None, rtol_inner: float = 1e-2):
    """Newton iterations for one load step from ``state``; returns the
    converged (u, p) as a new State (w_old and s_p unchanged) and stats."""
    u, p = state.u.copy(), state.p.copy()
    ns = NewtonStats()
    for k in range(maxit):
        sysm = assemble(case.mesh, case.itf, case.prm, u, p, state.w_old, state.s_p,
                        case.src_pnode, case.src_q0, w_max=state.w_max)
        ns.res_norm.append(float(np.linalg.norm(sysm.R)))
        dx, ls = linear_solve(case, sysm, solver, m, rtol, lin_maxit, rtol_inner)
        ns.linear_iterations += ls.iterations
        ns.ir_steps += ls.ir_steps
        ns.max_true_relres = max(ns.max_true_relres, ls.true_relres)
        if not ls.converged:
            ns.iterations = k + 1
            return State(u, p, state.w_old, state.s_p, state.w_max), ns
        du, dp = dx[:case.mesh.n_u], dx[case.mesh.n_u:]
        u = u + du
        p = p + dp
        if cutoff is not None:
            p = np.maximum(p, cutoff)
        nu, npn = np.linalg.norm(u), np.linalg.norm(p)
        ru = np.linalg.norm(du) / nu if nu > 0 else np.linalg.norm(du)
        rp = (np.linalg.norm(dp) / npn if npn > 0 else np.linalg.norm(dp)) if p.size else 0.0
        ns.du_rel.append(float(ru)); ns.dp_rel.append(float(rp))
        ns.iterations = k + 1
        if ru <= tol and rp <= tol:
            ns.converged = True
            break
    return State(u, p, state.w_old, state.s_p, state.w_max), ns


def end_load_step(case: Case, state: State) -> State:
    """w^n <- w(u) at the face points; s_p recomputed (alpha, beta frozen);
    with an unloading history, w_max <- max(w_max, w) at every face point
    (only the cohesive points use it)."""
    w = opening(case.mesh, state.u)
    wm = None if state.w_max is None else np.maximum(state.w_max, w)
    return State(state.u, state.p, w, fluid_scale(case, w), wm)


def run(case: Case, steps: int, predictor: bool = False, **kw):
    """Given-length load-step loop; returns the list of converged states and
    Newton statistics."""
    st = initial_state(case, predictor)
    out = []
    for _ in range(steps):
        st, ns = newton_solve(case, st, **kw)
        if not ns.converged:
            out.append((st, ns))
            break
        st = end_load_step(case, st)
        out.append((st, ns))
    return out


def staggered_step(case: Case, state: State, dir_node: int, dir_value: float = 0.0):
    """One iteration of the staggered (sequential) scheme of Sec. "Fully-coupled
    vs. staggered hydro-mechanics with applied inflow boundary conditions":
    each field is solved from its own equation with the other field taken
    from the previous iteration, i.e. the decoupled forms A U = E - B P and
    D P = F - C U of the linear system of eq. (fully-coupled-fully-discrete).

    1. Solid: with the pressure held, A dU = -R_u(U, P), U <- U + dU (A is
       the displacement block, dR_u/dU: one solve for the linear solid; a
       Newton sub-step where cohesive tractions make it nonlinear).
    2. Fluid: with the new opening held, D dP = -R_p(U, P), P <- P + dP.
       D = dR_p/dP is the Poiseuille flux operator alone (the storage term
       depends on the opening only), so the decoupled fluid equation is
       elliptic and needs an essential condition: the row of pressure node
       ``dir_node`` is replaced by P[dir_node] = dir_value.  Faces that
       are closed (w <= 0: no conductivity) can leave parts of the crack
       without a fixed pressure; the decoupled block is then singular
       (numpy.linalg.LinAlgError).

    Returns the new State and the increments (dU, dP)."""
    import scipy.sparse.linalg as spla
    from .assemble import bsr_A
    m = case.mesh
    S = assemble(m, case.itf, case.prm, state.u, state.p, state.w_old, state.s_p,
                 case.src_pnode, case.src_q0, w_max=state.w_max)
    du = spla.spsolve(bsr_A(m, S).tocsc(), -S.R_u)
    u = state.u + du
    S = assemble(m, case.itf, case.prm, u, state.p, state.w_old, state.s_p,
                 case.src_pnode, case.src_q0, w_max=state.w_max)
    D = S.D.toarray()
    r = S.R_p.copy()
    D[dir_node, :] = 0.0
    D[dir_node, dir_node] = 1.0
    r[dir_node] = state.p[dir_node] - dir_value
    dp = np.linalg.solve(D, -r)
    return State(u, state.p + dp, state.w_old, state.s_p, state.w_max), du, dp
