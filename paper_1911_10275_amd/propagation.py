"""Load-step driver with fracture and fluid activation (crack propagation).

After each converged load step (Sec. "Computational framework": the fluid flag
beta is only updated at the end of a time step) the activation checks of eq.
(fractureActivation) and eq. (fluidActivation) run on the GPU
(``hf_detect_activation``).  When they change the interface states, the
fluid unknowns may change with beta, so the driver builds a context with the
new states (``hf_upload_interfaces`` on the same mesh, material and
injection) and carries the state over: u and w^n unchanged, the pressure
kept on the nodes that existed (matched by their ``hf_get_pnodes`` keys), a
new node starting at the lowest existing pressure.  The next load step then
starts from there.  All compute runs in the library; this module only
sequences calls and maps node keys.
"""
from __future__ import annotations

import numpy as np

from . import Context, HF_OK, context_for_problem


def _keys(ctx, inst=0):
    return [tuple(int(x) for x in k) for k in ctx.pnodes(inst)]


class Propagation:
    """One instance through load steps with activation.  ``prob`` as for
    ``context_for_problem``; ``options`` are passed to every context."""

    def __init__(self, prob, b_stab: float = 10.0, **options):
        self.prob, self.b_stab, self.options = prob, b_stab, options
        self.ctx = context_for_problem(prob, b_stab=b_stab, **options)
        self.events = []

    def start(self, predictor: bool = True):
        s = self.ctx.sizes
        self.ctx.set_state(np.zeros(s.n_u), np.full(s.n_p, self.prob.material.sigma_c),
                           np.zeros((s.n_face, s.nq_face)))
        if predictor:
            self.ctx.initial_guess()

    def load_step(self):
        """Newton to convergence, end of the load step, activation checks and,
        if the states changed, the new context.  Returns (NewtonStats, points
        newly cohesive, faces newly fluid)."""
        ns = self.ctx.newton_solve(check=False)
        if ns.status != HF_OK or not ns.converged:
            return ns, 0, 0
        self.ctx.end_load_step()
        qp, beta, na, nb = self.ctx.detect_activation()
        if na or nb:
            self._rebuild(qp, beta)
        self.events.append((na, nb))
        return ns, na, nb

    def _rebuild(self, qp, beta):
        old = self.ctx
        u, p, _, wo = old.get_state()
        old_index = {k: i for i, k in enumerate(_keys(old))}
        prob = self.prob
        new = Context(b_stab=self.b_stab, **self.options)
        new.upload_mesh(prob.dim, prob.order, prob.xyz, prob.elem, prob.dirichlet_vert)
        new.upload_interfaces(qp, beta)
        m = prob.material
        new.set_material(m.E, m.nu, m.sigma_c, m.G_c, m.mu, m.dt)
        new.set_injection(np.asarray(prob.src_vert), np.asarray(prob.src_q0))
        new.finalize()
        low = float(p.min()) if p.size else 0.0
        p_new = np.array([p[old_index[k]] if k in old_index else low for k in _keys(new)])
        new.set_state(u, p_new, wo)
        if self.options.get("cohesive_unloading"):  # the faces keep their unloading history
            new.set_history(old.get_history())
        old.close()
        self.ctx = new

    def close(self):
        self.ctx.close()
