"""Fracture and fluid activation on the GPU (hf_get_interface_traction,
hf_detect_activation, the propagation driver) against the oracle's
``activation`` module.

* The DG normal traction at every face point matches the oracle's at random
  states on 2D/3D, P1/P2 meshes (1e-12 of the largest traction).
* The new interface states match the oracle's decisions exactly, from random
  states and random interface states (so that both rules fire).
* Three load steps of a propagating 2D crack (points turning cohesive after
  each step, a new context built with the new states) match the oracle's
  run: the same activation counts, states to 1e-8.
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import activation, newton
from oracle.newton import Case

pytestmark = pytest.mark.gpu

import paper_1911_10275_amd as hf  # noqa: E402  (a broken package fails, never skips)
from paper_1911_10275_amd.propagation import Propagation  # noqa: E402

SMALL = {
    "2d_p1": lambda: synth.kgd_small(9, 1, steps=2),
    "2d_p2": lambda: synth.kgd_small(7, 2, steps=2),
    "3d_p1": lambda: synth.penny_small(4, 1, steps=2),
    "3d_p2": lambda: synth.penny_small(4, 2, steps=2),
}


def _random(case, seed):
    m = case.mesh
    rng = np.random.default_rng(seed)
    return rng.normal(size=m.n_u) * 1e-3, rng.uniform(0.0, 2e-3, case.itf.n_p), np.zeros((m.nf, m.nq))


@pytest.mark.parametrize("name", list(SMALL))
def test_interface_traction_parity(name):
    prob = SMALL[name]()
    case = Case.from_problem(prob)
    ctx = hf.context_for_problem(prob)
    for seed in (1, 2):
        u, p, wo = _random(case, seed)
        ctx.set_state(u, p, wo)
        got = ctx.interface_traction()
        want = activation.dg_normal_traction(case, u)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    ctx.close()


@pytest.mark.parametrize("name", list(SMALL))
def test_detect_activation_matches_oracle(name):
    prob = SMALL[name]()
    base = Case.from_problem(prob)
    m = base.mesh
    rng = np.random.default_rng(9)
    # random interface states: intact, cohesive and traction-free points, some
    # faces fully open without fluid (candidates for the fluid rule)
    qp = rng.integers(0, 3, size=(m.nf, m.nq)).astype(np.uint8)
    open_faces = rng.random(m.nf) < 0.3
    qp[open_faces] = rng.integers(1, 3, size=(open_faces.sum(), m.nq)).astype(np.uint8)
    beta = base.itf.beta.copy()
    case = activation.rebuild(base, qp, beta)
    ctx = hf.Context(b_stab=10.0)
    ctx.upload_mesh(prob.dim, prob.order, prob.xyz, prob.elem, prob.dirichlet_vert)
    ctx.upload_interfaces(qp, beta)
    mt = dataclasses.replace(prob.material, sigma_c=2e-4, G_c=2e-4 * 1e-4 / 2)  # delta_c = 1e-4
    ctx.set_material(mt.E, mt.nu, mt.sigma_c, mt.G_c, mt.mu, mt.dt)
    ctx.set_injection(np.asarray(prob.src_vert), np.asarray(prob.src_q0))
    ctx.finalize()
    case = dataclasses.replace(case, prm=dataclasses.replace(case.prm, sigma_c=mt.sigma_c, G_c=mt.G_c))
    u = rng.normal(size=m.n_u) * 1e-3
    ctx.set_state(u, np.zeros(case.itf.n_p), np.zeros((m.nf, m.nq)))
    q_g, b_g, na_g, nb_g = ctx.detect_activation()
    ctx.close()
    q_o, b_o, na_o, nb_o = activation.detect(case, u)
    np.testing.assert_array_equal(q_g, q_o)
    np.testing.assert_array_equal(b_g, b_o)
    assert (na_g, nb_g) == (na_o, nb_o) and na_o > 0 and nb_o > 0


def test_propagation_matches_oracle():
    mat = synth.Material(E=1.0, nu=0.25, sigma_c=1e-2, G_c=1e-5, mu=1e-3, dt=1.0)
    prob = synth.kgd_problem(12, 1, 3, mat, 1e-4, half_length=0.2, ring=1, load_steps=3)
    ref = activation.run(Case.from_problem(prob), 3, solver="dense")
    drv = Propagation(prob, two_level=1)
    drv.start()
    for k, (case, st, ns_ref, na, nb) in enumerate(ref):
        ns, na_g, nb_g = drv.load_step()
        assert ns.converged and ns.lin.true_relres <= 1e-10, k
        assert (na_g, nb_g) == (na, nb), k
        u, p, _, wo = drv.ctx.get_state()
        assert np.linalg.norm(u - st.u) <= 1e-8 * np.linalg.norm(st.u), k
        assert np.linalg.norm(p - st.p) <= 1e-8 * np.linalg.norm(st.p), k
    drv.close()
    assert sum(na for *_, na, _ in ref) > 0
