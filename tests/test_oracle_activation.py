"""Activation checks of the oracle (eq. fractureActivation, eq. fluidActivation).

* The DG normal traction of a continuous linear displacement field is the
  normal traction of its uniform stress, computed here from the engineering
  constants in the plane-strain and 3D forms (no DG jump, no stabilisation).
* A rigid opening across a row of intact faces gives the stabilisation's
  normal traction (b/h_f) M w with the P-wave modulus M = E(1-nu)/((1+nu)(1-2nu)).
* detect() switches exactly the intact points above sigma_c and the eligible
  faces (all points cohesive or traction-free, no fluid yet) with an opening
  above delta_c at some point.
* The propagation driver rebuilds the case with the new states and keeps the
  pressure of existing nodes.
"""
import numpy as np
import pytest

import synth
from oracle import activation, newton
from oracle.mesh import Interfaces, Mesh
from oracle.newton import Case


def _case(dim, order, n, E=1.0, nu=0.25, sigma_c=1e-3):
    mat = synth.Material(E=E, nu=nu, sigma_c=sigma_c, G_c=1e-4, mu=1e-3, dt=1.0)
    if dim == 2:
        prob = synth.kgd_problem(n, order, 7, mat, 1e-4, half_length=0.2, ring=1, load_steps=1)
    else:
        prob = synth.penny_problem(n, order, 7, mat, 1e-4, radius=0.3, ring_width=0.2, load_steps=1)
    return Case.from_problem(prob)


def _linear_field(m, Eps):
    x = m.node_xyz().reshape(m.ne * m.nn, m.dim)
    return (x @ Eps.T).reshape(-1)


def _uniform_stress(dim, E, nu, Eps):
    e = 0.5 * (Eps + Eps.T)
    if dim == 2:   # plane strain, engineering form
        c = E / ((1 + nu) * (1 - 2 * nu))
        s11 = c * ((1 - nu) * e[0, 0] + nu * e[1, 1])
        s22 = c * (nu * e[0, 0] + (1 - nu) * e[1, 1])
        s12 = E / (1 + nu) * e[0, 1]
        return np.array([[s11, s12], [s12, s22]])
    c = E / ((1 + nu) * (1 - 2 * nu))
    S = np.empty((3, 3))
    for i in range(3):
        S[i, i] = c * ((1 - nu) * e[i, i] + nu * (np.trace(e) - e[i, i]))
        for j in range(3):
            if i != j:
                S[i, j] = E / (1 + nu) * e[i, j]
    return S


@pytest.mark.parametrize("dim,order,n", [(2, 1, 8), (2, 2, 6), (3, 1, 4), (3, 2, 4)])
def test_dg_traction_of_a_uniform_stress(dim, order, n):
    case = _case(dim, order, n)
    m = case.mesh
    Eps = np.random.default_rng(3).normal(size=(dim, dim)) * 1e-3
    u = _linear_field(m, Eps)
    tn = activation.dg_normal_traction(case, u)
    S = _uniform_stress(dim, case.prm.E, case.prm.nu, Eps)
    want = np.einsum("fi,ij,fj->f", m.normal, S, m.normal)
    np.testing.assert_allclose(tn, np.repeat(want[:, None], m.nq, axis=1), rtol=0,
                               atol=1e-12 * np.abs(S).max())


def test_dg_traction_of_a_rigid_opening():
    n, jc = 6, 3
    xyz, elem, _ = synth.grid2d(n, 5, keep_row=jc)
    m = Mesh(2, 1, xyz, elem, np.zeros(len(xyz), np.uint8))
    itf = Interfaces(m)
    prm_mat = synth.Material(E=2.0, nu=0.3, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=1.0)
    from oracle import assemble as asm
    prm = asm.Params(prm_mat.E, prm_mat.nu, prm_mat.sigma_c, prm_mat.G_c, prm_mat.mu, prm_mat.dt)
    case = Case(m, itf, prm, np.zeros(0, np.int64), np.zeros(0))
    upper = xyz[elem].mean(axis=1)[:, 1] > jc / n
    w0 = 1e-3
    u = np.zeros((m.ne, m.nn, 2))
    u[upper, :, 1] = w0
    u = u.reshape(-1)
    tn = activation.dg_normal_traction(case, u)
    M = prm.E * (1 - prm.nu) / ((1 + prm.nu) * (1 - 2 * prm.nu))
    cut = upper[m.face_em] != upper[m.face_ep]
    assert cut.sum() == n
    w = newton.opening(m, u)
    np.testing.assert_allclose(np.abs(w[cut]), w0, rtol=1e-13)
    want = prm.b_stab / m.hf[cut] * M * w[cut, 0]
    np.testing.assert_allclose(tn[cut], np.repeat(want[:, None], m.nq, axis=1), rtol=1e-12)
    np.testing.assert_allclose(tn[~cut], 0.0, atol=1e-15)


def test_detect_thresholds():
    case = _case(2, 1, 12)
    m, itf, prm = case.mesh, case.itf, case.prm
    rng = np.random.default_rng(4)
    u = rng.normal(size=m.n_u) * 1e-3
    tn = activation.dg_normal_traction(case, u)
    w = newton.opening(m, u)
    qp, beta, na, nb = activation.detect(case, u)
    intact = itf.qp_state == 0
    assert np.array_equal(qp[intact] == 1, tn[intact] > prm.sigma_c)
    assert np.array_equal(qp[~intact], itf.qp_state[~intact])
    assert na == int(np.sum(intact & (tn > prm.sigma_c)))
    elig = (itf.beta == 0) & np.all(qp >= 1, axis=1)
    assert np.array_equal(beta == 1, (itf.beta == 1) | (elig & np.any(w > prm.delta_c, axis=1)))
    assert nb == int(np.sum(elig & np.any(w > prm.delta_c, axis=1)))
    assert na > 0


def test_propagation_driver_carries_pressure():
    mat = synth.Material(E=1.0, nu=0.25, sigma_c=1e-2, G_c=1e-5, mu=1e-3, dt=1.0)
    prob = synth.kgd_problem(12, 1, 3, mat, 1e-4, half_length=0.2, ring=1, load_steps=4)
    case = Case.from_problem(prob)
    out = activation.run(case, 3, solver="dense")
    assert all(ns.converged for _, _, ns, _, _ in out)
    assert sum(na for *_, na, _ in out) > 0
    # the rebuilt case holds the new states and the same pressure numbering
    (c1, s1, _, na1, _), (c2, s2, _, na2, _) = out[0], out[1]
    assert np.sum(c2.itf.qp_state >= 1) == np.sum(c1.itf.qp_state >= 1) + na2


def test_dg_traction_averages_the_two_sides():
    """u_y = e1 (y - y_c) above a grid row and e2 (y - y_c) below it: continuous
    across the row (no jump), uniaxial strains e1 and e2 on the two sides, so
    the traction exchanged on the row is the mean M (e1 + e2) / 2."""
    n, jc = 6, 3
    xyz, elem, _ = synth.grid2d(n, 5, keep_row=jc)
    m = Mesh(2, 2, xyz, elem, np.zeros(len(xyz), np.uint8))
    from oracle import assemble as asm
    prm = asm.Params(1.5, 0.2, 1e-3, 1e-4, 1e-3, 1.0)
    case = Case(m, Interfaces(m), prm, np.zeros(0, np.int64), np.zeros(0))
    yc = jc / n
    upper = xyz[elem].mean(axis=1)[:, 1] > yc
    e1, e2 = 2e-3, -5e-4
    x = m.node_xyz()
    u = np.zeros((m.ne, m.nn, 2))
    u[..., 1] = np.where(upper[:, None], e1, e2) * (x[..., 1] - yc)
    tn = activation.dg_normal_traction(case, u.reshape(-1))
    M = prm.E * (1 - prm.nu) / ((1 + prm.nu) * (1 - 2 * prm.nu))
    cut = upper[m.face_em] != upper[m.face_ep]
    np.testing.assert_allclose(tn[cut], 0.5 * M * (e1 + e2), rtol=1e-11)
