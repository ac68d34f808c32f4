"""Oracle pins: DG patch test, finite-difference Jacobian, label /
translation / rotation invariance (no GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assemble as asm
from oracle import newton
from oracle.mesh import Interfaces, Mesh
from oracle.newton import Case


def _mesh(dim, order, n, seed=3, clamp=True):
    if dim == 2:
        xyz, elem, grid = synth.grid2d(n, seed)
    else:
        xyz, elem, grid = synth.kuhn3d(n, seed)
    dv = synth.boundary_vertices(grid, n) if clamp else np.zeros(len(xyz), np.uint8)
    return Mesh(dim, order, xyz, elem, dv)


@pytest.mark.parametrize("dim,order,n", [(2, 1, 4), (2, 2, 3), (3, 1, 2), (3, 2, 2)])
def test_patch_test_linear_field(dim, order, n):
    """alpha = 0 everywhere and u = ubar = G x + c on the clamped boundary:
    the discrete solution is the linear field itself and R(u_lin) = 0."""
    m = _mesh(dim, order, n)
    itf = Interfaces(m)
    prm = asm.Params(1.3, 0.27, 1e-3, 1e-4, 1e-3, 1.0)
    rng = np.random.default_rng(7)
    Gm = rng.normal(size=(dim, dim)); c = rng.normal(size=dim)
    u_lin = (m.node_xyz() @ Gm.T + c).reshape(-1)
    wo = np.zeros((m.nf, m.nq))
    S = asm.assemble(m, itf, prm, u_lin, np.zeros(0), wo, 1.0, [], [], ubar=u_lin)
    assert np.abs(S.R).max() <= 1e-12 * np.abs(u_lin).max() * prm.E
    S0 = asm.assemble(m, itf, prm, np.zeros(m.n_u), np.zeros(0), wo, 1.0, [], [], ubar=u_lin)
    A = asm.bsr_A(m, S0).tocsc()
    u = spla.spsolve(A, -S0.R_u)
    np.testing.assert_allclose(u, u_lin, atol=1e-10 * np.abs(u_lin).max())


def _random_state(case, seed, scale=0.15):
    m = case.mesh
    rng = np.random.default_rng(seed)
    u = rng.normal(size=m.n_u) * scale
    p = rng.uniform(0.0, 1e-2, case.itf.n_p)
    wo = rng.uniform(0.0, 0.05, (m.nf, m.nq))
    return u, p, wo


def _R(case, u, p, wo, s_p=10.0, jac=False):
    return asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, s_p, case.src_pnode,
                        case.src_q0, jacobian=jac)


def test_fd_jacobian_full_2d_p1():
    case = Case.from_problem(synth.kgd_small(6, 1))
    crack = case.itf.qp_state > 0
    dc = case.prm.delta_c
    for seed in range(200):       # first seeded state that visits every branch of the law
        u, p, wo = _random_state(case, seed)
        w = newton.opening(case.mesh, u)[crack]
        if np.any(w < 0) and np.any((w > 0) & (w < dc)) and np.any(w > dc):
            break
    else:
        raise AssertionError("no seeded state covers every traction-law branch")
    S = _R(case, u, p, wo, jac=True)
    J = asm.full_matrix(case.mesh, S).toarray()
    x = np.concatenate([u, p])
    nu = case.mesh.n_u
    h = 1e-7
    Jfd = np.empty_like(J)
    for k in range(len(x)):
        xp, xm = x.copy(), x.copy()
        xp[k] += h; xm[k] -= h
        Jfd[:, k] = (_R(case, xp[:nu], xp[nu:], wo).R - _R(case, xm[:nu], xm[nu:], wo).R) / (2 * h)
    err = np.abs(J - Jfd).max() / np.abs(J).max()
    assert err < 1e-6
    for blk in (S.B, S.C, S.D):
        assert blk.nnz > 0


def test_fd_jacobian_with_unloading_history():
    """The full finite-difference Jacobian with an unloading history w_max at
    the cohesive points, chosen so that the points visit every branch: the
    secant (0 < w < w_max), closed after unloading (w < 0 < w_max), the
    envelope beyond w_max and a fully softened history (w_max > delta_c)."""
    case = Case.from_problem(synth.kgd_small(6, 1))
    crack = case.itf.qp_state == 1
    dc = case.prm.delta_c
    rng = np.random.default_rng(5)
    for seed in range(200):
        u, p, wo = _random_state(case, seed)
        w = newton.opening(case.mesh, u)
        wm = np.where(rng.uniform(size=w.shape) < 0.6, np.abs(w) + rng.uniform(0.02, 0.3, w.shape),
                      np.abs(w) * rng.uniform(0.2, 0.8, w.shape))
        wc, mc = w[crack], wm[crack]
        if (np.any((wc > 0) & (wc < mc)) and np.any((wc < 0) & (mc > 0)) and np.any(wc > mc)
                and np.any(mc > dc)):
            break
    else:
        raise AssertionError("no seeded state covers every unloading branch")
    R = lambda uu, pp, jac=False: asm.assemble(case.mesh, case.itf, case.prm, uu, pp, wo, 10.0,
                                               case.src_pnode, case.src_q0, jacobian=jac, w_max=wm)
    S = R(u, p, jac=True)
    J = asm.full_matrix(case.mesh, S).toarray()
    x = np.concatenate([u, p])
    nu = case.mesh.n_u
    h = 1e-7
    Jfd = np.empty_like(J)
    for k in range(len(x)):
        xp, xm = x.copy(), x.copy()
        xp[k] += h; xm[k] -= h
        Jfd[:, k] = (R(xp[:nu], xp[nu:]).R - R(xm[:nu], xm[nu:]).R) / (2 * h)
    assert np.abs(J - Jfd).max() / np.abs(J).max() < 1e-6
    # the history changes the cohesive rows (and nothing when it is all zero)
    S0 = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, 10.0, case.src_pnode, case.src_q0)
    Sz = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, 10.0, case.src_pnode, case.src_q0,
                      w_max=np.zeros_like(wm))
    assert np.array_equal(S0.R, Sz.R) and np.abs(S.R - S0.R).max() > 1e-8


@pytest.mark.parametrize("prob", [synth.kgd_small(4, 2), synth.penny_small(4, 2)],
                         ids=["2d_p2", "3d_p2"])
def test_fd_jacobian_directional(prob):
    case = Case.from_problem(prob)
    u, p, wo = _random_state(case, 2)
    S = _R(case, u, p, wo, jac=True)
    J = asm.full_matrix(case.mesh, S)
    x = np.concatenate([u, p])
    nu = case.mesh.n_u
    rng = np.random.default_rng(3)
    h = 1e-7
    for _ in range(4):
        v = rng.normal(size=x.shape)
        fd = (_R(case, (x + h * v)[:nu], (x + h * v)[nu:], wo).R
              - _R(case, (x - h * v)[:nu], (x - h * v)[nu:], wo).R) / (2 * h)
        jv = J @ v
        assert np.abs(jv - fd).max() <= 1e-6 * np.abs(jv).max()
        # fluid rows separately (they are much smaller than the solid rows)
        if case.itf.n_p:
            assert np.abs(jv[nu:] - fd[nu:]).max() <= 1e-6 * np.abs(jv[nu:]).max()


@pytest.mark.parametrize("prob", [synth.kgd_small(6, 1), synth.kgd_small(4, 2),
                                  synth.penny_small(4, 1)],
                         ids=["2d_p1", "2d_p2", "3d_p1"])
def test_label_invariance(prob):
    """Swapping the +/- roles on every interface leaves R and J unchanged."""
    a = Case.from_problem(prob)
    b = Case.from_problem(prob, flip_labels=True)
    assert np.any(a.mesh.face_em != b.mesh.face_em)
    u, p, wo = _random_state(a, 4)
    Sa, Sb = _R(a, u, p, wo, jac=True), _R(b, u, p, wo, jac=True)
    scale = np.abs(Sa.R).max()
    np.testing.assert_allclose(Sa.R, Sb.R, atol=1e-12 * scale)
    Ja = asm.full_matrix(a.mesh, Sa).toarray(); Jb = asm.full_matrix(b.mesh, Sb).toarray()
    np.testing.assert_allclose(Ja, Jb, atol=1e-12 * np.abs(Ja).max())


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 2)])
def test_rigid_motion_invariance(dim, order):
    """No clamped nodes: translations and infinitesimal rotations of every DG
    node copy leave the residual unchanged (cracks included)."""
    prob = synth.kgd_small(6, order) if dim == 2 else synth.penny_small(4, order)
    prob.dirichlet_vert = np.zeros_like(prob.dirichlet_vert)
    case = Case.from_problem(prob)
    u, p, wo = _random_state(case, 5, scale=0.01)
    R0 = _R(case, u, p, wo).R
    X = case.mesh.node_xyz()
    rng = np.random.default_rng(6)
    c = rng.normal(size=dim)
    W = rng.normal(size=(dim, dim)); W = W - W.T
    for du in ((np.zeros_like(X) + c).reshape(-1), (X @ W.T).reshape(-1)):
        R1 = _R(case, u + 1e-3 * du, p, wo).R
        np.testing.assert_allclose(R1, R0, atol=1e-12 * np.abs(R0).max())
