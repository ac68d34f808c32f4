"""Oracle pins of the interface physics against values fixed by the paper and
by closed forms, independent of the oracle's own formulas (no GPU):

* eq. (tsl): the linear softening law starts at the strength sigma_c, ends at
  delta_c and encloses the fracture energy G_c = sigma_c delta_c / 2
  (Sec. "Governing equations", after eq. tsl);
* the balance of cohesive traction and fluid pressure on the lips of a
  crack opened rigidly: a literal pressure, worked out by hand from the law,
  makes the whole residual vanish (pins delta_c, the softening slope and the
  sign of both terms in the assembled residual);
* the cubic law of eq. (lubrication): on a straight crack of uniform opening
  the fluid block is the 1D Laplacian times the Poiseuille conductivity
  w^3 / (12 mu), and a linear pressure drives the Poiseuille flux out of the
  crack ends (literal numbers chosen so that the conductivity is 0.01);
* face geometry and the DG stabilisation of eq. (weakElastoStatics) on
  hand-built two-element meshes with rational coordinates: |f|, n, the
  penalty length h_f = min(|e+|, |e-|) / |f| and the penalty force
  (b / h_f) |f| Chat(n) [[u]] worked out by hand;
* Sneddon's penny crack under uniform pressure (textbook LEFM, not printed
  in the paper): the crack volume of the 3D P2 discretisation lies in the
  band that a coarse mesh in a clamped unit cube allows.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assemble as asm
from oracle import newton, nondim
from oracle.mesh import Interfaces, Mesh
from oracle.newton import Case


# --------------------------------------------------------------------------
# eq. (tsl) on its own
# --------------------------------------------------------------------------
def test_traction_law_envelope():
    """sigma_c = 1e-3, G_c = 1e-4: delta_c must be 0.2 (G_c is the area under
    the linear softening line), T(0+) = sigma_c, T(delta_c) = 0, slope
    -sigma_c / delta_c = -5e-3, zero beyond delta_c; a pre-crack is traction
    free in tension."""
    prm = asm.Params(1.0, 0.25, 1e-3, 1e-4, 1e-3, 1.0)
    assert prm.delta_c == pytest.approx(0.2, rel=1e-15)
    w = np.array([0.0, 0.05, 0.1, 0.2, 0.25, 1.0])
    kc = np.full_like(w, 7.0)
    T, dT = asm.traction_law(np.ones(w.shape, np.uint8), w, prm.sigma_c, prm.delta_c, kc)
    np.testing.assert_allclose(T, [1e-3, 0.75e-3, 0.5e-3, 0.0, 0.0, 0.0], atol=1e-18)
    np.testing.assert_allclose(dT, [-5e-3, -5e-3, -5e-3, -5e-3, 0.0, 0.0], rtol=1e-14)
    # fracture energy: the area under the law up to full separation is G_c
    ws = np.linspace(0.0, 0.3, 30001)
    Ts, _ = asm.traction_law(np.ones(ws.shape, np.uint8), ws, prm.sigma_c, prm.delta_c,
                             np.full_like(ws, 7.0))
    area = float(np.sum(0.5 * (Ts[1:] + Ts[:-1]) * np.diff(ws)))
    assert area == pytest.approx(1e-4, rel=1e-6)
    T2, dT2 = asm.traction_law(np.full(w.shape, 2, np.uint8), w, prm.sigma_c, prm.delta_c, kc)
    assert np.all(T2 == 0.0) and np.all(dT2 == 0.0)


def test_traction_law_unloading_branch():
    """Unloading of a cohesive point (the reading of irreversible linear
    unloading to the origin): sigma_c = 1e-3, delta_c = 0.2, k_c = 1.  With
    w_max = 0.1 (envelope value 0.5e-3) the point unloads on the secant of
    slope 5e-3: T(0.05) = 2.5e-4, T(0) = 0; from w_max on it follows the
    envelope again (T(0.15) = 0.25e-3); a closed face meets the contact
    penalty without the strength offset (T(-0.01) = -0.01); a point beyond
    delta_c has nothing left (secant slope 0); traction-free faces (state 2)
    and points with no history ignore it."""
    sc, dc = 1e-3, 0.2
    w = np.array([0.05, 0.0, 0.1, 0.15, -0.01, 0.1, 0.05, 0.05])
    wm = np.array([0.1, 0.1, 0.1, 0.1, 0.1, 0.3, 0.1, 0.0])
    st = np.array([1, 1, 1, 1, 1, 1, 2, 1])
    T, dT = asm.traction_law(st, w, sc, dc, np.ones_like(w), w_max=wm)
    np.testing.assert_allclose(T, [2.5e-4, 0.0, 0.5e-3, 0.25e-3, -0.01, 0.0, 0.0, 0.75e-3],
                               rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(dT, [5e-3, 5e-3, -5e-3, -5e-3, 1.0, 0.0, 0.0, -5e-3], rtol=1e-14)
    # a point loaded to delta_c and unloaded has dissipated all of G_c =
    # sigma_c delta_c / 2: the area under the envelope up to w_max minus the
    # triangle that unloading along the secant gives back
    for w_m, dissipated in ((0.2, 1e-4), (0.1, 0.75e-4 - 0.25e-4)):
        ws = np.linspace(0.0, w_m, 20001)
        Tl, _ = asm.traction_law(np.ones_like(ws, dtype=int), ws, sc, dc, np.ones_like(ws))
        Tu, _ = asm.traction_law(np.ones_like(ws, dtype=int), ws, sc, dc, np.ones_like(ws),
                                 w_max=np.full_like(ws, w_m))
        work = np.trapezoid(Tl, ws) - np.trapezoid(Tu, ws)
        assert work == pytest.approx(dissipated, rel=1e-8)


# --------------------------------------------------------------------------
# a crack opened rigidly: two bodies separated along a through crack
# --------------------------------------------------------------------------
def _through_crack(n=6, order=1, state=1, seed=5):
    """Unit square, row n//2 cut over its whole width (every edge of the row
    is an interface of the given state carrying fluid), no Dirichlet."""
    jc = n // 2
    xyz, elem, grid = synth.grid2d(n, seed, keep_row=jc)
    vid = lambda i, j: j * (n + 1) + i
    faces = np.array([sorted((vid(i, jc), vid(i + 1, jc))) for i in range(n)], np.int32)
    m = Mesh(2, order, xyz, elem, np.zeros(len(xyz), np.uint8))
    itf = Interfaces(m, faces, np.full(n, state, np.uint8), np.ones(n, np.uint8))
    yc = jc / n
    upper = xyz[elem].mean(axis=1)[:, 1] > yc
    return m, itf, upper, xyz[[vid(i, jc) for i in range(n + 1)], 0]


def _rigid_opening(m, upper, w0):
    """Upper body moved by +w0/2 in y, lower body by -w0/2: zero strain, zero
    jump on every intact face, opening w0 on the cut."""
    u = np.zeros((m.ne, m.nn, 2))
    u[upper, :, 1] = 0.5 * w0
    u[~upper, :, 1] = -0.5 * w0
    return u.reshape(-1)


@pytest.mark.parametrize("w0,p_lit", [(0.05, 0.75e-3), (0.12, 0.4e-3), (0.3, 0.0)])
def test_cohesive_traction_balances_pressure(w0, p_lit):
    """Cohesive lips held at opening w0 under the literal pressure that the
    law gives by hand (sigma_c = 1e-3, delta_c = 0.2: T(0.05) = 0.75e-3,
    T(0.12) = 0.4e-3, T(0.3) = 0): the pressure pushes the lips apart as hard
    as the cohesive traction pulls them together, the bodies are stress free
    and the fluid is at rest (uniform pressure, w = w_old), so R = 0."""
    m, itf, upper, _ = _through_crack(state=1)
    prm = asm.Params(1.0, 0.25, 1e-3, 1e-4, 1e-3, 1.0)
    u = _rigid_opening(m, upper, w0)
    w = newton.opening(m, u)
    fa = itf.active_faces
    np.testing.assert_allclose(w[fa], w0, rtol=1e-13)
    S = asm.assemble(m, itf, prm, u, np.full(itf.n_p, p_lit), w.copy(), 1.0, [], [],
                     jacobian=False)
    assert np.abs(S.R_u).max() <= 1e-16
    assert np.abs(S.R_p).max() <= 1e-16
    # a pressure off the law by 1% leaves an unbalanced load on the lips
    bad = asm.assemble(m, itf, prm, u, np.full(itf.n_p, p_lit + 1e-5), w.copy(), 1.0, [], [],
                       jacobian=False)
    assert np.abs(bad.R_u).max() > 1e-7


# --------------------------------------------------------------------------
# eq. (lubrication): the cubic law on a straight crack
# --------------------------------------------------------------------------
W0, MU, K_LIT = 0.06, 0.0018, 0.01   # 0.06^3 / (12 * 0.0018) = 2.16e-4 / 0.0216 = 0.01


def test_cubic_law_fluid_block_is_poiseuille_laplacian():
    """Straight traction-free crack at uniform opening 0.06 with mu = 0.0018:
    the Poiseuille conductivity is 0.01, and the fluid block D (s_p = 1) is
    0.01 times the 1D P1 Laplacian of the crack nodes (node spacing from the
    vertex coordinates)."""
    m, itf, upper, xs = _through_crack(n=8, state=2)
    prm = asm.Params(1.0, 0.25, 1e-3, 1e-4, MU, 1.0)
    u = _rigid_opening(m, upper, W0)
    w = newton.opening(m, u)
    S = asm.assemble(m, itf, prm, u, np.zeros(itf.n_p), w.copy(), 1.0, [], [])
    L = np.diff(xs)
    npn = len(xs)
    lap = np.zeros((npn, npn))
    for k, h in enumerate(L):
        lap[k:k + 2, k:k + 2] += np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    np.testing.assert_allclose(S.D.toarray(), K_LIT * lap, rtol=1e-12, atol=1e-15)


def test_linear_pressure_drives_poiseuille_flux():
    """The same crack under p = x: no storage (w = w_old), every interior
    node balances its in- and outflow, and the residual of the end nodes is
    the Poiseuille flux through the crack, -/+ w^3 / (12 mu) dp/dx = -/+ 0.01."""
    m, itf, upper, xs = _through_crack(n=8, state=2)
    prm = asm.Params(1.0, 0.25, 1e-3, 1e-4, MU, 1.0)
    u = _rigid_opening(m, upper, W0)
    w = newton.opening(m, u)
    S = asm.assemble(m, itf, prm, u, xs.copy(), w.copy(), 1.0, [], [], jacobian=False)
    ref = np.zeros(len(xs))
    ref[0], ref[-1] = -K_LIT, K_LIT
    np.testing.assert_allclose(S.R_p, ref, atol=1e-15)


# --------------------------------------------------------------------------
# face geometry and the DG stabilisation on two elements
# --------------------------------------------------------------------------
def _two_triangles(order=1):
    xyz = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 2.0], [3.0, 3.0]])
    elem = np.array([[0, 1, 2], [1, 3, 2]], np.int32)       # areas 2 and 4
    return Mesh(2, order, xyz, elem)


def _two_tets(order=1):
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]])
    elem = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32)  # volumes 1/6 and 1/3
    return Mesh(3, order, xyz, elem)


@pytest.mark.parametrize("order", [1, 2])
def test_face_geometry_two_elements(order):
    m = _two_triangles(order)
    assert m.nf == 1 and m.face_em[0] == 0 and m.face_ep[0] == 1
    assert m.area[0] == pytest.approx(math.sqrt(8.0), rel=1e-15)
    np.testing.assert_allclose(m.normal[0], [1 / math.sqrt(2), 1 / math.sqrt(2)], rtol=1e-15)
    assert m.hf[0] == pytest.approx(2.0 / math.sqrt(8.0), rel=1e-15)   # min(2, 4) / sqrt 8
    t = _two_tets(order)
    assert t.nf == 1
    assert t.area[0] == pytest.approx(math.sqrt(3.0) / 2.0, rel=1e-15)
    np.testing.assert_allclose(t.normal[0], np.full(3, 1 / math.sqrt(3)), rtol=1e-15)
    assert t.hf[0] == pytest.approx((1.0 / 6.0) / (math.sqrt(3.0) / 2.0), rel=1e-14)


@pytest.mark.parametrize("order", [1, 2])
def test_penalty_force_two_triangles(order):
    """Element 0 at rest, element 1 translated by c = (1, 0); every face is
    intact.  The strains vanish, so only the stabilisation acts: the force on
    element 1 (its residual summed over nodes) is (b / h_f) |f| Chat(n) c with
    b = 10, h_f = 1/sqrt(2), |f| = sqrt(8) -> factor 40; E = 1, nu = 0.25 ->
    lambda = G = 0.4; n = (1, 1)/sqrt(2): Chat c = (0.8, 0.4) -> (32, 16), and
    the opposite force on element 0."""
    m = _two_triangles(order)
    itf = Interfaces(m)
    prm = asm.Params(1.0, 0.25, 1e-3, 1e-4, 1e-3, 1.0, b_stab=10.0)
    u = np.zeros((2, m.nn, 2))
    u[1, :, 0] = 1.0
    S = asm.assemble(m, itf, prm, u.reshape(-1), np.zeros(0), np.zeros((1, m.nq)), 1.0, [], [],
                     jacobian=False)
    Ru = S.R_u.reshape(2, m.nn, 2).sum(axis=1)
    np.testing.assert_allclose(Ru[1], [32.0, 16.0], rtol=1e-13)
    np.testing.assert_allclose(Ru[0], [-32.0, -16.0], rtol=1e-13)


@pytest.mark.parametrize("order", [1, 2])
def test_contact_branch_matches_the_intact_penalty(order):
    """Contact branch of the traction law (the reading for w < 0): element 1
    pushed rigidly into element 0 by delta = 0.01 along n, so the opening is
    w = -0.01 at every point and the strains vanish.  On an intact face the
    stabilisation alone acts, (b/h_f)|f| Chat(n) (-delta n) = -40 (lambda + 2G)
    delta n (Chat n = (lambda + 2G) n); the contact stiffness k_c = (b/h_f)
    (lambda + 2G) gives a traction-free face (state 2) exactly that force, and
    a cohesive face (state 1, T = sigma_c + k_c w, continuous at w = 0) that
    force plus the strength sigma_c |f| n."""
    m = _two_triangles(order)
    prm = asm.Params(1.0, 0.25, 1e-3, 1e-4, 1e-3, 1.0, b_stab=10.0)
    n = np.array([1.0, 1.0]) / math.sqrt(2.0)
    delta = 0.01
    u = np.zeros((2, m.nn, 2))
    u[1, :, :] = -delta * n
    face = np.array([[1, 2]], np.int32)
    forces = {}
    for state in (0, 1, 2):
        itf = Interfaces(m, face, np.array([state], np.uint8), np.zeros(1, np.uint8))
        S = asm.assemble(m, itf, prm, u.reshape(-1), np.zeros(0), np.zeros((1, m.nq)), 1.0, [], [],
                         jacobian=False)
        Ru = S.R_u.reshape(2, m.nn, 2).sum(axis=1)
        np.testing.assert_allclose(Ru[0], -Ru[1], rtol=1e-13, atol=1e-18)
        forces[state] = Ru[1]
    lam_2g = 0.4 + 2 * 0.4                         # E = 1, nu = 0.25
    np.testing.assert_allclose(forces[0], -40.0 * lam_2g * delta * n, rtol=1e-13)
    np.testing.assert_allclose(forces[2], forces[0], rtol=1e-13)
    np.testing.assert_allclose(forces[1], forces[0] + 1e-3 * math.sqrt(8.0) * n, rtol=1e-13)


# --------------------------------------------------------------------------
# Sneddon's penny crack
# --------------------------------------------------------------------------
def test_sneddon_penny_volume():
    """Uniform pressure p = 1e-3 on a traction-free disk (state 2, pressure
    applied as a load) in the clamped unit cube, 3D P2 on the Kuhn n = 6 mesh
    (disk of radius 0.3 made of mid-plane triangles; R_eff from their area).
    Sneddon's infinite-medium volume is 16 (1 - nu^2) p R^3 / (3 E); the
    clamped cube (crack diameter 0.65 of its side) and the two cells per
    radius stiffen the response, so the volume lies between 0.6 and 1.0 of
    it (measured 0.71, and 0.74 / 0.82 / 0.76 at n = 8 / 10 / 12).  A flipped
    pressure or normal gives a negative volume, a face area off by 2 a ratio
    near 1.4."""
    mat = synth.Material(1.0, 0.2, 1e-3, 1e-4, 1e-3, 1.0)
    prob = synth.penny_problem(6, 2, 7, mat, 1e-4, radius=0.3, ring_width=0.0)
    case = Case.from_problem(prob)
    m = case.mesh
    p0 = 1e-3
    S = asm.assemble(m, case.itf, case.prm, np.zeros(m.n_u), np.full(case.itf.n_p, p0),
                     np.zeros((m.nf, m.nq)), 1.0, [], [])
    A = asm.bsr_A(m, S).tocsr()
    inv = np.linalg.inv(S.A_diag)
    M = spla.LinearOperator(A.shape, matvec=lambda r: np.einsum(
        "eij,ej->ei", inv, r.reshape(m.ne, m.bu)).reshape(-1))
    u, info = spla.gmres(A, -S.R_u, M=M, rtol=1e-10, restart=100, maxiter=5000)
    assert info == 0
    assert np.linalg.norm(A @ u + S.R_u) <= 1e-9 * np.linalg.norm(S.R_u)
    fa = case.itf.active_faces
    w = newton.opening(m, u)
    vol = float(np.sum(m.fq_w[None, :] * m.area[fa][:, None] * w[fa]))
    r_eff = math.sqrt(float(m.area[fa].sum()) / math.pi)
    ratio = vol / nondim.sneddon_volume_penny(p0, r_eff, nondim.e_prime(1.0, 0.2))
    assert 0.6 < ratio < 1.0, ratio
    # the opening is largest in the middle of the disk and positive everywhere
    assert np.all(w[fa] > 0.0)
