"""Oracle pins against closed forms and exact discrete invariants (no GPU):
printed nondimensional numbers, Sneddon's pressurised crack, the uniform-
pressure (toughness-dominated) KGD step, and discrete mass conservation."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assemble as asm
from oracle import newton, nondim
from oracle.newton import Case

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nondim_printed.json")


def _printed_close(val, printed):
    # printed values carry two significant figures: accept the rounding interval
    # plus a 1% margin for the rounding of the table's inputs
    mag = 10 ** (np.floor(np.log10(abs(printed))) - 1)
    return abs(val - printed) <= 0.5 * mag + 0.01 * abs(printed)


def test_printed_nondimensional_numbers():
    g = json.load(open(GOLD))
    for key in ("kgd_viscosity_regime", "kgd_toughness_regime"):
        c = g[key]
        K = nondim.kgd_toughness(c["E"], c["nu"], c["mu"], c["Q0"], c["G_c"])
        M = nondim.kgd_viscosity(c["E"], c["nu"], c["mu"], c["Q0"], c["G_c"])
        assert _printed_close(K, c["K"]) and _printed_close(M, c["M"]), (key, K, M)
        assert K == pytest.approx(M ** -0.25, rel=1e-13)
    c = g["penny_t0"]
    K = nondim.penny_toughness(c["t"], c["E"], c["nu"], c["mu"], c["Q0"], c["G_c"])
    M = nondim.penny_viscosity(c["t"], c["E"], c["nu"], c["mu"], c["Q0"], c["G_c"])
    assert _printed_close(K, c["K"]) and _printed_close(M, c["M"]), (K, M)
    assert M == pytest.approx(K ** (-18.0 / 5.0), rel=1e-12)
    c = g["penny_regime_times"]
    tv = nondim.penny_time_for_toughness(c["K_viscous"], c["E"], c["nu"], c["mu"], c["Q0"], c["G_c"])
    tt = nondim.penny_time_for_toughness(c["K_tough"], c["E"], c["nu"], c["mu"], c["Q0"], c["G_c"])
    assert _printed_close(tv, c["t_viscous"]) and _printed_close(tt, c["t_tough"]), (tv, tt)


def _sneddon_case(n, nu=0.4, half_length=0.08):
    mat = synth.Material(1.0, nu, 1e-3, 1e-4, 1e-3, 1.0)
    prob = synth.kgd_problem(n, 2, 7, mat, 1e-4, half_length=half_length, ring=0)
    case = Case.from_problem(prob)
    m = case.mesh
    p0 = 1e-3
    S = asm.assemble(m, case.itf, case.prm, np.zeros(m.n_u), np.full(case.itf.n_p, p0),
                     np.zeros((m.nf, m.nq)), 1.0, [], [])
    u = spla.spsolve(asm.bsr_A(m, S).tocsc(), -S.R_u)
    w = newton.opening(m, u)
    fa = case.itf.active_faces
    vol = float(np.sum(m.fq_w[None, :] * m.area[fa][:, None] * w[fa]))
    xs = prob.xyz[prob.crack_faces.ravel(), 0]
    ell = 0.5 * (xs.max() - xs.min())
    Ep = nondim.e_prime(1.0, nu)
    return vol, nondim.sneddon_volume_2d(p0, ell, Ep), case, w, ell, Ep, p0


def test_sneddon_pressurised_crack_2d():
    """Uniform pressure on a traction-free crack: the crack volume tends to
    Sneddon's 2 pi p l^2 / E' under refinement (finite clamped domain and
    the crack-tip singularity leave a few per cent at these sizes)."""
    v24, s24, *_ = _sneddon_case(24)
    v48, s48, case, w, ell, Ep, p0 = _sneddon_case(48)
    e24, e48 = v24 / s24 - 1.0, v48 / s48 - 1.0
    assert abs(e48) < abs(e24)
    assert abs(e48) < 0.10          # E instead of E' would be 19% off at nu = 0.4
    # opening profile in the middle of the crack
    m = case.mesh
    fa = case.itf.active_faces
    lam = m.fq_mu
    xq = np.einsum("qk,fkd->fqd", lam, m.xyz[m.face_vert[fa]])
    xc = 0.5 * (xq[..., 0].max() + xq[..., 0].min())
    sel = np.abs(xq[..., 0] - xc) < 0.6 * ell
    ref = np.array([nondim.sneddon_opening_2d(x - xc, p0, ell, Ep) for x in xq[..., 0][sel]])
    assert np.max(np.abs(w[fa][sel] / ref - 1.0)) < 0.12


def test_uniform_pressure_step_matches_linear_volume():
    """Toughness-dominated limit (viscosity -> 0, uniform pressure): with a
    linear elastic crack the volume is V = p V1, so every given-length step
    raises the pressure by exactly Q0 dt / V1, V1 being the volume of a
    separate unit-pressure elastic solve (V1 itself is pinned to Sneddon's
    closed form by the pressurised-crack test).
    Newton starts from the elastic state under the initial pressure so that
    the conductivity is not degenerate at the first iterate."""
    mat = synth.Material(1.0, 0.25, 1e-3, 1e-4, 1e-16, 1.0)
    prob = synth.kgd_problem(12, 1, 9, mat, 1e-4, half_length=0.2, ring=0, load_steps=2)
    case = Case.from_problem(prob)
    m = case.mesh
    fa = case.itf.active_faces
    st = newton.initial_state(case)
    S = asm.assemble(m, case.itf, case.prm, np.zeros(m.n_u), np.ones(case.itf.n_p),
                     st.w_old, 1.0, [], [])
    u1 = spla.spsolve(asm.bsr_A(m, S).tocsc(), -S.R_u)         # unit-pressure solve
    V1 = float(np.sum(m.fq_w[None, :] * m.area[fa][:, None] * newton.opening(m, u1)[fa]))
    st.u = u1 * case.prm.sigma_c
    ps = []
    for _ in range(2):
        new, ns = newton.newton_solve(case, st, solver="dense")
        assert ns.converged and ns.iterations <= 5
        assert np.ptp(new.p) <= 1e-6 * abs(new.p.mean())       # uniform pressure
        ps.append(new.p.mean())
        st = newton.end_load_step(case, new)
    q = case.src_q0.sum() * case.prm.dt
    assert ps[0] == pytest.approx(q / V1, rel=1e-6)             # w^0 = 0
    assert ps[1] - ps[0] == pytest.approx(q / V1, rel=1e-6)


@pytest.mark.parametrize("prob", [synth.kgd_small(8, 1), synth.kgd_small(6, 2),
                                  synth.penny_small(4, 2, steps=1)],
                         ids=["2d_p1", "2d_p2", "3d_p2"])
def test_discrete_mass_conservation(prob):
    """The pressure test functions are a partition of unity on the fluid
    faces, so a converged step injects exactly Q0 dt:
    sum_faces int (w^{n+1} - w^n) = Q0 dt."""
    case = Case.from_problem(prob)
    m = case.mesh
    fa = case.itf.active_faces
    W = m.fq_w[None, :] * m.area[fa][:, None]
    st = newton.initial_state(case)
    for _ in range(min(prob.load_steps, 2)):
        new, ns = newton.newton_solve(case, st)
        assert ns.converged
        w1 = newton.opening(m, new.u)
        dv = float(np.sum(W * (w1[fa] - st.w_old[fa])))
        assert dv == pytest.approx(case.src_q0.sum() * case.prm.dt, rel=1e-8)
        assert ns.iterations <= 8
        st = newton.end_load_step(case, new)


def test_viscosity_scaling_forms():
    """The scaling forms of the zero-toughness plane-strain solution (eq.
    DimensionalSol1-3): w ~ mu'^(1/6) Q0^(1/2) t^(1/3) E'^(-1/6),
    p ~ mu'^(1/3) E'^(2/3) t^(-1/3), l ~ Q0^(1/2) E'^(1/6) t^(2/3) mu'^(-1/6).
    Their exponents leave w and l unchanged and multiply p by the predicted
    factor under two rescalings of the inputs, which the discrete equations
    must reproduce exactly (one load step from the predictor, dense solves):
    (a) mu x a, t (the time step) x a, Q0 / a: predicted factors w a^0, p a^0;
    (b) E, sigma_c, G_c, mu all x b (delta_c fixed): w b^0, p b^1."""
    import dataclasses
    from oracle import newton
    from oracle.newton import Case

    def solve(mat, q0):
        prob = synth.kgd_problem(10, 1, 2, mat, q0, half_length=0.2, ring=1, load_steps=1)
        (st, ns), = newton.run(Case.from_problem(prob), 1, predictor=True, solver="dense")
        assert ns.converged
        return st

    base = synth.Material(E=1.0, nu=0.25, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=1.0)
    ref = solve(base, 1e-4)
    a, b = 10.0, 3.0
    pred_p = lambda fmu, fE, ft: fmu ** (1 / 3) * fE ** (2 / 3) * ft ** (-1 / 3)
    pred_w = lambda fmu, fq, ft, fE: fmu ** (1 / 6) * fq ** 0.5 * ft ** (1 / 3) * fE ** (-1 / 6)
    st = solve(dataclasses.replace(base, mu=base.mu * a, dt=base.dt * a), 1e-4 / a)
    assert pred_w(a, 1 / a, a, 1.0) == pytest.approx(1.0) and pred_p(a, 1.0, a) == pytest.approx(1.0)
    np.testing.assert_allclose(st.u, ref.u, rtol=0, atol=1e-9 * np.abs(ref.u).max())
    np.testing.assert_allclose(st.p, ref.p, rtol=1e-9)
    st = solve(dataclasses.replace(base, E=base.E * b, sigma_c=base.sigma_c * b, G_c=base.G_c * b,
                                   mu=base.mu * b), 1e-4)
    fw, fp = pred_w(b, 1.0, 1.0, b), pred_p(b, b, 1.0)
    assert fw == pytest.approx(1.0) and fp == pytest.approx(b)
    np.testing.assert_allclose(st.u, fw * ref.u, rtol=0, atol=1e-9 * np.abs(ref.u).max())
    np.testing.assert_allclose(st.p, fp * ref.p, rtol=1e-9)
