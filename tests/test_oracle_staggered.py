"""The staggered comparison scheme of Sec. "Fully-coupled vs. staggered
hydro-mechanics with applied inflow boundary conditions" in the oracle.

* Each half of an iteration solves its own decoupled equations: after a
  step on a crack without cohesive faces (a linear solid while the lips
  stay open), from a positive but nonuniform pressure, the solid rows vanish
  at (U_new, P_old) and the fluid rows vanish at (U_new, P_new) except the
  fixed node's, where the pressure takes its prescribed value (checked with
  a fresh assembly, relative to the size of each row's terms).
* The scheme does not converge on a plane-strain crack with inflow, the
  paper's finding: from the uniform-pressure predictor the pressure swings
  between a low and a high state (the mechanism the paper describes: a high
  pressure opens the mouth, the wider mouth drops the pressure, and back),
  while Newton on the monolithic system converges from the same start.
"""
import numpy as np
import pytest

import synth
from oracle import assemble as asm
from oracle import newton
from oracle.newton import Case


def _kgd(ring):
    mat = synth.Material(E=1.0, nu=0.25, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=1.0)
    prob = synth.kgd_problem(24, 1, 3, mat, 1e-4, half_length=0.25, ring=ring, load_steps=1)
    return Case.from_problem(prob)


@pytest.fixture(scope="module")
def kgd():
    case = _kgd(1)
    return case, newton.initial_state(case, predictor=True)


def test_staggered_halves_solve_their_own_equations():
    case = _kgd(0)
    pred = newton.initial_state(case, predictor=True)
    k = np.arange(case.itf.n_p)
    st0 = newton.State(pred.u, pred.p * (1.0 + 0.5 * np.sin(k)), pred.w_old, pred.s_p)
    m = case.mesh
    assert np.all(newton.opening(m, st0.u)[case.itf.active_faces] > 0.0)
    node, value = 3, 2.0 * st0.p[3]
    st1, du, dp = newton.staggered_step(case, st0, node, value)
    assert np.all(newton.opening(m, st1.u)[case.itf.active_faces] > 0.0)  # still linear
    args = (case.src_pnode, case.src_q0)
    # solid rows at (U_new, P_old)
    S = asm.assemble(m, case.itf, case.prm, st1.u, st0.p, st0.w_old, st0.s_p, *args)
    J = asm.full_matrix(m, S)
    mag = abs(J) @ np.abs(np.concatenate([st1.u, st0.p]))
    assert np.all(np.abs(S.R_u) <= 1e-10 * mag[:m.n_u].max())
    # fluid rows at (U_new, P_new), all but the fixed node
    S = asm.assemble(m, case.itf, case.prm, st1.u, st1.p, st0.w_old, st0.s_p, *args)
    J = asm.full_matrix(m, S)
    mag = (abs(J) @ np.abs(np.concatenate([st1.u, st1.p])))[m.n_u:]
    free = np.arange(case.itf.n_p) != node
    assert np.all(np.abs(S.R_p[free]) <= 1e-10 * mag.max())
    assert st1.p[node] == value
    assert np.array_equal(st1.p, st0.p + dp) and np.array_equal(st1.u, st0.u + du)


def test_staggered_does_not_converge_where_newton_does(kgd):
    case, st0 = kgd
    ref, ns = newton.newton_solve(case, st0, solver="dense")
    assert ns.converged and ns.iterations <= 10
    s, peaks, inc = st0, [], []
    for _ in range(10):
        s, du, dp = newton.staggered_step(case, s, 0, st0.p[0])
        peaks.append(np.abs(s.p).max())
        inc.append(max(np.linalg.norm(du) / np.linalg.norm(s.u), np.linalg.norm(dp) / np.linalg.norm(s.p)))
    # no iteration comes close to convergence, and the pressure swings by
    # orders of magnitude from one iteration to the next
    assert min(inc) > 0.5
    swings = [max(a, b) / min(a, b) for a, b in zip(peaks, peaks[1:])]
    assert min(swings) > 1e3
    assert np.linalg.norm(s.p - ref.p) > np.linalg.norm(ref.p)
