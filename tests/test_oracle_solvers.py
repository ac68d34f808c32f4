"""Oracle solver pins (no GPU): block inverses, GMRES against dense LU,
GMRES-IR against FP64, Newton iteration counts of given-length steps."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import assemble as asm
from oracle import newton, solve
from oracle.newton import Case

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nondim_printed.json")


def _system(prob):
    case = Case.from_problem(prob)
    st = newton.initial_state(case)
    S = asm.assemble(case.mesh, case.itf, case.prm, st.u, st.p, st.w_old, st.s_p,
                     case.src_pnode, case.src_q0)
    return case, S


@pytest.mark.parametrize("prob", [synth.kgd_small(8, 1), synth.penny_small(4, 2, steps=1)],
                         ids=["2d_p1", "3d_p2"])
def test_block_inverse(prob):
    case, S = _system(prob)
    pc = solve.BlockJacobi(case.mesh, S)
    eye = np.eye(case.mesh.bu)
    for e in range(0, case.mesh.ne, 7):
        err = np.abs(S.A_diag[e] @ pc.inv[e] - eye).max()
        assert err <= 1e-12 * np.linalg.cond(S.A_diag[e])
    # the pressure block is the Schur complement of the block-diagonal part
    J = asm.full_matrix(case.mesh, S).toarray()
    nu = case.mesh.n_u
    Minv_A = np.zeros((nu, nu))
    for e in range(case.mesh.ne):
        sl = slice(e * case.mesh.bu, (e + 1) * case.mesh.bu)
        Minv_A[sl, sl] = pc.inv[e]
    Sref = J[nu:, nu:] - J[nu:, :nu] @ Minv_A @ J[:nu, nu:]
    np.testing.assert_allclose(np.linalg.inv(pc.Sinv), Sref, rtol=1e-9,
                               atol=1e-9 * np.abs(Sref).max())


def test_gmres_matches_dense_lu():
    case, S = _system(synth.kgd_small(6, 2))
    b = -S.R
    x_lu = solve.dense_solve(case.mesh, S, b)
    op = solve.Operator(case.mesh, S)
    x, st = solve.gmres(op, b, solve.BlockJacobi(case.mesh, S), m=60, rtol=1e-10)
    assert st.converged and st.true_relres <= 1e-10
    J = asm.full_matrix(case.mesh, S).toarray()
    kappa = np.linalg.cond(J)
    assert np.linalg.norm(x - x_lu) <= kappa * 1e-10 * np.linalg.norm(x_lu)
    np.testing.assert_allclose(J @ x, b, atol=1e-9 * np.abs(b).max())


def test_newton_states_gmres_vs_dense_and_ir():
    """Converged Newton states do not depend on the linear solver: GMRES and
    GMRES-IR states match the dense-LU states to 1e-8 (the build's parity
    gate), and every solve reaches the 1e-10 true residual."""
    case = Case.from_problem(synth.kgd_small(8, 1, steps=2))
    ref = newton.run(case, 2, solver="dense")
    for solver in ("gmres", "ir"):
        out = newton.run(case, 2, solver=solver)
        for (a, na), (b, nb) in zip(ref, out):
            assert na.converged and nb.converged
            assert nb.max_true_relres <= 1e-10
            for x, y in ((a.u, b.u), (a.p, b.p), (a.w_old, b.w_old)):
                assert np.linalg.norm(x - y) <= 1e-8 * np.linalg.norm(x)
        if solver == "ir":
            assert all(ns.ir_steps >= 2 for _, ns in out)


def test_newton_iteration_counts_given_length():
    """Given-length steps converge in a handful of iterations (the paper
    reports 3 to 5 without propagation; the first step here starts from
    u = 0 where the conductivity is degenerate, so allow up to 8)."""
    g = json.load(open(GOLD))["newton_iterations_given_length"]
    case = Case.from_problem(synth.kgd_small(8, 2, steps=3))
    out = newton.run(case, 3)
    its = [ns.iterations for _, ns in out]
    assert all(ns.converged for _, ns in out)
    assert all(2 <= k <= 8 for k in its), its
    assert min(its[1:]) <= g["max"] + 1
    # quadratic contraction at the end of each step
    for _, ns in out:
        d = ns.du_rel
        assert d[-1] <= 1e-10 and d[-2] <= 1e-3
