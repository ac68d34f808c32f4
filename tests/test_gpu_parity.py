"""GPU parity of the HIP Newton-step path against the FP64 CPU oracle.

Every call goes through the C ABI (libhf.so via its ctypes binding).  Sizes
are chosen so that the oracle finishes in seconds while the kernels still
see several tiles and a ragged tail (element counts not divisible by the
rows per workgroup of the block product, vector lengths spanning several
reduction blocks).

Tolerances: assembled R and J blocks 1e-12 relative to the largest entry of
the compared array (same formulas, different summation order); Jacobian
products 1e-13; converged Newton states 1e-8 in u, p and the opening w
(the build's parity gate); every linear solve reaches a true relative
residual of 1e-10.
"""
import numpy as np
import pytest

import synth
from oracle import assemble as asm
from oracle import newton, solve
from oracle.newton import Case

pytestmark = pytest.mark.gpu

import paper_1911_10275_amd as hf  # noqa: E402  (a broken package fails, never skips)

SMALL = {
    "2d_p1_n9": lambda: synth.kgd_small(9, 1, steps=3),
    "2d_p2_n7": lambda: synth.kgd_small(7, 2, steps=2),
    "3d_p1_n4": lambda: synth.penny_small(4, 1, steps=2),
    "3d_p2_n3": lambda: synth.penny_problem(3, 2, 21, synth.Material(1.0, 0.2, 1e-3, 1e-4, 1e-3, 1.0),
                                            1e-4, radius=0.34, ring_width=0.2, load_steps=2,
                                            name="penny_n3_p2"),
}


def _pair(prob):
    case = Case.from_problem(prob)
    ctx = hf.context_for_problem(prob)
    fv, fe, nq = ctx.faces()
    # the canonical face order and labels are part of the boundary contract
    assert fv.shape == case.mesh.face_vert.shape
    np.testing.assert_array_equal(fv, case.mesh.face_vert)
    np.testing.assert_array_equal(fe[:, 0], case.mesh.face_em)
    np.testing.assert_array_equal(fe[:, 1], case.mesh.face_ep)
    assert nq == case.mesh.nq
    keys = ctx.pnodes()
    ok = [(k[1], -1) if k[0] == "v" else (k[1], k[2]) for k in case.itf.p_keys]
    np.testing.assert_array_equal(keys, np.array(ok, dtype=np.int64).reshape(-1, 2))
    return case, ctx


def _random_state(case, seed):
    m = case.mesh
    rng = np.random.default_rng(seed)
    u = rng.normal(size=m.n_u) * 0.05
    p = rng.uniform(0.0, 2e-3, case.itf.n_p)
    wo = rng.uniform(0.0, 1e-2, (m.nf, m.nq))
    return u, p, wo


def _rel(a, b):
    s = max(np.abs(a).max(), np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / s


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("incremental", [0, 1], ids=["full", "incremental"])
def test_assembly_parity(name, incremental):
    """The first assembly of a context is a full one; with incremental
    assembly the second one re-assembles only the elements with cohesive or
    fluid interfaces and takes the other residual rows from the cached
    blocks.  Both are checked, at two different states."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    ctx.set_options(incremental_assembly=incremental)
    for seed in (13, 3):
        _check_assembly_at(case, ctx, seed)
    ctx.close()


def _branch_state(case):
    """The first seeded state (larger displacements than ``_random_state``)
    whose cohesive points visit every branch of the traction law: state 1
    in contact (w < 0), softening (0 <= w <= delta_c) and fully softened
    (w > delta_c); state 2 in contact and open."""
    m = case.mesh
    st, dc = case.itf.qp_state, case.prm.delta_c
    c1, c2 = st == 1, st == 2
    for seed in range(2000):
        rng = np.random.default_rng(seed)
        u = rng.normal(size=m.n_u) * 0.25
        w = newton.opening(m, u)
        hit = [c1 & (w < 0), c1 & (w >= 0) & (w <= dc), c1 & (w > dc), c2 & (w < 0), c2 & (w >= 0)]
        if all(np.any(h) for h in hit):
            return u, rng.uniform(0.0, 2e-3, case.itf.n_p), rng.uniform(0.0, 1e-2, (m.nf, m.nq))
    raise AssertionError("no seeded state visits every traction-law branch")


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("incremental", [0, 1], ids=["full", "incremental"])
def test_assembly_parity_every_traction_branch(name, incremental):
    """R and every block at a state whose cohesive points lie in every
    branch of the traction law (checked on the oracle side first), after a
    full assembly at another state so that the incremental path is used."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    ctx.set_options(incremental_assembly=incremental)
    _check_assembly_at(case, ctx, 13)
    _check_assembly_at(case, ctx, _branch_state(case))
    ctx.close()


def _unloading_state(case):
    """A state of ``_branch_state`` with an unloading history that puts
    cohesive points on the secant (0 <= w < w_max), closed after unloading
    (w < 0 < w_max), beyond their history (w > w_max) and on a fully
    softened history (w_max > delta_c), each checked on the oracle side."""
    m = case.mesh
    u, p, wo = _branch_state(case)
    w = newton.opening(m, u)
    rng = np.random.default_rng(99)
    wm = np.where(rng.uniform(size=w.shape) < 0.6, np.abs(w) + rng.uniform(0.02, 0.3, w.shape),
                  np.abs(w) * rng.uniform(0.2, 0.8, w.shape))
    c1, dc = case.itf.qp_state == 1, case.prm.delta_c
    hit = [c1 & (w >= 0) & (w < wm), c1 & (w < 0) & (wm > 0), c1 & (w > wm), c1 & (wm > dc) & (w < wm)]
    assert all(np.any(h) for h in hit)
    return (u, p, wo), wm


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("incremental", [0, 1], ids=["full", "incremental"])
def test_assembly_parity_unloading(name, incremental):
    """With cohesive unloading on: a zero history gives the envelope (the
    oracle without history), and a history that puts cohesive points in
    every unloading branch gives the oracle's R and blocks with that history
    (1e-12), in full and incremental assembly."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    ctx.set_options(incremental_assembly=incremental, cohesive_unloading=1)
    _check_assembly_at(case, ctx, 13)
    st, wm = _unloading_state(case)
    ctx.set_history(wm)
    np.testing.assert_array_equal(ctx.get_history(), wm)
    _check_assembly_at(case, ctx, st, w_max=wm)
    ctx.close()


@pytest.mark.parametrize("name", ["2d_p1_n9", "3d_p2_n3"])
@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_newton_load_steps_unloading(name, precision):
    """Two load steps with cohesive unloading from a history that is zero at
    half of the face points and in [0.2, 0.8] delta_c at the others: the
    converged states match the oracle's (1e-8), every solve at 1e-10, and
    after each step the history is max(w_max, w) of the oracle (1e-8; the
    points without history take their opening)."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    m, dc = case.mesh, case.prm.delta_c
    rng = np.random.default_rng(7)
    H = np.where(rng.uniform(size=(m.nf, m.nq)) < 0.5, 0.0, rng.uniform(0.2 * dc, 0.8 * dc, (m.nf, m.nq)))
    st = newton.initial_state(case)
    st.w_max = H.copy()
    ctx.set_options(precision=precision, cohesive_unloading=1)
    ctx.set_state(st.u, st.p, st.w_old)
    ctx.set_history(H)
    c1 = case.itf.qp_state == 1
    for step in range(2):
        st, ns_ref = newton.newton_solve(case, st)
        assert ns_ref.converged
        w_ref = newton.opening(m, st.u)
        assert np.any(c1 & (w_ref >= 0) & (w_ref < st.w_max))   # the secant is in use
        st = newton.end_load_step(case, st)
        ns = ctx.newton_solve()
        assert ns.converged and ns.lin.true_relres <= 1e-10
        ctx.end_load_step()
        u, p, w, wo = ctx.get_state()
        assert np.linalg.norm(u - st.u) <= 1e-8 * np.linalg.norm(st.u)
        if case.itf.n_p:
            assert np.linalg.norm(p - st.p) <= 1e-8 * np.linalg.norm(st.p)
        wm = ctx.get_history()
        assert np.linalg.norm(wm - st.w_max) <= 1e-8 * np.linalg.norm(st.w_max)
    ctx.close()


def _check_assembly_at(case, ctx, seed, w_max=None):
    m = case.mesh
    u, p, wo = _random_state(case, seed) if isinstance(seed, int) else seed
    ctx.set_state(u, p, wo)
    rn = ctx.assemble()
    s_p = newton.fluid_scale(case, wo, u)
    S = asm.assemble(m, case.itf, case.prm, u, p, wo, s_p, case.src_pnode, case.src_q0, w_max=w_max)
    ru, rp = ctx.residual()
    assert _rel(ru, S.R_u) < 1e-12
    if case.itf.n_p:
        assert _rel(rp, S.R_p) < 1e-12
    assert rn == pytest.approx(np.linalg.norm(S.R), rel=1e-12)
    # every block row of A
    cols, blocks = ctx.block_rows(np.arange(m.ne))
    ref = {}
    for e in range(m.ne):
        ref[(e, e)] = S.A_diag[e]
    for f in range(m.nf):
        ref[(m.face_em[f], m.face_ep[f])] = S.A_mp[f]
        ref[(m.face_ep[f], m.face_em[f])] = S.A_pm[f]
    scale = max(np.abs(b).max() for b in ref.values())
    err = 0.0
    for e in range(m.ne):
        for s in range(cols.shape[1]):
            c = cols[e, s]
            if c < 0:
                assert not np.any(blocks[e, s])
                continue
            err = max(err, np.abs(blocks[e, s] - ref[(e, c)]).max())
    assert err / scale < 1e-12
    B, Cm, D = ctx.coupling()
    if case.itf.n_p:
        assert _rel(B, S.B.toarray()) < 1e-12
        assert _rel(Cm, S.C.toarray()) < 1e-12
        assert _rel(D, S.D.toarray()) < 1e-12


@pytest.mark.parametrize("name", list(SMALL))
def test_jacobian_product_parity(name):
    torch = pytest.importorskip("torch")
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    u, p, wo = _random_state(case, 4)
    ctx.set_state(u, p, wo)
    ctx.assemble()
    S = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, newton.fluid_scale(case, wo, u),
                     case.src_pnode, case.src_q0)
    op = solve.Operator(case.mesh, S)
    rng = np.random.default_rng(5)
    x = rng.normal(size=op.n)
    xd = torch.tensor(x, device="cuda")
    yd = torch.empty_like(xd)
    torch.cuda.synchronize()
    ctx.apply_jacobian(xd.data_ptr(), yd.data_ptr())
    torch.cuda.synchronize()
    assert _rel(yd.cpu().numpy(), op(x)) < 1e-13
    ctx.close()


def _gpu_run(ctx, case, steps, precision, predictor=False):
    ctx.set_options(precision=precision)
    st0 = newton.initial_state(case)
    ctx.set_state(st0.u, st0.p, st0.w_old)
    if predictor:
        ctx.initial_guess()
    out = []
    for _ in range(steps):
        ns = ctx.newton_solve()
        assert ns.converged
        assert ns.lin.true_relres <= 1e-10
        ctx.end_load_step()
        out.append((ctx.get_state(), ns))
    return out


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_newton_load_steps_parity(name, precision):
    """Converged states of every given-length load step match the oracle to
    1e-8 (u, p, and the opening w at every face point)."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    steps = prob.load_steps
    ref = newton.run(case, steps, solver="gmres")
    assert all(ns.converged for _, ns in ref)
    got = _gpu_run(ctx, case, steps, precision)
    for (st, ns_ref), ((u, p, w, wo), ns) in zip(ref, got):
        assert np.linalg.norm(u - st.u) <= 1e-8 * np.linalg.norm(st.u)
        if case.itf.n_p:
            assert np.linalg.norm(p - st.p) <= 1e-8 * np.linalg.norm(st.p)
        fa = case.itf.active_faces
        assert np.linalg.norm(wo[fa] - st.w_old[fa]) <= 1e-8 * np.linalg.norm(st.w_old[fa])
        assert np.linalg.norm(w - wo) <= 1e-14 * max(np.linalg.norm(wo), 1e-300)
        assert abs(ns.iterations - ns_ref.iterations) <= 1
    ctx.close()


@pytest.mark.parametrize("name", ["2d_p1_n9", "3d_p2_n3"])
@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_newton_load_steps_unfolded(name, precision):
    """With the preconditioner applied before each product instead of folded
    into the blocks, the converged states still match the oracle to 1e-8."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    ctx.set_options(fold_preconditioner=0)
    ref = newton.run(case, prob.load_steps, solver="gmres")
    got = _gpu_run(ctx, case, prob.load_steps, precision)
    for (st, _), ((u, p, w, wo), ns) in zip(ref, got):
        assert np.linalg.norm(u - st.u) <= 1e-8 * np.linalg.norm(st.u)
        assert np.linalg.norm(p - st.p) <= 1e-8 * np.linalg.norm(st.p)
    ctx.close()


# a long pre-crack: 77 pressure nodes, three panels of the blocked inverse
WIDE = dict(SMALL, **{
    "2d_p2_n48_long": lambda: synth.kgd_problem(48, 2, 31, synth.Material(1.0, 0.25, 1e-3, 1e-4, 1e-3, 1.0),
                                                1e-4, half_length=0.35, ring=2, load_steps=1,
                                                name="kgd_n48_p2_long"),
})


@pytest.mark.parametrize("name", ["2d_p2_n7", "3d_p2_n3", "2d_p2_n48_long"])
def test_dense_inverse_wide_path(name):
    """The pressure-block inverse by the grid-wide blocked Gauss-Jordan
    (forced for every block size; 77 nodes span three panels of 32 pivots)
    gives the preconditioner of the one-workgroup inverse and the oracle's
    M^-1 (J M^-1 x to 1e-10).  The two GPU inverses round differently (the
    blocked one applies a panel's eliminations to the other columns as one
    product), so they agree to the inversion's rounding, 10 kappa(S) u."""
    torch = pytest.importorskip("torch")
    prob = WIDE[name]()
    case, ctx = _pair(prob)
    u, p, wo = _random_state(case, 12)
    x = np.random.default_rng(13).normal(size=ctx.sizes.n_total)
    xd = torch.tensor(x, device="cuda")
    ys = []
    for wide in (0, 1):
        ctx.set_tuning(dense_wide_min=wide)
        ctx.set_options(gmres_maxit=1)
        ctx.set_state(u, p, wo)
        ctx.assemble()
        ctx.solve(check=False)
        yd = torch.empty_like(xd)
        torch.cuda.synchronize()
        ctx.apply_preconditioned(xd.data_ptr(), yd.data_ptr(), hf.HF_FP64, folded=0)
        torch.cuda.synchronize()
        ys.append(yd.cpu().numpy())
    ctx.close()
    S = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, newton.fluid_scale(case, wo, u),
                     case.src_pnode, case.src_q0)
    bj = solve.BlockJacobi(case.mesh, S)
    kappa = np.linalg.cond(bj.Sinv)
    assert _rel(ys[1], ys[0]) < max(10.0 * kappa * np.finfo(float).eps, 1e-13)
    ref = solve.Operator(case.mesh, S)(bj(x))
    assert _rel(ys[1], ref) < 1e-10


def test_restart_growth_on_stagnation():
    """GMRES(1) stagnates on the 3D P2 system; the restart length doubles
    (in a new workspace, the restart residual recomputed) until the solve
    reaches the 1e-10 true residual, checked again with the oracle's matrix
    (bound 1e-10 ||R|| plus 1e-11 sum_j |J_ij dx_j| for the two matrices'
    rounding)."""
    prob = SMALL["3d_p2_n3"]()
    case, ctx = _pair(prob)
    st0 = newton.initial_state(case)
    got = {}
    for m in (60, 1):
        ctx.set_options(gmres_m=m)
        ctx.set_state(st0.u, st0.p, st0.w_old)
        ctx.assemble()
        ctx.reset_profile()
        ls = ctx.solve()
        assert ls.true_relres <= 1e-10
        got[m] = (np.concatenate(ctx.increment()), ctx.profile().n_mgrow)
    assert got[60][1] == 0 and got[1][1] >= 1
    ctx.close()
    S = asm.assemble(case.mesh, case.itf, case.prm, st0.u, st0.p, st0.w_old, st0.s_p,
                     case.src_pnode, case.src_q0)
    J = asm.full_matrix(case.mesh, S)
    dx = got[1][0]
    r = J @ dx + S.R
    mag = abs(J) @ np.abs(dx)
    assert np.all(np.abs(r) <= 1e-10 * np.linalg.norm(S.R) + 1e-11 * mag)


def test_ir_restart_growth_on_stagnation():
    """GMRES-IR with one FP32 GMRES(1) cycle per refinement step stagnates as
    restarted GMRES(1) does; the inner restart length doubles until the
    refinement reaches the 1e-10 true residual, checked with the oracle's
    matrix as in the FP64 case."""
    prob = SMALL["3d_p2_n3"]()
    case, ctx = _pair(prob)
    st0 = newton.initial_state(case)
    ctx.set_options(precision=hf.HF_FP32_IR, gmres_m=1)
    ctx.set_state(st0.u, st0.p, st0.w_old)
    ctx.assemble()
    ctx.reset_profile()
    ls = ctx.solve()
    assert ls.true_relres <= 1e-10 and ls.ir_steps > 0
    assert ctx.profile().n_mgrow >= 1
    dx = np.concatenate(ctx.increment())
    ctx.close()
    S = asm.assemble(case.mesh, case.itf, case.prm, st0.u, st0.p, st0.w_old, st0.s_p,
                     case.src_pnode, case.src_q0)
    J = asm.full_matrix(case.mesh, S)
    r = J @ dx + S.R
    mag = abs(J) @ np.abs(dx)
    assert np.all(np.abs(r) <= 1e-10 * np.linalg.norm(S.R) + 1e-11 * mag)


@pytest.mark.parametrize("name", ["2d_p1_n9", "3d_p2_n3"])
def test_ir_fp64_finish(name):
    """The FP64 finish of a stalled GMRES-IR solve, forced for every solve
    (ir_stall_steps = 0): each solve runs entirely in FP64 GMRES on the
    refinement residual, and the converged states match the oracle."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    ctx.set_options(ir_stall_steps=0)
    ref = newton.run(case, prob.load_steps, solver="gmres")
    got = _gpu_run(ctx, case, prob.load_steps, hf.HF_FP32_IR)
    for (st, _), ((u, p, w, wo), ns) in zip(ref, got):
        assert np.linalg.norm(u - st.u) <= 1e-8 * np.linalg.norm(st.u)
        assert np.linalg.norm(p - st.p) <= 1e-8 * np.linalg.norm(st.p)
        assert ns.lin.ir_steps == 0 and ns.lin.fp64_iters == ns.lin.gmres_iters > 0
    ctx.close()


@pytest.mark.parametrize("name", list(SMALL))
def test_folded_operator(name):
    """J M^-1 x from the folded blocks equals M^-1 then J (FP64: 1e-13 of the
    largest entry; FP32: 1e-5, the two round differently) and the oracle's
    J M^-1 x with its own block inverses and Schur block (1e-10).  Two states
    per precision: the second build re-inverts and re-folds only what the
    crack elements touch."""
    torch = pytest.importorskip("torch")
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    rng = np.random.default_rng(9)
    for precision, dt, tol, seed in ((hf.HF_FP64, torch.float64, 1e-13, 8), (hf.HF_FP64, torch.float64, 1e-13, 10),
                                     (hf.HF_FP32_IR, torch.float32, 1e-5, 8),
                                     (hf.HF_FP32_IR, torch.float32, 1e-5, 10)):
        u, p, wo = _random_state(case, seed)
        ctx.set_options(precision=precision, gmres_maxit=1)
        ctx.set_state(u, p, wo)
        ctx.assemble()
        ctx.solve(check=False)  # builds the factors and the folded blocks; one iteration
        n = ctx.sizes.n_total
        x = rng.normal(size=n)
        xd = torch.tensor(x, device="cuda", dtype=dt)
        y1, y0 = torch.empty_like(xd), torch.empty_like(xd)
        torch.cuda.synchronize()
        ctx.apply_preconditioned(xd.data_ptr(), y1.data_ptr(), precision, folded=1)
        ctx.apply_preconditioned(xd.data_ptr(), y0.data_ptr(), precision, folded=0)
        torch.cuda.synchronize()
        a, b = y1.double().cpu().numpy(), y0.double().cpu().numpy()
        assert _rel(a, b) < tol
        if precision == hf.HF_FP64:
            S = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, newton.fluid_scale(case, wo, u),
                             case.src_pnode, case.src_q0)
            ref = solve.Operator(case.mesh, S)(solve.BlockJacobi(case.mesh, S)(x))
            assert _rel(a, ref) < 1e-10
    ctx.close()


@pytest.mark.parametrize("name", ["2d_p1_n9", "3d_p2_n3"])
def test_predictor_and_load_steps_parity(name):
    """The uniform-pressure elastic predictor (pressure and crack volume) and
    the load steps that start from it match the oracle."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    ref0 = newton.initial_state(case, predictor=True)
    st0 = newton.initial_state(case)
    ctx.set_state(st0.u, st0.p, st0.w_old)
    p0 = ctx.initial_guess()
    u, p, _, _ = ctx.get_state()
    assert p0 == pytest.approx(ref0.p[0], rel=1e-8)
    np.testing.assert_allclose(p, ref0.p, rtol=1e-8)
    assert np.linalg.norm(u - ref0.u) <= 1e-7 * np.linalg.norm(ref0.u)
    # the fluid rows carry the scale of the predictor's opening
    ctx.assemble()
    _, rp = ctx.residual()
    S = asm.assemble(case.mesh, case.itf, case.prm, ref0.u, ref0.p, ref0.w_old, ref0.s_p,
                     case.src_pnode, case.src_q0)
    assert np.linalg.norm(rp - S.R_p) <= 1e-6 * np.linalg.norm(S.R_p)
    ref = newton.run(case, prob.load_steps, predictor=True)
    got = _gpu_run(ctx, case, prob.load_steps, hf.HF_FP64, predictor=True)
    for (st, _), ((u, p, w, wo), ns) in zip(ref, got):
        assert np.linalg.norm(u - st.u) <= 1e-8 * np.linalg.norm(st.u)
        assert np.linalg.norm(p - st.p) <= 1e-8 * np.linalg.norm(st.p)
    ctx.close()


def test_determinism_bitwise():
    """Repeated assemble + solve from the same state give identical bits (the
    first assembly of a context is a full one, the later ones incremental:
    the second and third repetitions are compared)."""
    prob = SMALL["3d_p2_n3"]()
    case, ctx = _pair(prob)
    u, p, wo = _random_state(case, 6)
    res = []
    for _ in range(3):
        ctx.set_state(u, p, wo)
        ctx.assemble()
        st = ctx.solve()
        ru, rp = ctx.residual()
        du, dp = ctx.increment()
        res.append((ru, rp, du, dp, st.gmres_iters))
    for a, b in zip(res[1][:4], res[2][:4]):
        np.testing.assert_array_equal(a, b)
    assert res[1][4] == res[2][4]
    ctx.close()


def test_failure_paths():
    prob = SMALL["2d_p1_n9"]()
    case, ctx = _pair(prob)
    st0 = newton.initial_state(case)
    # call order
    with pytest.raises(hf.HFError) as ei:
        ctx.assemble()
    assert ei.value.status == hf.HF_ESTATE
    # non-finite state
    bad = st0.u.copy()
    bad[3] = np.nan
    with pytest.raises(hf.HFError) as ei:
        ctx.set_state(bad, st0.p, st0.w_old)
    assert ei.value.status == hf.HF_ENONFINITE
    # iteration cap: GMRES stops at 1 iteration, the state stays unchanged
    ctx.set_state(st0.u, st0.p, st0.w_old)
    ctx.set_options(gmres_maxit=1)
    with pytest.raises(hf.HFError) as ei:
        ctx.newton_solve()
    assert ei.value.status == hf.HF_ENOCONV
    u, p, _, _ = ctx.get_state()
    np.testing.assert_array_equal(u, st0.u)
    np.testing.assert_array_equal(p, st0.p)
    ctx.set_options(gmres_maxit=20000)
    ns = ctx.newton_solve()
    assert ns.converged
    ctx.close()


def test_block_inverses_fp32_on_matrix_cores():
    """FP32-IR on 30 x 30 blocks: the matrix-core inverses are FP32 inverses
    of the FP64 blocks (|X - A^-1| <= 50 eps32 kappa(A) |A^-1| per block),
    they are not the rounded FP64 inverses (a different computation), and
    with mfma_inverse = 0 the FP32 blocks are exactly the rounded FP64
    Gauss-Jordan inverses."""
    prob = SMALL["3d_p2_n3"]()
    case, ctx = _pair(prob)
    u, p, wo = _random_state(case, 8)
    E = np.arange(case.mesh.ne, dtype=np.int32)
    out = {}
    for mf in (1, 0):
        ctx.set_options(precision=hf.HF_FP32_IR, mfma_inverse=mf)
        ctx.reset_profile()
        ctx.set_state(u, p, wo)
        ctx.assemble()
        st = ctx.solve()
        assert st.status == hf.HF_OK and st.true_relres <= 1e-10
        prof = ctx.profile()
        assert prof.n_inv_mfma == mf and prof.n_inv_fallback == 0
        out[mf] = ctx.block_inverse(E, hf.HF_FP32_IR)
    _, blocks = ctx.block_rows(E)
    ctx.set_options(precision=hf.HF_FP64)
    ctx.solve()
    inv64 = ctx.block_inverse(E, hf.HF_FP64)
    eps32 = np.finfo(np.float32).eps
    for k in range(len(E)):
        A = blocks[k, 0]
        Ainv = np.linalg.inv(A)
        kappa = np.linalg.cond(A)
        err = np.abs(out[1][k] - Ainv).max() / np.abs(Ainv).max()
        assert err <= 50 * eps32 * kappa, (k, err, kappa)
        np.testing.assert_array_equal(out[0][k], inv64[k].astype(np.float32).astype(np.float64))
    assert not np.array_equal(out[1], out[0])
    ctx.close()


def _floating_pair():
    """Two P1 triangles that share only a vertex: no interior face, no
    clamped boundary, so each diagonal block is a bare element stiffness
    with the three rigid-body modes in its kernel (singular by construction)."""
    xyz = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [2.0, 0.0], [1.0, 1.0]])
    elem = np.array([[0, 1, 2], [1, 3, 4]], np.int32)
    return synth.Problem(2, 1, xyz, elem, np.zeros(5, np.uint8), np.zeros((0, 2), np.int32),
                         np.zeros(0, np.uint8), np.zeros(0, np.uint8), np.zeros(0, np.int64),
                         np.zeros(0), synth.Material(1.0, 0.25, 1e-3, 1e-4, 1e-3, 1.0), 1,
                         "floating")


@pytest.mark.parametrize("precision,mfma", [(hf.HF_FP64, 1), (hf.HF_FP32_IR, 0)],
                         ids=["fp64", "fp32ir"])
def test_singular_block_reports_esingular(precision, mfma):
    """A batch of a regular KGD instance and an instance whose element blocks
    are singular (forced from the host by the mesh itself): the solve
    reports HF_ESINGULAR for the second instance only, its Newton step
    keeps its state, and the first instance's increment equals its solo
    run bit for bit."""
    good = SMALL["2d_p1_n9"]()
    bad = _floating_pair()
    ctx = hf.context_for_problems([good, bad], precision=precision, mfma_inverse=mfma)
    case = Case.from_problem(good)
    st0 = newton.initial_state(case)
    ub = np.random.default_rng(3).normal(size=bad.n_udof) * 1e-3
    ctx.set_state(st0.u, st0.p, st0.w_old, inst=0)
    ctx.set_state(ub, np.zeros(0), np.zeros((0, 2)), inst=1)
    ctx.assemble()
    with pytest.raises(hf.HFError) as ei:
        ctx.solve()
    assert ei.value.status == hf.HF_ESINGULAR
    stats = ctx.solve(check=False)
    assert stats[1].status == hf.HF_ESINGULAR
    assert stats[0].status == hf.HF_OK and stats[0].true_relres <= 1e-10
    du0, dp0 = ctx.increment(0)
    ns = ctx.newton_step(check=False)
    assert ns[1].status == hf.HF_ESINGULAR and ns[0].status == hf.HF_OK
    np.testing.assert_array_equal(ctx.get_state(1)[0], ub)
    ctx.close()
    solo = hf.context_for_problem(good, precision=precision, mfma_inverse=mfma)
    solo.set_state(st0.u, st0.p, st0.w_old)
    solo.assemble()
    s1 = solo.solve()
    du1, dp1 = solo.increment()
    solo.close()
    assert s1.gmres_iters == stats[0].gmres_iters
    np.testing.assert_array_equal(du0, du1)
    np.testing.assert_array_equal(dp0, dp1)


@pytest.mark.parametrize("name", ["2d_p1_n9", "3d_p2_n3"])
@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_per_block_residuals(name, precision):
    """relres_u and relres_p are the true residual of the solve split over
    the displacement and pressure rows: recombined with the blocks of b they
    give true_relres, and both agree with the oracle's J applied to the
    increment (plain FP64 product, so to within its rounding)."""
    prob = SMALL[name]()
    case, ctx = _pair(prob)
    ctx.set_options(precision=precision)
    u, p, wo = _random_state(case, 21)
    ctx.set_state(u, p, wo)
    ctx.assemble()
    st = ctx.solve()
    ru, rp = ctx.residual()
    bu, bp = np.linalg.norm(ru), np.linalg.norm(rp)
    comb = np.hypot(st.relres_u * bu, st.relres_p * bp) / np.hypot(bu, bp)
    assert comb == pytest.approx(st.true_relres, rel=1e-6)
    du, dp = ctx.increment()
    S = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, newton.fluid_scale(case, wo, u),
                     case.src_pnode, case.src_q0)
    J = asm.full_matrix(case.mesh, S)
    r = -S.R - J @ np.concatenate([du, dp])
    n_u = case.mesh.n_u
    scale = np.abs(J).max() * np.abs(np.concatenate([du, dp])).max() * 1e-14
    assert abs(np.linalg.norm(r[:n_u]) - st.relres_u * bu) <= scale * np.sqrt(len(r))
    assert abs(np.linalg.norm(r[n_u:]) - st.relres_p * bp) <= scale * np.sqrt(len(r))
    assert st.true_relres <= 1e-10
    ctx.close()


@pytest.mark.parametrize("name", ["2d_p1_n9", "3d_p1_n4"])
def test_unscaled_fluid_rows(name):
    """scale_fluid_rows = 0: the fluid rows are those of eq. (discreteLubrication)
    as written (s_p = 1): R_p and D equal the oracle's assembled with s_p = 1,
    switching the option on a live context rescales them, and a converged
    load step ends at the same state as with the scaled rows (the Newton
    iterates do not depend on the row scale)."""
    prob = SMALL[name]()
    case = Case.from_problem(prob)
    ctx = hf.context_for_problem(prob, scale_fluid_rows=0)
    u, p, wo = _random_state(case, 31)
    ctx.set_state(u, p, wo)
    ctx.assemble()
    _, rp = ctx.residual()
    S1 = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, 1.0, case.src_pnode, case.src_q0)
    assert np.abs(rp - S1.R_p).max() <= 1e-12 * np.abs(S1.R_p).max()
    ctx.set_options(scale_fluid_rows=1)
    ctx.assemble()
    _, rp = ctx.residual()
    sp = newton.fluid_scale(case, wo, u)
    S2 = asm.assemble(case.mesh, case.itf, case.prm, u, p, wo, sp, case.src_pnode, case.src_q0)
    assert np.abs(rp - S2.R_p).max() <= 1e-12 * np.abs(S2.R_p).max()
    ctx.close()
    ref = newton.run(case, 1, solver="gmres")
    ctx = hf.context_for_problem(prob, scale_fluid_rows=0)
    st0 = newton.initial_state(case)
    ctx.set_state(st0.u, st0.p, st0.w_old)
    ns = ctx.newton_solve()
    u1, p1, _, _ = ctx.get_state()
    ctx.close()
    assert ns.converged
    st = ref[0][0]
    assert np.linalg.norm(u1 - st.u) <= 1e-8 * np.linalg.norm(st.u)
    assert np.linalg.norm(p1 - st.p) <= 1e-8 * np.linalg.norm(st.p)
