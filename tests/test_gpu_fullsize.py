"""Parity at the full size of the 3D penny workload (48,000 P2 tetrahedra,
1.44M displacement DOF), of its precision form (384,000 P2 tetrahedra,
11.52M displacement DOF, viscosity-dominated parameters) and of the
three-disk multi-crack workload (196,608 P2 tetrahedra, 5.9M displacement
DOF, three flat disks), in the launch configuration the benchmark times
(one context on the caller's torch stream, GMRES(60), graph-replayed
iterations, the two-level preconditioner).

The oracle cannot assemble or solve the whole system in test time, so it
checks sampled outputs it computes one by one: the residual rows, the
Jacobian block rows of a sample of elements (every 300th element plus every
element touching a fluid face; their faces' terms are all included), the
whole pressure block, and -- after a GPU solve -- the linear-system residual
R + J dx on the sampled rows and on every pressure row, which the true
relative residual of 1e-10 bounds.  Tolerances: Jacobian entries 1e-12
relative to the largest compared entry (as for the small meshes); residual
rows 1e-12 relative to the largest of their entries and of sum_j |J_ij x_j|
(at a near-equilibrium state such as the predictor's the residual is a
cancellation of terms of that size, and its rounding error scales with
them, not with the small result); the solve residual 1e-10 ||R|| plus a
rounding allowance of 1e-11 sum_j |J_ij dx_j| for the difference between the
oracle's and the GPU's matrix entries.
"""
import numpy as np
import pytest

import synth
from oracle import assemble as asm
from oracle import newton
from oracle.newton import Case

pytestmark = pytest.mark.gpu

import paper_1911_10275_amd as hf  # noqa: E402  (a broken package fails, never skips)
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", params=[2, 3, 5], ids=["penny48k", "penny384k", "multicrack197k"])
def penny(request):
    prob = synth.config(request.param)
    case = Case.from_problem(prob)
    m = case.mesh
    fa = case.itf.active_faces
    near = np.unique(np.concatenate([m.face_em[fa], m.face_ep[fa]]))
    E = np.unique(np.concatenate([np.arange(0, m.ne, 300), near]))
    F = np.nonzero(np.isin(m.face_em, E) | np.isin(m.face_ep, E))[0]
    F = np.unique(np.concatenate([F, fa]))
    stream = torch.cuda.current_stream().cuda_stream
    ctx = hf.context_for_problem(prob, device=0, stream=stream, gmres_m=60, two_level=1)
    yield prob, case, ctx, E, F
    ctx.close()


def _oracle(case, E, F, u, p, w_old):
    s_p = newton.fluid_scale(case, w_old, u)
    return asm.assemble(case.mesh, case.itf, case.prm, u, p, w_old, s_p, case.src_pnode,
                        case.src_q0, faces=F, elements=E)


def _rel(a, b):
    s = max(np.abs(a).max(), np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / s


def _term_size(case, E, S, ref, cols, u, p):
    """sum_j |J_ij x_j| on the sampled displacement rows and the pressure rows."""
    bu = case.mesh.bu
    rows = (E[:, None] * bu + np.arange(bu)[None, :]).reshape(-1)
    mag_u = abs(S.B.tocsr()[rows]) @ np.abs(p)
    for k, e in enumerate(E):
        sl = slice(k * bu, (k + 1) * bu)
        for s in range(cols.shape[1]):
            c = e if s == 0 else cols[k, s]
            if c >= 0:
                blk = S.A_diag[e] if s == 0 else ref[(e, c)]
                mag_u[sl] += np.abs(blk) @ np.abs(u[c * bu:(c + 1) * bu])
    mag_p = abs(S.C) @ np.abs(u) + abs(S.D) @ np.abs(p)
    return mag_u, mag_p


def _check_assembly(ctx, case, E, F, S, u, p):
    m = case.mesh
    bu = m.bu
    ru, rp = ctx.residual()
    rows = (E[:, None] * bu + np.arange(bu)[None, :]).reshape(-1)
    cols, blocks = ctx.block_rows(E)
    ref = {}
    for f in F:
        ref[(m.face_em[f], m.face_ep[f])] = S.A_mp[f]
        ref[(m.face_ep[f], m.face_em[f])] = S.A_pm[f]
    mag_u, mag_p = _term_size(case, E, S, ref, cols, u, p)
    scale_u = max(np.abs(S.R_u[rows]).max(), mag_u.max())
    scale_p = max(np.abs(S.R_p).max(), mag_p.max())
    assert np.abs(ru[rows] - S.R_u[rows]).max() <= 1e-12 * scale_u
    assert np.abs(rp - S.R_p).max() <= 1e-12 * scale_p
    got, want = [], []
    for k, e in enumerate(E):
        got.append(blocks[k, 0])
        want.append(S.A_diag[e])
        for s in range(1, cols.shape[1]):
            c = cols[k, s]
            if c >= 0:
                got.append(blocks[k, s])
                want.append(ref[(e, c)])
    assert _rel(np.array(got), np.array(want)) < 1e-12
    n_p = case.itf.n_p
    D = np.empty((n_p, n_p))
    st = ctx.lib.hf_get_coupling(ctx.h, 0, None, None, D.ctypes.data_as(hf.C.c_void_p))
    assert st == hf.HF_OK
    assert _rel(D, S.D.toarray()) < 1e-12


def _check_solve(ctx, case, E, S):
    """R + J dx on the sampled displacement rows and every pressure row."""
    m = case.mesh
    bu = m.bu
    du, dp = ctx.increment()
    ru, rp = ctx.residual()
    Rn = np.sqrt(np.dot(ru, ru) + np.dot(rp, rp))
    cols, blocks = ctx.block_rows(E)
    rows = (E[:, None] * bu + np.arange(bu)[None, :]).reshape(-1)
    # displacement rows with the oracle's blocks: diagonal, neighbours, B
    r_u = S.R_u[rows].copy()
    mag = np.zeros_like(r_u)
    Bcsr = S.B.tocsr()[rows]
    r_u += Bcsr @ dp
    mag += abs(Bcsr) @ np.abs(dp)
    face_of = {}
    for f in np.nonzero(np.isin(m.face_em, E) | np.isin(m.face_ep, E))[0]:
        face_of[(m.face_em[f], m.face_ep[f])] = S.A_mp[f]
        face_of[(m.face_ep[f], m.face_em[f])] = S.A_pm[f]
    for k, e in enumerate(E):
        sl = slice(k * bu, (k + 1) * bu)
        for s in range(cols.shape[1]):
            c = e if s == 0 else cols[k, s]
            if c < 0:
                continue
            blk = S.A_diag[e] if s == 0 else face_of[(e, c)]
            x = du[c * bu:(c + 1) * bu]
            r_u[sl] += blk @ x
            mag[sl] += np.abs(blk) @ np.abs(x)
    assert np.all(np.abs(r_u) <= 1e-10 * Rn + 1e-11 * mag)
    # every pressure row
    r_p = S.R_p + S.C @ du + S.D @ dp
    mag_p = abs(S.C) @ np.abs(du) + abs(S.D) @ np.abs(dp)
    assert np.all(np.abs(r_p) <= 1e-10 * Rn + 1e-11 * mag_p)


def test_fullsize_assembly_random_state(penny):
    prob, case, ctx, E, F = penny
    m = case.mesh
    rng = np.random.default_rng(7)
    u = rng.normal(size=m.n_u) * 1e-3
    p = rng.uniform(0.0, 2e-3, case.itf.n_p)
    wo = rng.uniform(0.0, 1e-3, (m.nf, m.nq))
    ctx.set_state(u, p, wo)
    ctx.assemble()
    _check_assembly(ctx, case, E, F, _oracle(case, E, F, u, p, wo), u, p)


@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_fullsize_predictor_state_solve(penny, precision):
    prob, case, ctx, E, F = penny
    m = case.mesh
    ctx.set_options(precision=precision)
    st0 = newton.initial_state(case)
    ctx.set_state(st0.u, st0.p, st0.w_old)
    ctx.initial_guess()
    u, p, _, wo = ctx.get_state()
    ctx.assemble()
    S = _oracle(case, E, F, u, p, wo)
    _check_assembly(ctx, case, E, F, S, u, p)
    st = ctx.solve()
    assert st.status == hf.HF_OK and st.true_relres <= 1e-10
    _check_solve(ctx, case, E, S)


def _crack_volume(case, w):
    m = case.mesh
    fa = case.itf.active_faces
    return float(np.sum(m.fq_w[None, :] * m.area[fa][:, None] * w[fa]))


def test_fullsize_load_steps(penny):
    """The first two load steps from the predictor, in FP64 and in FP32-IR:
    every Newton iteration's solve reaches the true relative residual 1e-10
    and Newton converges; both precisions end at the same states (1e-8);
    the crack holds the injected volume, sum Q0 n dt after load step n
    (1e-8: summing the fluid rows over all pressure nodes cancels the flux
    terms, since the test functions sum to one, and leaves the global
    balance of stored and injected volume); and at each converged state the
    oracle's residual on the sampled displacement rows and on every pressure
    row vanishes to 1e-9 of the size of its terms, sum_j |J_ij x_j|."""
    prob, case, ctx, E, F = penny
    m = case.mesh
    q = float(np.sum(case.src_q0)) * prob.material.dt
    finals = {}
    for precision in (hf.HF_FP64, hf.HF_FP32_IR):
        ctx.set_options(precision=precision)
        st0 = newton.initial_state(case)
        ctx.set_state(st0.u, st0.p, st0.w_old)
        ctx.initial_guess()
        states = []
        for n in (1, 2):
            its = 0
            for _ in range(25):
                ns = ctx.newton_step(check=False)
                assert ns.status == hf.HF_OK and ns.lin.true_relres <= 1e-10, (precision, n, its)
                its += 1
                if ns.converged:
                    break
            assert ns.converged, (precision, n)
            u, p, w, wo = ctx.get_state()
            assert _crack_volume(case, w) == pytest.approx(n * q, rel=1e-8)
            if precision == hf.HF_FP64:
                S = _oracle(case, E, F, u, p, wo)
                ctx.assemble()
                cols, _ = ctx.block_rows(E)
                ref = {}
                for f in F:
                    ref[(m.face_em[f], m.face_ep[f])] = S.A_mp[f]
                    ref[(m.face_ep[f], m.face_em[f])] = S.A_pm[f]
                mag_u, mag_p = _term_size(case, E, S, ref, cols, u, p)
                rows = (E[:, None] * m.bu + np.arange(m.bu)[None, :]).reshape(-1)
                assert np.all(np.abs(S.R_u[rows]) <= 1e-9 * mag_u.max())
                assert np.all(np.abs(S.R_p) <= 1e-9 * mag_p.max())
            print(f"{prob.name} precision {precision} load step {n}: {its} Newton iterations",
                  flush=True)
            states.append((u, p))
            ctx.end_load_step()
        finals[precision] = states
    for (u64, p64), (u32, p32) in zip(finals[hf.HF_FP64], finals[hf.HF_FP32_IR]):
        assert np.linalg.norm(u32 - u64) <= 1e-8 * np.linalg.norm(u64)
        assert np.linalg.norm(p32 - p64) <= 1e-8 * np.linalg.norm(p64)
