"""Contexts of different element types driven concurrently.

A 2D P1, a 2D P2 and a 3D P2 context, each on its own stream, are driven
from two host threads at the same time (as the benchmark drives the P1 and
P2 halves of the ensemble): repeated assemblies at seeded states, then the
predictor and one converged load step.  Every context owns its quadrature
rules and all its device data, so each result must equal the oracle's at
the same state element by element (R and every block row of A, B, C, D to
1e-12 of the largest entry; converged u, p, w to 1e-8).
"""
import threading

import numpy as np
import pytest

import synth
from oracle import assemble as asm
from oracle import newton
from oracle.newton import Case

pytestmark = pytest.mark.gpu

import paper_1911_10275_amd as hf  # noqa: E402  (a broken package fails, never skips)
torch = pytest.importorskip("torch")

N_ASSEMBLIES = 6


def _problems():
    return {
        "2d_p1": synth.kgd_small(9, 1, steps=1),
        "2d_p2": synth.kgd_small(7, 2, steps=1),
        "3d_p2": synth.penny_problem(3, 2, 21, synth.Material(1.0, 0.2, 1e-3, 1e-4, 1e-3, 1.0),
                                     1e-4, radius=0.34, ring_width=0.2, load_steps=1,
                                     name="penny_n3_p2"),
    }


def _state(case, seed):
    m = case.mesh
    rng = np.random.default_rng(seed)
    return (rng.normal(size=m.n_u) * 0.05, rng.uniform(0.0, 2e-3, case.itf.n_p),
            rng.uniform(0.0, 1e-2, (m.nf, m.nq)))


def _drive(name, case, ctx, out, errors):
    """Assemblies at seeded states, then predictor + one load step."""
    try:
        rec = []
        for k in range(N_ASSEMBLIES):
            u, p, wo = _state(case, 100 + k)
            ctx.set_state(u, p, wo)
            ctx.assemble()
            ru, rp = ctx.residual()
            cols, blocks = ctx.block_rows(np.arange(case.mesh.ne))
            rec.append((k, ru, rp, cols, blocks, ctx.coupling()))
        st0 = newton.initial_state(case)
        ctx.set_state(st0.u, st0.p, st0.w_old)
        ctx.initial_guess()
        ns = ctx.newton_solve()
        ctx.end_load_step()
        out[name] = (rec, ns, ctx.get_state())
    except Exception as exc:  # reported by the main thread
        errors.append((name, exc))


def _rel(a, b):
    s = max(np.abs(a).max(), np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / s


def test_concurrent_contexts_match_oracle():
    probs = _problems()
    cases = {k: Case.from_problem(p) for k, p in probs.items()}
    streams = {k: torch.cuda.Stream() for k in probs}
    ctxs = {k: hf.context_for_problem(p, device=0, stream=streams[k].cuda_stream)
            for k, p in probs.items()}
    out, errors = {}, []

    def thread_a():
        _drive("2d_p1", cases["2d_p1"], ctxs["2d_p1"], out, errors)

    def thread_b():
        # the 2D P2 and the 3D P2 contexts, interleaved call by call
        for name in ("2d_p2", "3d_p2"):
            _drive(name, cases[name], ctxs[name], out, errors)

    ths = [threading.Thread(target=thread_a), threading.Thread(target=thread_b)]
    try:
        for t in ths:
            t.start()
        for t in ths:
            t.join()
    finally:
        torch.cuda.synchronize()
        for c in ctxs.values():
            c.close()
    assert not errors, errors
    for name, case in cases.items():
        m = case.mesh
        rec, ns, (u, p, _, wo) = out[name]
        for k, ru, rp, cols, blocks, (B, Cm, D) in rec:
            us, ps, wos = _state(case, 100 + k)
            S = asm.assemble(m, case.itf, case.prm, us, ps, wos, newton.fluid_scale(case, wos, us),
                             case.src_pnode, case.src_q0)
            assert _rel(ru, S.R_u) < 1e-12, (name, k)
            assert _rel(rp, S.R_p) < 1e-12, (name, k)
            ref = {(e, e): S.A_diag[e] for e in range(m.ne)}
            for f in range(m.nf):
                ref[(m.face_em[f], m.face_ep[f])] = S.A_mp[f]
                ref[(m.face_ep[f], m.face_em[f])] = S.A_pm[f]
            scale = max(np.abs(b).max() for b in ref.values())
            err = max(np.abs(blocks[e, s] - ref[(e, cols[e, s])]).max()
                      for e in range(m.ne) for s in range(cols.shape[1]) if cols[e, s] >= 0)
            assert err / scale < 1e-12, (name, k)
            assert _rel(B, S.B.toarray()) < 1e-12 and _rel(Cm, S.C.toarray()) < 1e-12
            assert _rel(D, S.D.toarray()) < 1e-12, (name, k)
        assert ns.converged == 1 and ns.lin.true_relres <= 1e-10, name
        (ref_state, _), = newton.run(case, 1, predictor=True)
        fa = case.itf.active_faces
        assert np.linalg.norm(u - ref_state.u) <= 1e-8 * np.linalg.norm(ref_state.u), name
        assert np.linalg.norm(p - ref_state.p) <= 1e-8 * np.linalg.norm(ref_state.p), name
        assert (np.linalg.norm(wo[fa] - ref_state.w_old[fa])
                <= 1e-8 * np.linalg.norm(ref_state.w_old[fa])), name
