"""Kernel schedules, solver choices and the autotuner.

Every schedule variant (lanes per row of the Jacobian product and of the
block-Jacobi apply, rows per thread of the Gram-Schmidt passes) and every
orthogonalisation scheme must leave the converged Newton states within
the parity bar of the FP64 oracle (1e-8) with every solve at a true relative
residual of 1e-10.  The autotuner must return valid choices, apply them, and
read them back from its cache file without timing.
"""
import numpy as np
import pytest

import synth
from oracle import newton
from oracle.newton import Case

pytestmark = pytest.mark.gpu

import paper_1911_10275_amd as hf  # noqa: E402  (a broken package fails, never skips)

CASES = {
    "2d_p1_n9": lambda: synth.kgd_small(9, 1, steps=2),
    "2d_p2_n7": lambda: synth.kgd_small(7, 2, steps=2),
    "3d_p2_n3": lambda: synth.penny_problem(3, 2, 21, synth.Material(1.0, 0.2, 1e-3, 1e-4, 1e-3, 1.0),
                                            1e-4, radius=0.34, ring_width=0.2, load_steps=2),
}
VARIANTS = [
    dict(spmv_var=1, prec_var=1, ortho_var=1, reorth=1),
    dict(spmv_var=0, prec_var=1, ortho_var=2, reorth=2),
    dict(spmv_var=1, prec_var=0, ortho_var=0, reorth=0, gmres_m=90),
    dict(spmv_var=0, prec_var=0, ortho_var=0, reorth=4),
    dict(spmv_var=1, prec_var=1, ortho_var=1, reorth=3, gmres_m=90),
]


_REF = {}


def _reference(name):
    if name not in _REF:
        prob = CASES[name]()
        _REF[name] = (prob, newton.run(Case.from_problem(prob), 2, predictor=True))
    return _REF[name]


def _steps(ctx, case, steps, precision):
    ctx.set_options(precision=precision)
    st0 = newton.initial_state(case)
    ctx.set_state(st0.u, st0.p, st0.w_old)
    ctx.initial_guess()
    out = []
    for _ in range(steps):
        ns = ctx.newton_solve()
        assert ns.converged and ns.lin.true_relres <= 1e-10
        ctx.end_load_step()
        out.append(ctx.get_state())
    return out


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("vi", range(len(VARIANTS)))
@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_variants_match_oracle(name, vi, precision):
    prob, ref = _reference(name)
    case = Case.from_problem(prob)
    ctx = hf.context_for_problem(prob)
    ctx.set_tuning(**VARIANTS[vi])
    t = ctx.tuning()
    for k, v in VARIANTS[vi].items():
        assert getattr(t, k) == v
    got = _steps(ctx, case, 2, precision)
    ctx.close()
    for (st, _), (u, p, w, wo) in zip(ref, got):
        assert np.linalg.norm(u - st.u) <= 1e-8 * np.linalg.norm(st.u)
        assert np.linalg.norm(p - st.p) <= 1e-8 * np.linalg.norm(st.p)


def test_set_tuning_rejects_out_of_range():
    ctx = hf.context_for_problem(synth.kgd_small(6, 1))
    before = ctx.tuning().as_dict()
    for bad in (dict(spmv_var=2), dict(ortho_var=3), dict(reorth=5), dict(reorth=-1), dict(gmres_m=300)):
        with pytest.raises(hf.HFError) as ei:
            ctx.set_tuning(**bad)
        assert ei.value.status == hf.HF_EINVAL
        assert ctx.tuning().as_dict() == before
    ctx.close()


@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_autotune_and_cache(tmp_path, precision):
    prob = CASES["3d_p2_n3"]()
    case = Case.from_problem(prob)
    cache = tmp_path / "tune.txt"
    ctx = hf.context_for_problem(prob, precision=precision)
    st0 = newton.initial_state(case)
    ctx.set_state(st0.u, st0.p, st0.w_old)
    ctx.initial_guess()
    ctx.assemble()
    t = ctx.autotune(level=1, cache_path=str(cache))
    assert t.spmv_var in (0, 1) and t.prec_var in (0, 1) and t.ortho_var in (0, 1, 2)
    assert t.reorth in ((0, 3) if precision == hf.HF_FP64 else (0, 4)) and t.gmres_m in (30, 60, 120)
    assert not (precision == hf.HF_FP32_IR and t.reorth == 4 and t.gmres_m > 60)
    assert ctx.tuning().as_dict() == t.as_dict()
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:] == [str(v) for v in t.as_dict().values()]
    # the tuned context still solves to the bar
    st = ctx.solve()
    assert st.status == hf.HF_OK and st.true_relres <= 1e-10
    ctx.close()
    # a second context reads the choice back without timing (no new line)
    ctx2 = hf.context_for_problem(prob, precision=precision)
    ctx2.set_state(st0.u, st0.p, st0.w_old)
    ctx2.assemble()
    t2 = ctx2.autotune(level=1, cache_path=str(cache))
    assert t2.as_dict() == t.as_dict()
    assert len(cache.read_text().splitlines()) == 1
    ctx2.close()
