"""The allocation-free folded product against the allocating one.

hf_apply_preconditioned_noalloc computes y = J M^-1 x with the folded blocks
like hf_apply_preconditioned(folded = 1), but stages S^-1 x_p in the
library's fixed device array instead of a context buffer.  Same kernels,
same arithmetic: the two results must be equal bit for bit.  Two contexts
in a row, the second with fewer pressure unknowns (the array then still
holds the first call's longer staging vector), then the first one again;
FP64 and FP32-IR.
"""
import numpy as np
import pytest

import synth
from oracle import newton
from oracle.newton import Case

pytestmark = pytest.mark.gpu

import paper_1911_10275_amd as hf  # noqa: E402  (a broken package fails, never skips)
torch = pytest.importorskip("torch")


def _solved(prob, precision):
    case = Case.from_problem(prob)
    ctx = hf.context_for_problem(prob, precision=precision)
    st = newton.initial_state(case, predictor=True)
    ctx.set_state(st.u, st.p, st.w_old)
    ctx.assemble()
    ctx.solve()
    return ctx


def _compare(ctx, precision, seed):
    n = ctx.sizes.n_total
    dt = torch.float64 if precision == hf.HF_FP64 else torch.float32
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(n, generator=g, dtype=torch.float64).to(dt).to("cuda")
    y_ref = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    y_na = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    torch.cuda.synchronize()
    ctx.apply_preconditioned(x.data_ptr(), y_ref.data_ptr(), precision, folded=1)
    torch.cuda.synchronize()
    ctx.apply_preconditioned_noalloc(x.data_ptr(), y_na.data_ptr(), precision)
    torch.cuda.synchronize()
    a, b = y_ref.cpu().numpy(), y_na.cpu().numpy()
    assert np.all(np.isfinite(b))
    np.testing.assert_array_equal(a, b)
    return ctx.sizes.n_p


@pytest.mark.parametrize("precision", [hf.HF_FP64, hf.HF_FP32_IR], ids=["fp64", "fp32ir"])
def test_noalloc_folded_product_equals_allocating(precision):
    big = _solved(synth.penny_small(4, 2, steps=1), precision)
    small = _solved(synth.kgd_small(7, 1, steps=1), precision)
    try:
        # before any solve the folded operator does not exist
        fresh = hf.context_for_problem(synth.kgd_small(6, 1, steps=1), precision=precision)
        x = torch.zeros(fresh.sizes.n_total, dtype=torch.float64, device="cuda")
        with pytest.raises(hf.HFError) as ei:
            fresh.apply_preconditioned_noalloc(x.data_ptr(), x.data_ptr(), precision)
        assert ei.value.status == hf.HF_ESTATE
        fresh.close()
        n_big = _compare(big, precision, 1)
        n_small = _compare(small, precision, 2)
        assert n_small < n_big
        _compare(big, precision, 3)
    finally:
        big.close()
        small.close()
