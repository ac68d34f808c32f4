"""Validation of the GPU path against a closed form at scale: the crack volume
of a pressurised plane-strain crack (Sneddon, the toughness limit of the KGD
problem: uniform pressure, V = 2 pi p l^2 / E' in an infinite plane).

The elastic predictor (hf_initial_guess) solves the displacement rows under
a uniform unit pressure and returns p0 = Q0 dt / V1, so V1 = Q0 dt / p0 is the
crack volume per unit pressure.  The unit square is clamped all round, so the
computed volume sits below Sneddon's by the stiffening of the finite domain,
which falls like (l / L)^2.  With P2 elements and about 26 elements per crack
half-length l = 0.1, 0.05, 0.025 (256^2, 512^2, 1024^2 quads: 1.6M to 25M
displacement DOF, two-level preconditioner) the relative error must fall by
at least 2.5x per halving of l and end below 1%.  The oracle's own Sneddon pin
covers the same formula at sizes it can solve.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

import paper_1911_10275_amd as hf  # noqa: E402  (a broken package fails, never skips)


def _v1(n, nu=0.3, half_length=0.05):
    mat = synth.Material(E=1.0, nu=nu, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=1.0)
    prob = synth.kgd_problem(n, 2, 17, mat, 1e-4, half_length=half_length, ring=0, load_steps=1)
    ctx = hf.context_for_problem(prob, two_level=1)
    s = ctx.sizes
    ctx.set_state(np.zeros(s.n_u), np.zeros(s.n_p), np.zeros((s.n_face, s.nq_face)))
    p0 = ctx.initial_guess()
    ctx.close()
    v1 = float(np.sum(prob.src_q0)) * mat.dt / p0
    xs = prob.xyz[np.asarray(prob.crack_faces).ravel(), 0]
    ell = 0.5 * (xs.max() - xs.min())
    sneddon = 2.0 * math.pi * ell ** 2 / (mat.E / (1.0 - nu * nu))
    return v1 / sneddon - 1.0


def test_pressurised_crack_volume_converges_to_sneddon():
    errs = [_v1(n, half_length=hl) for n, hl in ((256, 0.1), (512, 0.05), (1024, 0.025))]
    print("relative error of the crack volume vs Sneddon:", errs, flush=True)
    assert all(e < 0.0 for e in errs)          # a clamped finite domain is stiffer
    assert abs(errs[0]) > 2.5 * abs(errs[1]) and abs(errs[1]) > 2.5 * abs(errs[2])
    assert abs(errs[2]) < 0.01
