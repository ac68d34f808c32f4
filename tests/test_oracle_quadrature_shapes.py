"""Pins of the oracle's quadrature, shape functions and element stiffness
against closed forms and invariants (no GPU)."""
import itertools
import math

import numpy as np
import pytest

from oracle import quadrature, shapes


def _monomial_exact(exps):
    # int over the reference simplex of prod x_i^a_i = prod a_i! / (sum a_i + d)!
    d = len(exps)
    return math.prod(math.factorial(a) for a in exps) / math.factorial(sum(exps) + d)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_conical_rule_exact_to_degree(dim, n):
    pts, w = quadrature.simplex_rule(dim, n)
    assert len(w) == n ** dim
    deg = 2 * n - 1
    for exps in itertools.product(range(deg + 1), repeat=dim):
        if sum(exps) > deg:
            continue
        val = float(np.sum(w * np.prod(pts ** np.array(exps), axis=1)))
        assert val == pytest.approx(_monomial_exact(exps), rel=1e-13, abs=1e-15)
    # and not exact one degree higher (the rule is exactly of degree 2n-1)
    exps = (2 * n,) + (0,) * (dim - 1)
    val = float(np.sum(w * pts[:, 0] ** (2 * n)))
    assert abs(val - _monomial_exact(exps)) > 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_face_rule_normalised(dim):
    for order in (1, 2):
        pts, w = quadrature.face_rule(dim, order)
        assert w.sum() == pytest.approx(1.0, rel=1e-15)
        assert np.all(pts >= 0) and np.all(pts.sum(axis=1) <= 1)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_lagrange_basis(dim, order):
    nb = shapes.node_bary(dim, order)
    P = shapes.phi(nb, dim, order)
    np.testing.assert_allclose(P, np.eye(len(nb)), atol=1e-15)          # nodal property
    rng = np.random.default_rng(0)
    lam = rng.dirichlet(np.ones(dim + 1), size=20)
    np.testing.assert_allclose(shapes.phi(lam, dim, order).sum(axis=1), 1.0, atol=1e-14)
    # derivative wrt barycentrics by central differences
    D = shapes.dphi_dlam(lam, dim, order)
    h = 1e-6
    for k in range(dim + 1):
        e = np.zeros(dim + 1); e[k] = h
        fd = (shapes.phi(lam + e, dim, order) - shapes.phi(lam - e, dim, order)) / (2 * h)
        np.testing.assert_allclose(D[..., k], fd, atol=1e-8)
