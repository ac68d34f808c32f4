"""Element stiffness pins: P1 closed form |e| B^T D B (engineering-strain
Voigt form, written independently of the oracle's tensor form), symmetry,
positive semi-definiteness and the rigid-body kernel (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import assemble as asm
from oracle.mesh import Interfaces, Mesh


def _element_blocks(dim, order, nu=0.3, E=2.5):
    if dim == 2:
        xyz, elem, _ = synth.grid2d(2, seed=5)
    else:
        xyz, elem, _ = synth.kuhn3d(1, seed=5)
    m = Mesh(dim, order, xyz, elem)           # no clamped nodes
    itf = Interfaces(m)
    prm = asm.Params(E, nu, 1e-3, 1e-4, 1e-3, 1.0)
    S = asm.assemble(m, itf, prm, np.zeros(m.n_u), np.zeros(0), np.zeros((m.nf, m.nq)),
                     1.0, [], [])
    # volume part only = A_diag minus the face self-terms: recompute with no faces
    S0 = asm.assemble(m, itf, prm, np.zeros(m.n_u), np.zeros(0), np.zeros((m.nf, m.nq)),
                      1.0, [], [], faces=np.zeros(0, dtype=np.int64))
    return m, S0.A_diag, prm


def test_p1_triangle_closed_form():
    m, K, prm = _element_blocks(2, 1)
    E, nu = prm.E, prm.nu
    Dm = E / ((1 + nu) * (1 - 2 * nu)) * np.array([[1 - nu, nu, 0], [nu, 1 - nu, 0],
                                                   [0, 0, (1 - 2 * nu) / 2]])
    for e in range(m.ne):
        (x1, y1), (x2, y2), (x3, y3) = m.xyz[m.elem[e]]
        two_a = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1)
        b = [y2 - y3, y3 - y1, y1 - y2]
        c = [x3 - x2, x1 - x3, x2 - x1]
        B = np.zeros((3, 6))
        for i in range(3):
            B[0, 2 * i] = b[i]; B[1, 2 * i + 1] = c[i]
            B[2, 2 * i] = c[i]; B[2, 2 * i + 1] = b[i]
        B /= two_a
        Kref = abs(two_a) / 2 * B.T @ Dm @ B
        np.testing.assert_allclose(K[e], Kref, rtol=1e-12, atol=1e-12 * np.abs(Kref).max())


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_stiffness_kernel_is_rigid_motions(dim, order):
    m, K, _ = _element_blocks(dim, order)
    X = m.node_xyz()                                   # (ne, nn, d)
    n_rigid = 3 if dim == 2 else 6
    for e in range(m.ne):
        Ke = K[e]
        np.testing.assert_allclose(Ke, Ke.T, atol=1e-13 * np.abs(Ke).max())
        ev = np.linalg.eigvalsh(Ke)
        tol = 1e-10 * ev.max()
        assert np.sum(np.abs(ev) < tol) == n_rigid
        assert ev.min() > -tol
        # rigid modes: translations and infinitesimal rotations are in the kernel
        modes = []
        for c in range(dim):
            t = np.zeros((m.nn, dim)); t[:, c] = 1.0; modes.append(t.ravel())
        pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
        for a, b in pairs:
            r = np.zeros((m.nn, dim)); r[:, a] = -X[e, :, b]; r[:, b] = X[e, :, a]
            modes.append(r.ravel())
        for v in modes:
            assert np.linalg.norm(Ke @ v) <= 1e-12 * np.abs(Ke).max() * np.linalg.norm(v)
