"""Linear solvers for the Newton correction J dx = -R (oracle).

The paper solves the linearised system with a domain-decomposition
preconditioned Krylov method with subdomain LU (Sec. "Computational
framework", implementation paragraph).  The oracle provides:

  * dense LU with partial pivoting (library) -- the reference truth on tiny
    meshes;
  * restarted right-preconditioned GMRES(m) with modified Gram-Schmidt and
    Givens rotations, x0 = 0, stopping on the explicitly recomputed true
    residual ||b - J x|| <= rtol ||b||;
  * the block-Jacobi preconditioner: the inverse (LU with partial pivoting,
    library) of every diagonal element block of A; the pressure unknowns
    form one more block holding the approximate Schur complement
    S = D - C M_A^-1 B (M_A = the element blocks), also inverted by LU.  A
    reading: D alone vanishes at zero opening (K(0) = 0) and a scalar
    fallback on those rows makes restarted GMRES stagnate;
  * GMRES-IR: FP64 outer residual and update, FP32 inner GMRES on
    round-to-nearest FP32 copies of J and of the block inverses.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assemble import System, bsr_A
from .mesh import Mesh


class Operator:
    """y = J x with J = [[A, B], [C, D]] in the given floating type."""

    def __init__(self, mesh: Mesh, sysm: System, dtype=np.float64):
        self.n_u = mesh.n_u
        self.n = mesh.n_u + sysm.R_p.shape[0]
        self.A = bsr_A(mesh, sysm).astype(dtype)
        self.B = sysm.B.astype(dtype)
        self.C = sysm.C.astype(dtype)
        self.D = sysm.D.astype(dtype)
        self.dtype = dtype

    def __call__(self, x):
        xu, xp = x[:self.n_u], x[self.n_u:]
        yu = self.A @ xu
        if xp.size:
            yu = yu + self.B @ xp
            yp = self.C @ xu + self.D @ xp
        else:
            yp = xp
        return np.concatenate([yu, yp]).astype(self.dtype, copy=False)


class BlockJacobi:
    """z = M^-1 r, M = blockdiag(A_ee, ..., S) with S = D - C M_A^-1 B."""

    def __init__(self, mesh: Mesh, sysm: System, dtype=np.float64):
        self.ne, self.bu = mesh.ne, mesh.bu
        inv = np.linalg.inv(sysm.A_diag)                      # LU + partial pivoting
        if not np.all(np.isfinite(inv)):
            raise np.linalg.LinAlgError("singular element block")
        n_p = sysm.D.shape[0]
        if n_p:
            Minv_A = _block_diag(inv)
            S = sysm.D.toarray() - (sysm.C @ (Minv_A @ sysm.B)).toarray()
            Sinv = np.linalg.inv(S)
            if not np.all(np.isfinite(Sinv)):
                raise np.linalg.LinAlgError("singular pressure block")
        else:
            Sinv = np.zeros((0, 0))
        self.inv = inv.astype(dtype)
        self.Sinv = Sinv.astype(dtype)
        self.dtype = dtype

    def __call__(self, r):
        ru = r[:self.ne * self.bu].reshape(self.ne, self.bu)
        zu = np.einsum("eij,ej->ei", self.inv, ru).reshape(-1)
        zp = self.Sinv @ r[self.ne * self.bu:]
        return np.concatenate([zu, zp]).astype(self.dtype, copy=False)


def _block_diag(blocks: np.ndarray) -> sp.bsr_matrix:
    ne, b, _ = blocks.shape
    return sp.bsr_matrix((blocks, np.arange(ne), np.arange(ne + 1)), shape=(ne * b, ne * b))


@dataclasses.dataclass
class SolveStats:
    iterations: int = 0
    restarts: int = 0
    ir_steps: int = 0
    true_relres: float = np.inf
    converged: bool = False


def gmres(op: Callable, b: np.ndarray, prec: Callable, m: int = 60, rtol: float = 1e-10,
          maxit: int = 20000, x0: Optional[np.ndarray] = None, dtype=np.float64,
          stats: Optional[SolveStats] = None, explicit_check: bool = True):
    """Right-preconditioned restarted GMRES(m), modified Gram-Schmidt.

    Solves op(x) = b, x = x0 + M^-1 V y each cycle.  A cycle ends when the
    recursive residual estimate |g_{j+1}| <= rtol ||b|| or after m steps; the
    explicit residual b - op(x) is then recomputed and decides convergence.
    With ``explicit_check=False`` (the inner solve of GMRES-IR, whose outer
    loop recomputes the residual in FP64) the recursive estimate decides.
    """
    st = stats if stats is not None else SolveStats()
    b = b.astype(dtype)
    n = b.shape[0]
    x = np.zeros(n, dtype=dtype) if x0 is None else x0.astype(dtype).copy()
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        st.true_relres, st.converged = 0.0, True
        return x, st
    r = b - op(x) if x0 is not None else b.copy()
    while True:
        beta = float(np.linalg.norm(r))
        if beta <= rtol * bnorm:
            st.true_relres, st.converged = beta / bnorm, True
            return x, st
        if st.iterations >= maxit:
            st.true_relres = beta / bnorm
            return x, st
        V = np.zeros((m + 1, n), dtype=dtype)
        H = np.zeros((m + 1, m), dtype=np.float64)
        cs = np.zeros(m); sn = np.zeros(m)
        g = np.zeros(m + 1); g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            wv = op(prec(V[j]))
            st.iterations += 1
            for i in range(j + 1):
                H[i, j] = float(np.dot(wv, V[i]))
                wv = wv - dtype(H[i, j]) * V[i]
            H[j + 1, j] = float(np.linalg.norm(wv))
            if H[j + 1, j] != 0.0:
                V[j + 1] = wv / dtype(H[j + 1, j])
            for i in range(j):                      # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (1.0, 0.0) if den == 0.0 else (H[j, j] / den, H[j + 1, j] / den)
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            if abs(g[j + 1]) <= rtol * bnorm or st.iterations >= maxit:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + prec((V[:k].T @ y.astype(dtype)).astype(dtype))
        if not explicit_check and (abs(g[k]) <= rtol * bnorm or st.iterations >= maxit):
            st.true_relres, st.converged = abs(g[k]) / bnorm, abs(g[k]) <= rtol * bnorm
            return x, st
        r = b - op(x)
        st.restarts += 1


def gmres_ir(op64: Callable, op32: Callable, prec32: Callable, b: np.ndarray, m: int = 60,
             rtol: float = 1e-10, rtol_inner: float = 1e-2, maxit: int = 20000,
             max_outer: int = 100, inner_maxit: Optional[int] = None):
    """GMRES-IR: r = b - J x in FP64; inner FP32 GMRES on J32 d = r until
    its recursive residual estimate reaches rtol_inner (at most
    ``inner_maxit`` iterations, default 20 m); x += d in FP64; until
    ||r|| <= rtol ||b||."""
    cap = 20 * m if inner_maxit is None else inner_maxit
    st = SolveStats()
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        st.true_relres, st.converged = 0.0, True
        return x, st
    r = b.copy()
    for _ in range(max_outer):
        rn = float(np.linalg.norm(r))
        st.true_relres = rn / bnorm
        if rn <= rtol * bnorm:
            st.converged = True
            return x, st
        inner = SolveStats()
        d, inner = gmres(op32, (r / rn).astype(np.float32), prec32, m=m, rtol=rtol_inner,
                         maxit=min(cap, maxit - st.iterations), dtype=np.float32,
                         stats=inner, explicit_check=False)
        st.iterations += inner.iterations
        st.ir_steps += 1
        x = x + rn * d.astype(np.float64)
        r = b - op64(x)
        if st.iterations >= maxit:
            break
    st.true_relres = float(np.linalg.norm(r)) / bnorm
    st.converged = st.true_relres <= rtol
    return x, st


def dense_solve(mesh: Mesh, sysm: System, rhs: np.ndarray) -> np.ndarray:
    """Dense LU with partial pivoting (library) of the full Jacobian."""
    from .assemble import full_matrix
    J = full_matrix(mesh, sysm).toarray()
    lu = sla.lu_factor(J)
    return sla.lu_solve(lu, rhs)
