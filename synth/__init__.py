"""Seeded synthetic inputs for the hydraulic-fracture Newton step.

This package produces *inputs only*: meshes, Dirichlet flags, the crack
(pre-cracked and cohesive faces, given by their sorted vertex ids), injection
points and material/run parameters.  It contains none of the method's
arithmetic (no shape functions, quadrature, residuals or solvers), so that
both the CPU oracle and the HIP library can be fed from it without sharing
any code of the method.

Workload shapes follow the paper's verification problems: a plane-strain KGD
crack on a 2D domain (Sec. "Verification of the fully-coupled algorithm") and
a penny-shaped crack in a 3D cube (Sec. "... penny-shaped crack"), at
nondimensional scale (unit domain, E ~ 1).

Random numbers come from a counter-based SplitMix64: draw k of stream s under
seed S is ``mix(base(S, s) + (k + 1) * 0x9E3779B97F4A7C15)`` where ``mix`` is
the SplitMix64 output function and ``base(S, s) = mix(S * 0x100000001B3 + s)``.
Uniform doubles use the top 53 bits.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# streams used by the generators (fixed, documented)
STREAM_JITTER = 1
STREAM_DISK = 2
STREAM_ENSEMBLE = 3


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, stream: int, count: int) -> np.ndarray:
    """``count`` uniform doubles in [0, 1) from (seed, stream), counter-based."""
    with np.errstate(over="ignore"):
        base = _mix(np.array([np.uint64(seed) * np.uint64(0x100000001B3)
                              + np.uint64(stream)], dtype=np.uint64))[0]
        k = np.arange(1, count + 1, dtype=np.uint64)
        x = _mix(base + k * _GOLDEN)
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# Problem container
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Material:
    E: float
    nu: float
    sigma_c: float
    G_c: float
    mu: float
    dt: float


@dataclasses.dataclass
class Problem:
    """One fracture instance.

    dim, order       : spatial dimension (2 or 3) and polynomial order (1 or 2)
    xyz              : (n_vert, dim) float64 vertex coordinates
    elem             : (n_elem, dim+1) int32 vertex ids of each simplex
    dirichlet_vert   : (n_vert,) uint8, 1 = vertex lies on the clamped boundary
    crack_faces      : (n_crack, dim) int32 sorted vertex ids of interface
                       elements that are not intact
    crack_state      : (n_crack,) uint8 interface state applied at every
                       integration point of the face (1 = cohesive law active,
                       2 = traction-free pre-crack)
    crack_beta       : (n_crack,) uint8 fluid flag of the face
    src_vert         : (n_src,) int64 vertex id of each point injection
    src_q0           : (n_src,) float64 injection rate of each source
    material         : Material
    load_steps       : number of quasi-static load steps of the run
    name             : label
    """
    dim: int
    order: int
    xyz: np.ndarray
    elem: np.ndarray
    dirichlet_vert: np.ndarray
    crack_faces: np.ndarray
    crack_state: np.ndarray
    crack_beta: np.ndarray
    src_vert: np.ndarray
    src_q0: np.ndarray
    material: Material
    load_steps: int
    name: str = ""

    @property
    def n_elem(self) -> int:
        return int(self.elem.shape[0])

    @property
    def nodes_per_elem(self) -> int:
        d, k = self.dim, self.order
        return (d + 1) if k == 1 else (d + 1) * (d + 2) // 2

    @property
    def n_udof(self) -> int:
        return self.n_elem * self.nodes_per_elem * self.dim


# ---------------------------------------------------------------------------
# Structured meshes with seeded jitter
# ---------------------------------------------------------------------------

def _jitter(grid: np.ndarray, n: int, seed: int, keep_axis: Optional[int],
            keep_index: Optional[int], amp: float = 0.05) -> np.ndarray:
    """grid: (n_vert, d) integer lattice coordinates in [0, n].

    Each coordinate moves by U(-amp*h, amp*h) except coordinates on an outer
    boundary plane and, if given, the plane-normal coordinate of vertices on
    the crack plane ``grid[:, keep_axis] == keep_index``.
    """
    nv, d = grid.shape
    h = 1.0 / n
    u = uniform(seed, STREAM_JITTER, nv * d).reshape(nv, d)
    delta = (2.0 * u - 1.0) * amp * h
    fixed = (grid == 0) | (grid == n)
    if keep_axis is not None:
        fixed[:, keep_axis] |= grid[:, keep_axis] == keep_index
    delta[fixed] = 0.0
    return grid.astype(np.float64) * h + delta


def grid2d(n: int, seed: int, keep_row: Optional[int] = None):
    """Unit square, n x n quads, each split into two triangles.

    Quad (i, j) is split along (i,j)-(i+1,j+1) when i+j is even, else along
    (i+1,j)-(i,j+1).  Vertex id = j*(n+1) + i.  Returns (xyz, elem, grid).
    """
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    grid = np.stack([ii.ravel(), jj.ravel()], axis=1)
    vid = lambda i, j: j * (n + 1) + i
    tris = []
    for j in range(n):
        for i in range(n):
            v00, v10, v01, v11 = vid(i, j), vid(i + 1, j), vid(i, j + 1), vid(i + 1, j + 1)
            if (i + j) % 2 == 0:
                tris.append((v00, v10, v11))
                tris.append((v00, v11, v01))
            else:
                tris.append((v00, v10, v01))
                tris.append((v10, v11, v01))
    elem = np.asarray(tris, dtype=np.int32)
    xyz = _jitter(grid, n, seed, 1 if keep_row is not None else None, keep_row)
    return xyz, elem, grid


_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn3d(n: int, seed: int, keep_layer: Optional[int] = None):
    """Unit cube, n^3 cubes, each split into the 6 Kuhn tetrahedra along the
    (0,0,0)-(1,1,1) diagonal (same orientation everywhere, so conforming).

    Vertex id = (k*(n+1) + j)*(n+1) + i.  Returns (xyz, elem, grid).
    """
    r = np.arange(n + 1)
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    grid = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    # cell origin lattice
    c = np.arange(n)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    org = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)  # (n^3, 3)
    vid = lambda p: (p[:, 2] * (n + 1) + p[:, 1]) * (n + 1) + p[:, 0]
    tets = []
    for perm in _KUHN_PERMS:
        p0 = org.copy()
        p1 = p0.copy(); p1[:, perm[0]] += 1
        p2 = p1.copy(); p2[:, perm[1]] += 1
        p3 = org + 1
        tets.append(np.stack([vid(p0), vid(p1), vid(p2), vid(p3)], axis=1))
    # element order: cell-major, then the 6 permutations
    elem = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    xyz = _jitter(grid, n, seed, 2 if keep_layer is not None else None, keep_layer)
    return xyz, elem, grid


def boundary_vertices(grid: np.ndarray, n: int) -> np.ndarray:
    return np.any((grid == 0) | (grid == n), axis=1).astype(np.uint8)


def interior_faces(elem: np.ndarray):
    """Faces shared by two elements: (sorted vertex ids (nf, d), e_lo, e_hi).

    Topology only, used to place cracks on the generated meshes.
    """
    ne, nv = elem.shape
    d = nv - 1
    allf = []
    owner = []
    for lf in range(nv):
        cols = [c for c in range(nv) if c != lf]
        allf.append(np.sort(elem[:, cols], axis=1))
        owner.append(np.arange(ne))
    allf = np.concatenate(allf)
    owner = np.concatenate(owner)
    order = np.lexsort(allf.T[::-1])
    allf = allf[order]
    owner = owner[order]
    same = np.all(allf[1:] == allf[:-1], axis=1)
    idx = np.nonzero(same)[0]
    faces = allf[idx]
    e_a, e_b = owner[idx], owner[idx + 1]
    return faces.astype(np.int32), np.minimum(e_a, e_b), np.maximum(e_a, e_b)


# ---------------------------------------------------------------------------
# Crack placement
# ---------------------------------------------------------------------------

def _nearest_vertex(xyz: np.ndarray, cand: np.ndarray, point: np.ndarray) -> int:
    cand = np.unique(cand)
    dist = np.linalg.norm(xyz[cand] - point[None, :], axis=1)
    return int(cand[np.argmin(dist)])


def kgd_problem(n: int, order: int, seed: int, material: Material, q0: float,
                half_length: float = 0.05, ring: int = 2, load_steps: int = 10,
                name: str = "") -> Problem:
    """Plane-strain KGD instance: a pre-cracked horizontal segment centred in
    the unit square, on grid row n//2.  Pre-crack edges: the row's edges whose
    unjittered midpoint satisfies |x-0.5| < half_length; the next ``ring``
    edges on each side are cohesive.  All of them carry fluid.  Injection at
    the crack vertex nearest the centre.  The whole outer boundary is clamped.
    """
    jc = n // 2
    xyz, elem, grid = grid2d(n, seed, keep_row=jc)
    vid = lambda i, j: j * (n + 1) + i
    h = 1.0 / n
    faces, states = [], []
    pre = [i for i in range(n) if abs((i + 0.5) * h - 0.5) < half_length]
    if not pre:
        raise ValueError("mesh too coarse for the requested pre-crack")
    lo, hi = min(pre), max(pre)
    for i in range(max(lo - ring, 0), min(hi + ring, n - 1) + 1):
        a, b = sorted((vid(i, jc), vid(i + 1, jc)))
        faces.append((a, b))
        states.append(2 if lo <= i <= hi else 1)
    faces = np.asarray(faces, dtype=np.int32)
    states = np.asarray(states, dtype=np.uint8)
    beta = np.ones_like(states)
    centre = np.array([0.5, jc * h])
    src = _nearest_vertex(xyz, faces.ravel(), centre)
    return Problem(2, order, xyz, elem, boundary_vertices(grid, n), faces, states, beta,
                   np.array([src], dtype=np.int64), np.array([q0]), material, load_steps,
                   name)


def penny_problem(n: int, order: int, seed: int, material: Material, q0: float,
                  radius: float = 0.05, ring_width: Optional[float] = None,
                  load_steps: int = 5, name: str = "") -> Problem:
    """Penny-shaped crack on the mid plane z = (n//2)/n of a Kuhn-meshed unit
    cube.  Plane faces with unjittered centroid radius < ``radius`` about the
    plane centre are pre-cracked; radius in [radius, radius + ring_width) are
    cohesive (default ring width 2h).  All carry fluid.
    """
    kc = n // 2
    xyz, elem, grid = kuhn3d(n, seed, keep_layer=kc)
    h = 1.0 / n
    if ring_width is None:
        ring_width = 2.0 * h
    vid = lambda i, j: (kc * (n + 1) + j) * (n + 1) + i
    faces, states = [], []
    cz = kc * h
    for j in range(n):
        for i in range(n):
            tri1 = ((i, j), (i + 1, j), (i + 1, j + 1))
            tri2 = ((i, j), (i, j + 1), (i + 1, j + 1))
            for tri in (tri1, tri2):
                cx = sum(p[0] for p in tri) / 3.0 * h
                cy = sum(p[1] for p in tri) / 3.0 * h
                r = math.hypot(cx - 0.5, cy - 0.5)
                if r < radius:
                    st = 2
                elif r < radius + ring_width:
                    st = 1
                else:
                    continue
                faces.append(tuple(sorted(vid(a, b) for a, b in tri)))
                states.append(st)
    if not any(s == 2 for s in states):
        raise ValueError("mesh too coarse for the requested pre-crack")
    faces = np.asarray(faces, dtype=np.int32)
    states = np.asarray(states, dtype=np.uint8)
    centre = np.array([0.5, 0.5, cz])
    src = _nearest_vertex(xyz, faces.ravel(), centre)
    return Problem(3, order, xyz, elem, boundary_vertices(grid, n), faces, states,
                   np.ones_like(states), np.array([src], dtype=np.int64), np.array([q0]),
                   material, load_steps, name)


def multicrack_problem(n: int, order: int, seed: int, material: Material, q0: float,
                       n_disks: int = 3, radius: float = 0.05, load_steps: int = 5,
                       name: str = "") -> Problem:
    """Several pre-cracked disks in a Kuhn-meshed unit cube, of random centre
    (U[0.3, 0.7]^3) and random orientation among the three coordinate planes
    the mesh resolves: disk k lies on the grid plane x_a = l h nearest its
    centre, a drawn from {x, y, z}, and the vertices on that plane keep their
    normal coordinate (no jitter across it), so the crack is flat and made of
    whole mesh faces.  Its faces are the faces of that plane whose centroid
    lies within ``radius`` of the disk centre (pre-cracked) or within
    ``radius + 2h`` (cohesive).  One injection per disk at the crack vertex
    nearest its centre.
    """
    h = 1.0 / n
    u = uniform(seed, STREAM_DISK, 5 * n_disks).reshape(n_disks, 5)
    centres = 0.3 + 0.4 * u[:, :3]
    axes = np.minimum((3.0 * u[:, 3]).astype(np.int64), 2)
    levels = np.rint(centres[np.arange(n_disks), axes] * n).astype(np.int64)
    xyz, elem, grid = kuhn3d(n, seed)
    for a, lev in zip(axes, levels):
        xyz[grid[:, a] == lev, a] = lev * h
    faces, _, _ = interior_faces(elem)
    cent_f = xyz[faces].mean(axis=1)
    state = np.zeros(len(faces), dtype=np.uint8)
    srcs = []
    for k in range(n_disks):
        a, lev = int(axes[k]), int(levels[k])
        c = centres[k].copy()
        c[a] = lev * h
        inplane = np.all(grid[faces][:, :, a] == lev, axis=1)
        rel = cent_f - c
        rel[:, a] = 0.0
        rproj = np.linalg.norm(rel, axis=1)
        pre = inplane & (rproj < radius)
        ring = inplane & (rproj >= radius) & (rproj < radius + 2.0 * h)
        state[ring & (state == 0)] = 1
        state[pre] = 2
        if np.any(pre):
            srcs.append(_nearest_vertex(xyz, faces[pre].ravel(), c))
    sel = state > 0
    return Problem(3, order, xyz, elem, boundary_vertices(grid, n), faces[sel],
                   state[sel], np.ones(int(sel.sum()), dtype=np.uint8),
                   np.asarray(srcs, dtype=np.int64), np.full(len(srcs), q0), material,
                   load_steps, name)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def kgd_small(n: int = 8, order: int = 1, seed: int = 11, steps: int = 3) -> Problem:
    """Small 2D KGD instance for tests (pre-crack of about 0.25, ring 1)."""
    mat = Material(E=1.0, nu=0.25, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=1.0)
    return kgd_problem(n, order, seed, mat, 1e-4, half_length=0.15, ring=1,
                       load_steps=steps, name=f"kgd_n{n}_p{order}")


def penny_small(n: int = 4, order: int = 2, seed: int = 12, steps: int = 2) -> Problem:
    """Small 3D penny instance for tests (pre-crack radius about 0.3)."""
    mat = Material(E=1.0, nu=0.2, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=1.0)
    return penny_problem(n, order, seed, mat, 1e-4, radius=0.3, ring_width=0.2,
                         load_steps=steps, name=f"penny_n{n}_p{order}")


def config(idx: int) -> Problem:
    """The five synthetic workloads.

    The time step is not part of the workload descriptions; it is chosen per
    workload so that a load step lies where the coupled Newton iteration
    converges from the uniform-pressure predictor: dt = 1 for the 2D KGD
    instances, dt = 10 for the 3D cracks (at dt = 1 the 3D penny step is so
    viscosity-dominated that the first iterates put all injected fluid on
    the source patch and Newton diverges).

    1: 2D KGD, 32x32 quads -> 2048 P1 triangles, 12,288 DOF, FP64
    2: 3D penny, Kuhn n=20 -> 48,000 P2 tets, 1.44M DOF
    3: 3D penny, Kuhn n=40 -> 384,000 P2 tets, 11.52M DOF, viscosity params
    4: ensemble of 64 2D KGD instances (use ``ensemble()``)
    5: 3D three-disk multi-crack, Kuhn n=32 -> 196,608 P2 tets, 5.90M DOF (disks on
       coordinate planes of the mesh, see ``multicrack_problem``)
    """
    if idx == 1:
        mat = Material(E=1.0, nu=0.25, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=1.0)
        return kgd_problem(32, 1, 1, mat, 1e-4, half_length=0.05, ring=2, load_steps=10,
                           name="kgd2d_p1_2048tri")
    if idx == 2:
        mat = Material(E=1.0, nu=0.2, sigma_c=1e-3, G_c=1e-4, mu=1e-3, dt=10.0)
        return penny_problem(20, 2, 2, mat, 1e-4, radius=0.05, load_steps=5,
                             name="penny3d_p2_48k")
    if idx == 3:
        mat = Material(E=1.0, nu=0.2, sigma_c=1e-3, G_c=1e-6, mu=1e-1, dt=10.0)
        return penny_problem(40, 2, 3, mat, 1e-4, radius=0.05, load_steps=5,
                             name="penny3d_p2_384k")
    if idx == 5:
        mat = Material(E=1.0, nu=0.25, sigma_c=1e-3, G_c=1e-4, mu=1e-2, dt=10.0)
        return multicrack_problem(32, 2, 5, mat, 1e-4, n_disks=3, radius=0.05,
                                  load_steps=5, name="multicrack3d_p2_197k")
    raise ValueError(f"no single-instance workload {idx}")


def ensemble(count: int = 64, seed: int = 4) -> List[Problem]:
    """Batched 2D KGD ensemble: instance i uses seed 1000*seed + i; triangle
    count log-uniform in [1e3, 2e4] (n = round(sqrt(n_tri/2))), order P1/P2 by
    coin flip, E ~ U[0.5, 2], nu ~ U[0.15, 0.35], mu and Q0 log-uniform in
    [1e-4, 1e-1] and [1e-5, 1e-3].  The time step is dt = 1e-4 / Q0, so that
    every instance injects the same volume per load step as the 2D KGD
    workload (Q0 = 1e-4, dt = 1); with dt = 1 the instances with the largest
    Q0 take steps too long for the Newton iteration to converge."""
    out = []
    for i in range(count):
        s = 1000 * seed + i
        u = uniform(s, STREAM_ENSEMBLE, 6)
        n_tri = math.exp(math.log(1e3) + u[0] * (math.log(2e4) - math.log(1e3)))
        n = max(int(round(math.sqrt(n_tri / 2.0))), 10)
        order = 1 if u[1] < 0.5 else 2
        mat = Material(E=0.5 + 1.5 * u[2], nu=0.15 + 0.2 * u[3],
                       sigma_c=1e-3, G_c=1e-4,
                       mu=math.exp(math.log(1e-4) + u[4] * (math.log(1e-1) - math.log(1e-4))),
                       dt=1.0)
        q0 = math.exp(math.log(1e-5) + u[5] * (math.log(1e-3) - math.log(1e-5)))
        mat = dataclasses.replace(mat, dt=1e-4 / q0)
        out.append(kgd_problem(n, order, s, mat, q0, half_length=0.05, ring=2,
                               load_steps=10, name=f"ens{i}_n{n}_p{order}"))
    return out
