"""Seeded synthetic inputs for the exponential-propagator hot path.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no arithmetic of the method itself: only structured hex8 meshes (node
coordinates and connectivity), boundary node / face sets, load time tables,
material constants and initial fields, all drawn from fixed seeds.

The paper's own meshes (unstructured quadratic hexahedra generated with a
commercial mesher) and most of its material constants are not published, so
the workloads below are synthetic stand-ins with the shapes of its benchmark
families (Sec. 6: cantilever beam, soft-tissue block, rubber blocks).

Conventions
-----------
* node id of lattice point (i, j, k) = i + (nx+1) * (j + (ny+1) * k)
* element id of cell (i, j, k)       = i + nx * (j + ny * k)
* hex8 local node order (VTK): (0,0,0) (1,0,0) (1,1,0) (0,1,0) then the same
  four at the upper z level.
* DOF id = 3 * node + component; all nodal vectors are node-major (x, y, z).
* a quad face lists its 4 nodes counter-clockwise seen from outside, so the
  right-hand rule gives the outward normal.
* hex27 (quadratic, Q2) elements: local node a = i + 3 j + 9 k, (i, j, k) in {0,1,2}^3 at
  local coordinates (i-1, j-1, k-1); a box of nx x ny x nz Q2 elements has the node
  lattice of the 2nx x 2ny x 2nz hex8 box.  A loaded Q2 face lists its 9 nodes p + 3 q,
  (p, q) in {0,1,2}^2 along its two in-plane axes, ordered so that the derivatives of the
  face map along p then q give the outward normal.
* material models and their parameter tuples:
    'linear' : (E [Pa], nu)
    'nh'     : (mu [Pa], lambda [Pa])            compressible Neo-Hookean
    'yeoh'   : (C10, C20, C30 [Pa], D1 [1/Pa])   decoupled Yeoh; C20=C30=0 is
               the decoupled Neo-Hookean solid (mu = 2 C10, kappa = 2 / D1)
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

__all__ = [
    "Problem", "box_mesh", "box_face_quads", "box_face_nodes", "config",
    "batch_instances", "distort", "MODELS", "q2_of", "box_mesh_q2", "box_face_quads_q2",
]

MODELS = {"linear": 0, "nh": 1, "yeoh": 2}


@dataclass
class Problem:
    """One elastodynamics instance: mesh, material, boundary data, loads, IC."""
    name: str
    xyz: np.ndarray            # (n_nodes, 3) float64 reference coordinates [m]
    conn: np.ndarray           # (n_elems, 8) int32 hex8 connectivity (VTK order)
    model: str                 # 'linear' | 'nh' | 'yeoh'
    params: tuple              # see module docstring
    rho: float                 # reference density [kg/m^3]
    clamped: np.ndarray        # (n_c,) int32 DOF ids held at u = v = 0
    faces: np.ndarray          # (n_f, 4) int32 loaded quad faces
    t0: np.ndarray             # (3,) nominal (dead) traction vector [Pa]
    knots_t: np.ndarray        # load time table: times (ascending)
    knots_s: np.ndarray        # load time table: scale(t), piecewise linear,
                               # held constant before the first / after the last knot
    u0: np.ndarray             # (3 n_nodes,) initial displacement [m]
    v0: np.ndarray             # (3 n_nodes,) initial velocity [m/s]
    dt: float                  # time-step [s]
    n_steps: int
    tol: float = 1e-10         # Krylov tolerance (relative to the propagated norm)
    grid: Optional[tuple] = None   # (nx, ny, nz) when the mesh is a lattice box
    extra: dict = field(default_factory=dict)
    elem: str = "hex8"         # 'hex8' (trilinear) or 'hex27' (quadratic Lagrange, Q2)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_free(self) -> int:
        return 3 * self.n_nodes - int(np.unique(self.clamped).size)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


# ----------------------------------------------------------------------------
# structured box meshes
# ----------------------------------------------------------------------------
def box_mesh(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float):
    """Lattice box [0,lx]x[0,ly]x[0,lz] split into nx*ny*nz hex8 cells."""
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    conn = np.stack([
        nid(i, j, k), nid(i + 1, j, k), nid(i + 1, j + 1, k), nid(i, j + 1, k),
        nid(i, j, k + 1), nid(i + 1, j, k + 1), nid(i + 1, j + 1, k + 1), nid(i, j + 1, k + 1),
    ], axis=1).astype(np.int32)
    return xyz, conn


def box_face_nodes(nx: int, ny: int, nz: int, axis: int, side: int) -> np.ndarray:
    """Node ids on the lattice face axis in {0,1,2}, side in {0 (min), 1 (max)}."""
    dims = (nx, ny, nz)
    idx = [np.arange(d + 1) for d in dims]
    idx[axis] = np.array([0 if side == 0 else dims[axis]])
    K, J, I = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
    return (I + (nx + 1) * (J + (ny + 1) * K)).ravel().astype(np.int32)


def box_face_quads(nx: int, ny: int, nz: int, axis: int, side: int) -> np.ndarray:
    """Quad faces of the lattice boundary face, outward normal by right-hand rule."""
    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    dims = (nx, ny, nz)
    a, b = [d for d in range(3) if d != axis]          # in-plane axes, a < b
    fixed = 0 if side == 0 else dims[axis]
    quads = []
    for q in range(dims[b]):
        for p in range(dims[a]):
            corners = []
            for (dp, dq) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                ijk = [0, 0, 0]
                ijk[axis] = fixed
                ijk[a] = p + dp
                ijk[b] = q + dq
                corners.append(nid(*ijk))
            # (a, b, axis) is a cyclic permutation of (0,1,2) except for axis == 1
            outward_is_ab = (axis != 1) == (side == 1)
            quads.append(corners if outward_is_ab else corners[::-1])
    return np.asarray(quads, dtype=np.int32)


def box_mesh_q2(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float):
    """Lattice box split into nx*ny*nz quadratic (27-node) hexahedra; the nodes are the
    lattice of the 2nx x 2ny x 2nz hex8 box, node (I, J, K) = I + (2nx+1)(J + (2ny+1)K)."""
    xyz, _ = box_mesh(2 * nx, 2 * ny, 2 * nz, lx, ly, lz)
    NX, NY = 2 * nx + 1, 2 * ny + 1
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    cols = []
    for k in range(3):
        for j in range(3):
            for i in range(3):
                cols.append((2 * ex + i) + NX * ((2 * ey + j) + NY * (2 * ez + k)))
    return xyz, np.stack(cols, axis=1).astype(np.int32)


def box_face_quads_q2(nx: int, ny: int, nz: int, axis: int, side: int) -> np.ndarray:
    """9-node faces of a Q2 box's boundary face axis / side (outward orientation)."""
    NX, NY = 2 * nx + 1, 2 * ny + 1

    def nid(I, J, K):
        return I + NX * (J + NY * K)

    dims = (nx, ny, nz)
    a, b = [d for d in range(3) if d != axis]
    fixed = 0 if side == 0 else 2 * dims[axis]
    outward_is_ab = (axis != 1) == (side == 1)
    faces = []
    for q in range(dims[b]):
        for p in range(dims[a]):
            nodes = []
            for qq in range(3):
                for pp in range(3):
                    ijk = [0, 0, 0]
                    ijk[axis] = fixed
                    # swapping the in-plane roles flips the face's orientation
                    if outward_is_ab:
                        ijk[a], ijk[b] = 2 * p + pp, 2 * q + qq
                    else:
                        ijk[a], ijk[b] = 2 * p + qq, 2 * q + pp
                    nodes.append(nid(*ijk))
            faces.append(nodes)
    return np.asarray(faces, dtype=np.int32)


def q2_of(prob: Problem) -> Problem:
    """The same box, loads, supports and initial fields on quadratic (Q2) elements: a lattice
    box of nx x ny x nz hex8 cells (nx, ny, nz even) has the nodes of the nx/2 x ny/2 x nz/2
    Q2 box, so nodal data carry over; the loaded faces become 9-node faces."""
    nx, ny, nz = prob.grid
    if nx % 2 or ny % 2 or nz % 2:
        raise ValueError("Q2 box needs even hex8 cell counts")
    lx, ly, lz = (prob.xyz.max(axis=0) - prob.xyz.min(axis=0))
    xyz, conn = box_mesh_q2(nx // 2, ny // 2, nz // 2, lx, ly, lz)
    xyz = xyz + prob.xyz.min(axis=0)
    assert np.allclose(xyz, prob.xyz)
    # loaded faces: find which box face the hex8 quads lie on
    faces = np.zeros((0, 9), np.int32)
    if len(prob.faces):
        c = prob.xyz[np.asarray(prob.faces)].reshape(-1, 3)
        span = c.max(axis=0) - c.min(axis=0)
        axis = int(np.argmin(span))
        side = int(abs(c[0, axis] - prob.xyz[:, axis].max()) < 1e-12 * max(1.0, abs(c[0, axis])))
        faces = box_face_quads_q2(nx // 2, ny // 2, nz // 2, axis, side)
    return replace(prob, name=prob.name + "-q2", conn=conn, faces=faces, elem="hex27",
                   grid=(nx // 2, ny // 2, nz // 2))


def _dofs_of_nodes(nodes: np.ndarray, comps=(0, 1, 2)) -> np.ndarray:
    nodes = np.asarray(nodes, dtype=np.int64)
    return np.sort(np.concatenate([3 * nodes + c for c in comps])).astype(np.int32)


def distort(prob: Problem, amplitude: float, seed: int = 7) -> Problem:
    """Move interior nodes randomly by up to amplitude * (smallest cell edge).

    Gives non-affine (general trilinear) hexahedra for geometry-general tests.
    """
    if prob.grid is None:
        raise ValueError("distort() needs a lattice box problem")
    nx, ny, nz = prob.grid
    rng = np.random.default_rng(seed)
    xyz = prob.xyz.copy()
    lo, hi = xyz.min(0), xyz.max(0)
    h = ((hi - lo) / np.array([nx, ny, nz])).min()
    interior = np.all((xyz > lo + 1e-12) & (xyz < hi - 1e-12), axis=1)
    xyz[interior] += amplitude * h * rng.uniform(-1.0, 1.0, size=(int(interior.sum()), 3))
    return prob.with_(xyz=xyz, name=prob.name + "-distorted")


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
_STEEL = ("linear", (200e9, 0.3), 7800.0)


def _cantilever(name, nx, ny, nz, lx, ly, lz, model, params, rho, traction_z,
                knots_t, knots_s, dt, n_steps, tol=1e-10, v_sigma=0.0, v_seed=0):
    xyz, conn = box_mesh(nx, ny, nz, lx, ly, lz)
    clamped = _dofs_of_nodes(box_face_nodes(nx, ny, nz, 0, 0))
    faces = box_face_quads(nx, ny, nz, 0, 1)
    n = xyz.shape[0]
    u0 = np.zeros(3 * n)
    v0 = np.zeros(3 * n)
    if v_sigma > 0.0:
        free = np.setdiff1d(np.arange(3 * n), clamped)
        rng = np.random.default_rng(v_seed)
        v0[free] = rng.normal(0.0, v_sigma, size=free.size)
    return Problem(name=name, xyz=xyz, conn=conn, model=model, params=tuple(params), rho=rho,
                   clamped=clamped, faces=faces, t0=np.array([0.0, 0.0, traction_z]),
                   knots_t=np.asarray(knots_t, float), knots_s=np.asarray(knots_s, float),
                   u0=u0, v0=v0, dt=dt, n_steps=n_steps, tol=tol, grid=(nx, ny, nz))


def config(name: str, **over) -> Problem:
    """Named workload.  Keyword overrides: nx, ny, nz, dt, n_steps, tol.

    c1  linear steel cantilever 10x2x2, 1.0x0.2x0.2 m, tip traction 1e5 Pa (-z),
        dt 1e-4, 200 steps
    c2  linear steel cantilever 80x8x8, same box and load, initial velocity
        N(0, (1e-3 m/s)^2) per free DOF (seed 0), dt 1e-4 (sweep 1e-5..1e-3)
    c3  compressible Neo-Hookean cantilever 160x16x16 (mu 0.4 MPa, lambda 2 MPa,
        rho 1100), tip traction ramped 0 -> 2e4 Pa over [0, 0.025] s then held,
        dt 1e-4 (also 5e-4), to 0.05 s
    c4  nearly incompressible decoupled Neo-Hookean unit cube 64^3 (mu 10 kPa,
        kappa 1 MPa, rho 1000), bottom (z = 0) clamped, dead pressure pulse of
        1 kPa x sin(pi t / 0.1) on the top face for t <= 0.1 s, dt 1e-3, 500 steps
    bar 1D-reducible bar nx x 1 x 1 (all y/z DOFs and the x = 0 face clamped),
        linear steel, no load, at rest (tests set the initial field)
    """
    g = lambda k, d: over.get(k, d)
    if name == "c1":
        p = _cantilever("c1", g("nx", 10), g("ny", 2), g("nz", 2), 1.0, 0.2, 0.2,
                        *_STEEL, -1e5, [0.0], [1.0], g("dt", 1e-4), g("n_steps", 200))
    elif name == "c2":
        p = _cantilever("c2", g("nx", 80), g("ny", 8), g("nz", 8), 1.0, 0.2, 0.2,
                        *_STEEL, -1e5, [0.0], [1.0], g("dt", 1e-4), g("n_steps", 500),
                        v_sigma=1e-3, v_seed=0)
    elif name == "c3":
        p = _cantilever("c3", g("nx", 160), g("ny", 16), g("nz", 16), 1.0, 0.2, 0.2,
                        "nh", (0.4e6, 2.0e6), 1100.0, -2e4, [0.0, 0.025], [0.0, 1.0],
                        g("dt", 1e-4), g("n_steps", 500))
    elif name == "c4":
        nx, ny, nz = g("nx", 64), g("ny", 64), g("nz", 64)
        xyz, conn = box_mesh(nx, ny, nz, 1.0, 1.0, 1.0)
        clamped = _dofs_of_nodes(box_face_nodes(nx, ny, nz, 2, 0))
        faces = box_face_quads(nx, ny, nz, 2, 1)
        kt = np.linspace(0.0, 0.1, 201)
        ks = np.sin(np.pi * kt / 0.1)
        ks[-1] = 0.0
        n = xyz.shape[0]
        p = Problem(name="c4", xyz=xyz, conn=conn, model="yeoh",
                    params=(5.0e3, 0.0, 0.0, 2.0e-6), rho=1000.0, clamped=clamped,
                    faces=faces, t0=np.array([0.0, 0.0, -1.0e3]), knots_t=kt, knots_s=ks,
                    u0=np.zeros(3 * n), v0=np.zeros(3 * n), dt=g("dt", 1e-3),
                    n_steps=g("n_steps", 500), tol=1e-10, grid=(nx, ny, nz))
    elif name == "bar":
        nx = g("nx", 16)
        h = g("h", 0.0625)
        xyz, conn = box_mesh(nx, 1, 1, nx * h, h, h)
        n = xyz.shape[0]
        x0 = box_face_nodes(nx, 1, 1, 0, 0)
        clamped = np.unique(np.concatenate([
            _dofs_of_nodes(np.arange(n), comps=(1, 2)), _dofs_of_nodes(x0)])).astype(np.int32)
        p = Problem(name="bar", xyz=xyz, conn=conn, model="linear", params=(200e9, 0.3),
                    rho=7800.0, clamped=clamped, faces=np.zeros((0, 4), np.int32),
                    t0=np.zeros(3), knots_t=np.array([0.0]), knots_s=np.array([0.0]),
                    u0=np.zeros(3 * n), v0=np.zeros(3 * n), dt=g("dt", 1e-5),
                    n_steps=g("n_steps", 10), tol=1e-12, grid=(nx, 1, 1))
    else:
        raise KeyError(name)
    if "tol" in over:
        p = p.with_(tol=over["tol"])
    return p


def batch_instances(n_inst: int = 256, seed: int = 5, dt: float = 6.25e-6,
                    n_steps: int = 1000, nx_range=(20, 60), nyz_range=(4, 8),
                    h: float = 0.01) -> list:
    """c5: independent rubber blocks of uneven size.

    nx ~ U{20..60}, ny = nz ~ U{4..8} (drawn jointly), cubic cells of edge h;
    compressible Neo-Hookean with mu ~ U[0.2, 1] MPa, lambda = 5 mu, rho 1100;
    x = 0 clamped, constant tip traction (-z) ~ U[1e3, 1e4] Pa, at rest.  dt = 6.25e-6 s (1e-4
    halved four times) keeps the relative energy error of every instance below 1e-6 over the
    1000 steps (with the augmented entry at each block's scale; 1.25e-5 s reaches 1.4e-6).
    """
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n_inst):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nyz = int(rng.integers(nyz_range[0], nyz_range[1] + 1))
        mu = float(rng.uniform(0.2e6, 1.0e6))
        tz = float(rng.uniform(1e3, 1e4))
        p = _cantilever(f"c5[{q}]", nx, nyz, nyz, nx * h, nyz * h, nyz * h, "nh",
                        (mu, 5.0 * mu), 1100.0, -tz, [0.0], [1.0], dt, n_steps)
        out.append(p)
    return out
