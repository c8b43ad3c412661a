"""Biomechanical consumer of the block-matching output (CPU).

The physics-based registration (Section "Physics-Based Non-Rigid
Registration", the FEM update equation) turns the sparse block displacements
D into displacements U of the vertices of a linear-elastic finite-element
mesh by iterating

    F_i = K U_i,    U_{i+1} = (K + H^T S H)^{-1} (H^T S D + F_i),

with K the stiffness matrix, H the interpolation from mesh vertices to the
block centres and S the blocks' confidence.  Each step adds the elastic
force of the current shape back as an external force, so the mechanical
regularisation fades over the iterations while the data term keeps pulling
the mesh to the measured displacements.

This module is the CPU side of that loop (the paper runs the solve on the
CPU too): a box mesh of linear tetrahedra, K, H, S, the iteration and the
dense displacement field on the voxel grid.  Mesh generation from a
segmentation is not part of it: the mesh is a regular grid of cubes, each
split into six tetrahedra that share the cube's main diagonal (the Kuhn
split, conforming across cubes).

Coordinates are voxel units, (x, y, z) order, the same as block centres and
displacements from the search.  Degrees of freedom are node-major:
U[3 * node + axis].
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "Mesh",
    "box_mesh",
    "elasticity_matrix",
    "stiffness",
    "interpolation",
    "confidence_matrix",
    "solve",
    "dense_field",
    "register",
]

# The six tetrahedra of the unit cube: for each order (a0, a1, a2) of the
# axes, the path 000 -> +e_a0 -> +e_a1 -> +e_a2 = 111 through the corners.
_KUHN_ORDERS = list(itertools.permutations(range(3)))


@dataclass
class Mesh:
    nodes: np.ndarray      # float64 [n_nodes, 3], (x, y, z) voxel coordinates
    tets: np.ndarray       # int64 [n_tets, 4] node indices
    shape: tuple           # nodes per axis (nx, ny, nz)
    origin: np.ndarray     # float64 [3]
    spacing: np.ndarray    # float64 [3], node pitch per axis

    @property
    def n_nodes(self) -> int:
        return self.nodes.shape[0]


def box_mesh(dims, spacing) -> Mesh:
    """Regular mesh covering voxel centres 0 .. dims-1 on each axis with cubes
    of about `spacing` voxels (the last cube stretched to end on the border).
    dims = (nx, ny, nz); spacing a number or per-axis triple."""
    dims = np.asarray(dims, dtype=np.int64)
    sp_req = np.broadcast_to(np.asarray(spacing, dtype=np.float64), (3,))
    if np.any(dims < 2) or np.any(sp_req <= 0):
        raise ValueError("box_mesh needs dims >= 2 and spacing > 0")
    cells = np.maximum(1, np.round((dims - 1) / sp_req).astype(np.int64))
    pitch = (dims - 1) / cells
    shape = tuple(int(c) + 1 for c in cells)
    xs = [np.arange(shape[a]) * pitch[a] for a in range(3)]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    nodes = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)

    def nid(i, j, k):
        return (k * shape[1] + j) * shape[0] + i

    ci, cj, ck = np.meshgrid(np.arange(cells[0]), np.arange(cells[1]), np.arange(cells[2]),
                             indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets = []
    for order in _KUHN_ORDERS:
        corner = np.zeros((3, ci.size), dtype=np.int64)
        verts = [nid(ci, cj, ck)]
        for a in order:
            corner[a] += 1
            verts.append(nid(ci + corner[0], cj + corner[1], ck + corner[2]))
        tets.append(np.stack(verts, axis=1))
    tets = np.concatenate(tets, axis=0)
    return Mesh(nodes, tets, shape, np.zeros(3), pitch)


def elasticity_matrix(young: float, poisson: float) -> np.ndarray:
    """Isotropic linear-elastic 6x6 matrix in Voigt order
    (xx, yy, zz, yz, xz, xy) with engineering shear strains."""
    if not (young > 0) or not (-1.0 < poisson < 0.5):
        raise ValueError("need young > 0 and -1 < poisson < 0.5")
    lam = young * poisson / ((1 + poisson) * (1 - 2 * poisson))
    mu = young / (2 * (1 + poisson))
    d = np.zeros((6, 6))
    d[:3, :3] = lam
    d[[0, 1, 2], [0, 1, 2]] += 2 * mu
    d[[3, 4, 5], [3, 4, 5]] = mu
    return d


def _shape_gradients(mesh: Mesh):
    """Per tetrahedron: gradients of the four linear shape functions
    [n_tets, 4, 3] and volumes [n_tets]."""
    x = mesh.nodes[mesh.tets]                       # [t, 4, 3]
    m = np.concatenate([np.ones(x.shape[:2] + (1,)), x], axis=2)   # rows [1, x, y, z]
    det = np.linalg.det(m)
    if np.any(np.abs(det) < 1e-12):
        raise ValueError("degenerate tetrahedron in the mesh")
    coef = np.linalg.inv(m)                         # N_a = coef[:, 0, a] + coef[:, 1:, a] . X
    return np.transpose(coef[:, 1:, :], (0, 2, 1)), np.abs(det) / 6.0


def stiffness(mesh: Mesh, young: float = 1.0, poisson: float = 0.45) -> sp.csr_matrix:
    """Global stiffness K = sum over tetrahedra of V_e B_e^T D B_e (3 dof per
    node, symmetric, six rigid-body modes in its null space)."""
    grads, vol = _shape_gradients(mesh)
    t = grads.shape[0]
    b = np.zeros((t, 6, 12))
    for a in range(4):
        gx, gy, gz = grads[:, a, 0], grads[:, a, 1], grads[:, a, 2]
        c = 3 * a
        b[:, 0, c] = gx
        b[:, 1, c + 1] = gy
        b[:, 2, c + 2] = gz
        b[:, 3, c + 1], b[:, 3, c + 2] = gz, gy     # yz
        b[:, 4, c], b[:, 4, c + 2] = gz, gx         # xz
        b[:, 5, c], b[:, 5, c + 1] = gy, gx         # xy
    d = elasticity_matrix(young, poisson)
    ke = np.einsum("tki,kl,tlj->tij", b, d, b) * vol[:, None, None]
    dof = (3 * mesh.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(t, 12)
    rows = np.repeat(dof, 12, axis=1).ravel()
    cols = np.tile(dof, (1, 12)).ravel()
    n = 3 * mesh.n_nodes
    return sp.coo_matrix((ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()


def _locate(mesh: Mesh, points: np.ndarray):
    """Containing tetrahedron's nodes [m, 4] and barycentric weights [m, 4]
    of each point, from its cube and the order of its local coordinates."""
    p = (np.asarray(points, dtype=np.float64) - mesh.origin) / mesh.spacing
    cells = np.array(mesh.shape) - 1
    if np.any(p < -1e-9) or np.any(p > cells + 1e-9):
        raise ValueError("a point lies outside the mesh")
    cell = np.clip(np.floor(p).astype(np.int64), 0, cells - 1)
    loc = np.clip(p - cell, 0.0, 1.0)
    order = np.argsort(-loc, axis=1, kind="stable")  # axes by falling local coordinate
    s = np.take_along_axis(loc, order, axis=1)
    w = np.stack([1 - s[:, 0], s[:, 0] - s[:, 1], s[:, 1] - s[:, 2], s[:, 2]], axis=1)
    nx, ny = mesh.shape[0], mesh.shape[1]
    corner = cell.copy()
    ids = [(corner[:, 2] * ny + corner[:, 1]) * nx + corner[:, 0]]
    for j in range(3):
        corner[np.arange(len(p)), order[:, j]] += 1
        ids.append((corner[:, 2] * ny + corner[:, 1]) * nx + corner[:, 0])
    return np.stack(ids, axis=1), w


def interpolation(mesh: Mesh, points) -> sp.csr_matrix:
    """H [3m, 3 n_nodes]: displacement at each point as the linear
    interpolation of the displacements of its tetrahedron's nodes."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    m = points.shape[0]
    ids, w = _locate(mesh, points)
    rows = (3 * np.arange(m)[:, None, None] + np.arange(3)[None, None, :])
    rows = np.broadcast_to(rows, (m, 4, 3))
    cols = 3 * ids[:, :, None] + np.arange(3)[None, None, :]
    vals = np.broadcast_to(w[:, :, None], (m, 4, 3))
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())),
                         shape=(3 * m, 3 * mesh.n_nodes)).tocsr()


def confidence_matrix(conf) -> sp.csr_matrix:
    """S [3m, 3m], block diagonal.  conf [m]: S_k = conf_k I (scalar weight);
    conf [m, 6] = (xx, yy, zz, xy, xz, yz): S_k the symmetric 3x3 of those
    entries (the directional confidence)."""
    c = np.asarray(conf, dtype=np.float64)
    m = c.shape[0]
    if c.ndim == 1:
        blocks = c[:, None, None] * np.eye(3)[None]
    elif c.ndim == 2 and c.shape[1] == 6:
        blocks = np.empty((m, 3, 3))
        blocks[:, 0, 0], blocks[:, 1, 1], blocks[:, 2, 2] = c[:, 0], c[:, 1], c[:, 2]
        blocks[:, 0, 1] = blocks[:, 1, 0] = c[:, 3]
        blocks[:, 0, 2] = blocks[:, 2, 0] = c[:, 4]
        blocks[:, 1, 2] = blocks[:, 2, 1] = c[:, 5]
    else:
        raise ValueError("conf must be [m] or [m, 6]")
    return sp.block_diag(list(blocks), format="csr") if m else sp.csr_matrix((0, 0))


def solve(k: sp.spmatrix, h: sp.spmatrix, s: sp.spmatrix, d, iterations: int = 10, u0=None):
    """The FEM update iterated `iterations` times from U_0 (zero by default).
    Returns (U [3 n_nodes], misfit per iteration: sqrt(r^T S r) with
    r = D - H U_i, including U_0's)."""
    d = np.asarray(d, dtype=np.float64).reshape(-1)
    hts = (h.T @ s).tocsr()
    a = (k + hts @ h).tocsc()
    singular = "K + H^T S H is singular: the blocks do not pin the mesh"
    try:
        lu = spla.splu(a)
    except RuntimeError as e:  # exactly singular
        raise ValueError(singular) from e
    piv = np.abs(lu.U.diagonal())
    if piv.min() <= 1e-12 * piv.max():  # a rigid mode left free (pivot at rounding level)
        raise ValueError(singular)
    rhs_data = hts @ d
    u = np.zeros(k.shape[0]) if u0 is None else np.asarray(u0, dtype=np.float64).copy()

    def misfit(u):
        r = d - h @ u
        return float(np.sqrt(max(r @ (s @ r), 0.0)))

    hist = [misfit(u)]
    for _ in range(iterations):
        f = k @ u
        u = lu.solve(rhs_data + f)
        hist.append(misfit(u))
    return u, np.array(hist)


def dense_field(mesh: Mesh, u, dims) -> np.ndarray:
    """Displacement at every voxel centre, float64 [nz, ny, nx, 3] (x, y, z
    components), by the mesh's linear interpolation of the node
    displacements U."""
    nx, ny, nz = (int(v) for v in dims)
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    out = np.empty((nz, ny, nx, 3))
    ys, xs = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    plane = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size)], axis=1).astype(np.float64)
    for z in range(nz):
        plane[:, 2] = z
        ids, w = _locate(mesh, plane)
        out[z] = np.einsum("pa,pac->pc", w, u[ids]).reshape(ny, nx, 3)
    return out


def register(dims, centers, disp, conf, spacing=16.0, young: float = 1.0,
             poisson: float = 0.45, iterations: int = 10):
    """Block displacements -> mesh displacements: builds the box mesh, K, H
    and S (conf [m] or [m, 6]) and iterates the update.  Blocks with zero
    confidence carry no weight.  Returns (mesh, U [n_nodes, 3], misfits)."""
    mesh = box_mesh(dims, spacing)
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    k = stiffness(mesh, young, poisson)
    h = interpolation(mesh, centers)
    s = confidence_matrix(conf)
    u, hist = solve(k, h, s, np.asarray(disp, dtype=np.float64), iterations)
    return mesh, u.reshape(-1, 3), hist
