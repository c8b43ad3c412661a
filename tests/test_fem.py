"""CPU: the biomechanical consumer (linear-elastic FEM update) pinned to what
elasticity and linear interpolation fix: rigid modes, the energy of a
homogeneous strain, the patch test, exact affine interpolation, the
least-squares limit of the iteration, and a shift recovered end to end from
the oracle's block matches."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2308_10868_amd import fem, synth


def rigid_modes(nodes):
    """Three translations and three infinitesimal rotations, [3n, 6]."""
    n = nodes.shape[0]
    out = np.zeros((n, 3, 6))
    for a in range(3):
        out[:, a, a] = 1.0
    x, y, z = nodes[:, 0], nodes[:, 1], nodes[:, 2]
    out[:, 0, 3], out[:, 1, 3] = -y, x      # about z
    out[:, 0, 4], out[:, 2, 4] = z, -x      # about y
    out[:, 1, 5], out[:, 2, 5] = -z, y      # about x
    return out.reshape(3 * n, 6)


def affine_nodes(nodes, a, t):
    return nodes @ a.T + t


@pytest.fixture(scope="module")
def small():
    mesh = fem.box_mesh((13, 10, 8), (4, 3, 3.5))
    return mesh, fem.stiffness(mesh, young=2.0, poisson=0.3)


def test_mesh_is_conforming_and_fills_the_box(small):
    mesh, _ = small
    grads, vol = fem._shape_gradients(mesh)
    assert np.isclose(vol.sum(), 12.0 * 9.0 * 7.0)
    # every interior triangle is shared by exactly two tetrahedra, boundary ones by one
    faces = {}
    for t in mesh.tets:
        for drop in range(4):
            f = tuple(sorted(np.delete(t, drop)))
            faces[f] = faces.get(f, 0) + 1
    assert set(faces.values()) <= {1, 2}
    lo, hi = mesh.nodes.min(0), mesh.nodes.max(0)
    for f, c in faces.items():
        if c == 1:  # a boundary face lies on one of the box's six planes
            p = mesh.nodes[list(f)]
            assert np.any(np.all(np.isclose(p, lo), axis=0) | np.all(np.isclose(p, hi), axis=0))


def test_stiffness_symmetric_with_six_rigid_modes(small):
    mesh, k = small
    assert abs(k - k.T).max() < 1e-12 * abs(k).max()
    r = rigid_modes(mesh.nodes)
    assert np.abs(k @ r).max() < 1e-10 * abs(k).max() * np.abs(mesh.nodes).max()
    ev = np.linalg.eigvalsh(k.toarray())
    scale = ev[-1]
    assert np.all(ev > -1e-10 * scale)
    assert np.sum(ev < 1e-9 * scale) == 6


@pytest.mark.parametrize("which", ["stretch", "shear", "general"])
def test_homogeneous_strain_energy(small, which):
    """0.5 u^T K u for u = A x equals the box volume times the energy density
    lambda/2 tr(eps)^2 + mu eps:eps of the constant strain eps = sym(A)."""
    mesh, k = small
    young, nu = 2.0, 0.3
    lam = young * nu / ((1 + nu) * (1 - 2 * nu))
    mu = young / (2 * (1 + nu))
    a = {"stretch": np.diag([0.01, 0.0, 0.0]),
         "shear": np.array([[0, 0.02, 0], [0, 0, 0], [0, 0, 0]]),
         "general": np.random.default_rng(0).normal(0, 0.01, (3, 3))}[which]
    u = affine_nodes(mesh.nodes, a, np.zeros(3)).reshape(-1)
    eps = 0.5 * (a + a.T)
    density = 0.5 * lam * np.trace(eps) ** 2 + mu * np.sum(eps * eps)
    assert np.isclose(0.5 * u @ (k @ u), density * 12.0 * 9.0 * 7.0, rtol=1e-10)


def test_patch_test_interior_forces_vanish(small):
    mesh, k = small
    a = np.random.default_rng(1).normal(0, 0.05, (3, 3))
    f = (k @ affine_nodes(mesh.nodes, a, np.array([1.0, -2.0, 0.5])).reshape(-1)).reshape(-1, 3)
    lo, hi = mesh.nodes.min(0), mesh.nodes.max(0)
    interior = np.all((mesh.nodes > lo + 1e-9) & (mesh.nodes < hi - 1e-9), axis=1)
    assert interior.sum() > 0
    assert np.abs(f[interior]).max() < 1e-10 * np.abs(f).max()


def test_interpolation_reproduces_affine_fields(small):
    mesh, _ = small
    rng = np.random.default_rng(2)
    pts = rng.uniform(0, 1, (500, 3)) * np.array([12.0, 9.0, 7.0])
    pts[:5] = mesh.nodes[[0, 1, 17, -2, -1]]   # on nodes and on the border
    h = fem.interpolation(mesh, pts)
    a, t = rng.normal(0, 0.1, (3, 3)), rng.normal(0, 1, 3)
    got = (h @ affine_nodes(mesh.nodes, a, t).reshape(-1)).reshape(-1, 3)
    assert np.allclose(got, affine_nodes(pts, a, t), atol=1e-12)
    ids, w = fem._locate(mesh, pts)
    assert np.all(w >= -1e-15) and np.allclose(w.sum(1), 1.0)
    # the containing simplex is an element of the mesh and the weights are its barycentrics
    tets = {tuple(sorted(t)) for t in mesh.tets}
    for i in range(0, 500, 37):
        assert tuple(sorted(ids[i])) in tets
        m = np.vstack([np.ones(4), mesh.nodes[ids[i]].T])
        assert np.allclose(np.linalg.solve(m, np.r_[1.0, pts[i]]), w[i], atol=1e-12)
    with pytest.raises(ValueError):
        fem.interpolation(mesh, [[13.0, 0, 0]])


def test_confidence_matrix_forms():
    s = fem.confidence_matrix(np.array([0.5, 2.0])).toarray()
    assert np.allclose(s, np.diag([0.5] * 3 + [2.0] * 3))
    d = np.array([[1.0, 2.0, 3.0, 0.1, 0.2, 0.3]])
    s = fem.confidence_matrix(d).toarray()
    assert np.allclose(s, [[1.0, 0.1, 0.2], [0.1, 2.0, 0.3], [0.2, 0.3, 3.0]])


def test_rigid_motion_recovered_in_one_step(small):
    mesh, k = small
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 1, (60, 3)) * np.array([12.0, 9.0, 7.0])
    coef = rng.normal(0, 0.02, 6)
    u_true = rigid_modes(mesh.nodes) @ coef
    h = fem.interpolation(mesh, pts)
    d = h @ u_true
    s = fem.confidence_matrix(rng.uniform(0.2, 1.0, 60))
    u, hist = fem.solve(k, h, s, d, iterations=3)
    assert np.allclose(u, u_true, atol=1e-10)
    assert hist[1] < 1e-10


def test_iteration_decreases_misfit_to_least_squares(small):
    """The misfit sqrt(r^T S r) never grows, and the iteration tends to the
    weighted least-squares fit H^T S (D - H U) = 0 (elastic forces cancelled)."""
    mesh, k = small
    rng = np.random.default_rng(4)
    pts = rng.uniform(0, 1, (400, 3)) * np.array([12.0, 9.0, 7.0])
    h = fem.interpolation(mesh, pts)
    d = rng.normal(0, 1, 3 * 400)
    conf = rng.uniform(0.0, 1.0, (400, 6))
    conf[:, 3:] *= 0.1  # keep each 3x3 positive definite
    s = fem.confidence_matrix(conf)
    # softer tissue: the elastic part fades at rate kappa / (kappa + sigma) per step
    u, hist = fem.solve(0.01 * k, h, s, d, iterations=200)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    normal = h.T @ (s @ (d - h @ u))
    assert np.abs(normal).max() < 1e-6 * np.abs(h.T @ (s @ d)).max()


def test_singular_system_is_rejected(small):
    mesh, k = small
    h = fem.interpolation(mesh, np.zeros((1, 3)))
    with pytest.raises(ValueError):
        fem.solve(k, h, fem.confidence_matrix(np.zeros(1)), np.zeros(3), iterations=1)


def test_dense_field_matches_affine_nodes():
    mesh = fem.box_mesh((9, 7, 5), 3)
    a, t = np.array([[0.01, 0.02, 0], [0, -0.01, 0.03], [0.02, 0, 0]]), np.array([1.0, 2.0, 3.0])
    u = affine_nodes(mesh.nodes, a, t)
    field = fem.dense_field(mesh, u, (9, 7, 5))
    z, y, x = np.meshgrid(np.arange(5), np.arange(7), np.arange(9), indexing="ij")
    p = np.stack([x, y, z], axis=-1).astype(np.float64)
    assert np.allclose(field, p @ a.T + t, atol=1e-12)


def shifted_pair(shift, n=32, seed=7):
    """Textured volume and its copy moved by an integer shift (x, y, z)."""
    ref = synth.gen_random(seed, (n, n, n), "f32", smooth=1.0).ref
    flt = np.roll(ref, shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2))
    return ref, flt


@pytest.mark.parametrize("directional", [False, True])
@pytest.mark.parametrize("block", [5, 7])
def test_shift_recovered_from_oracle_matches(directional, block):
    """Blocks masked to where the moved block stays inside the volume all
    match the shift exactly; a translation is a rigid mode, so one update
    carries every mesh node to it (scalar or directional confidence)."""
    shift = (2, -1, 1)
    ref, flt = shifted_pair(shift)
    mask = np.zeros(ref.shape, np.uint8)
    mask[5:27, 5:27, 5:27] = 1
    centers, _ = oracle.select_ex(ref, block, 3, 0.5, mask, 6)
    disp, ncc, conf = oracle.match(ref, flt, centers, block, 3)
    assert np.all(disp == shift)
    c = oracle.structure_confidence(ref, centers, block, conf) if directional else conf
    mesh, u, hist = fem.register((32, 32, 32), centers, disp, c, spacing=8.0, iterations=3)
    assert np.abs(u - np.array(shift, dtype=np.float64)).max() < 1e-9
    field = fem.dense_field(mesh, u, (32, 32, 32))
    assert np.abs(field - np.array(shift, dtype=np.float64)).max() < 1e-9
