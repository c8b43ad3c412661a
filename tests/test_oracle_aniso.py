"""Pins of the oracle's per-axis (anisotropic) block selection and search:
closed forms that tell the axes apart, the cubic special case against the
independently written cubic functions, the NumPy twin, axis-permutation
symmetry, exact recovery of a shift inside a per-axis window and the tie
rule on a flat volume."""

import numpy as np
import pytest

import oracle
from oracle import twin
from paper_2308_10868_amd import synth


def ramp_x(dims, a=3.0):
    nx, ny, nz = dims
    return np.broadcast_to((np.arange(nx) * a).astype(np.float32), (nz, ny, nx)).copy()


def test_variance_of_a_ramp_tells_axes_apart():
    """v = a*x: a block of edge 3 along x holds {0, a, 2a} in every row, so
    its variance is 2a^2/3; a block that is 3 long along y only is flat."""
    vol = ramp_x((9, 8, 7), a=3.0)
    _, var = oracle.select_aniso(vol, (3, 1, 1), (1, 1, 1), 1.0)
    assert np.allclose(var, 2.0 * 9.0 / 3.0, rtol=0, atol=1e-12)
    _, var = oracle.select_aniso(vol, (1, 3, 5), (1, 1, 1), 1.0)
    assert np.all(var == 0.0)
    # a 5 x 1 x 3 block: every row holds five consecutive ramp values
    _, var = oracle.select_aniso(vol, (5, 1, 3), (2, 1, 1), 1.0)
    assert np.allclose(var, 9.0 * np.var(np.arange(5.0)), rtol=0, atol=1e-12)


def test_grid_and_centres_per_axis():
    vol = synth.gen_random(1, (17, 12, 9), "f32").ref
    c, _ = oracle.select_aniso(vol, (5, 3, 7), (4, 3, 1), 1.0)
    gx, gy, gz = (17 - 5) // 4 + 1, (12 - 3) // 3 + 1, (9 - 7) // 1 + 1
    assert len(c) == gx * gy * gz
    assert set(np.unique(c[:, 0])) == {2 + 4 * i for i in range(gx)}
    assert set(np.unique(c[:, 1])) == {1 + 3 * i for i in range(gy)}
    assert set(np.unique(c[:, 2])) == {3 + i for i in range(gz)}


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_cubic_case_equals_cubic_functions(dtype):
    p = synth.gen_random(2, (15, 13, 11), dtype, smooth=1.0)
    for b, s, f in [(3, 2, 0.3), (5, 3, 0.6)]:
        ca, va = oracle.select_aniso(p.ref, (b, b, b), (s, s, s), f)
        ci, vi = oracle.select(p.ref, b, s, f)
        assert np.array_equal(ca, ci) and np.allclose(va, vi, rtol=1e-13, atol=0)
        for w in (1, 2):
            da, na, fa = oracle.match_aniso(p.ref, p.flt, ci, (b, b, b), (w, w, w))
            di, ni, fi = oracle.match(p.ref, p.flt, ci, b, w)
            assert np.array_equal(da, di)
            assert np.allclose(na, ni, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("b,s,w", [((3, 5, 1), (2, 2, 1), (2, 1, 0)),
                                   ((5, 1, 3), (3, 1, 2), (0, 2, 1)),
                                   ((1, 3, 3), (1, 2, 2), (1, 1, 2))])
def test_twin_agrees(dtype, b, s, w):
    p = synth.gen_random(3, (13, 11, 9), dtype, smooth=0.8)
    c, _ = oracle.select_aniso(p.ref, b, s, 0.5)
    assert np.array_equal(c, twin.select_aniso(p.ref, b, s, 0.5))
    edge = np.array([[b[0] // 2, b[1] // 2, b[2] // 2], [12, 10, 8], [0, 5, 4]], np.int32)
    cen = np.concatenate([c, edge])  # a centre on the border and blocks that fall outside
    d, n, f = oracle.match_aniso(p.ref, p.flt, cen, b, w)
    dt, nt, ft = twin.match_aniso(p.ref, p.flt, cen, b, w)
    assert np.array_equal(d, dt)
    assert np.allclose(n, nt, rtol=0, atol=1e-12, equal_nan=True)
    assert np.array_equal(np.isnan(n), np.isnan(nt))


def test_axis_permutation_symmetry():
    """Swapping the x and y axes of the volumes and of every per-axis size
    swaps the selected centres and displacements (generic data: no ties)."""
    p = synth.gen_random(4, (14, 12, 10), "f32", smooth=1.0)
    b, s, w = (5, 3, 3), (2, 3, 2), (2, 1, 1)
    sw = lambda t: (t[1], t[0], t[2])  # noqa: E731
    ref_t = np.ascontiguousarray(p.ref.transpose(0, 2, 1))
    flt_t = np.ascontiguousarray(p.flt.transpose(0, 2, 1))
    c, _ = oracle.select_aniso(p.ref, b, s, 0.4)
    ct, _ = oracle.select_aniso(ref_t, sw(b), sw(s), 0.4)
    assert {tuple(v) for v in c[:, [1, 0, 2]]} == {tuple(v) for v in ct}
    d, n, _ = oracle.match_aniso(p.ref, p.flt, c, b, w)
    dt, nt, _ = oracle.match_aniso(ref_t, flt_t, c[:, [1, 0, 2]], sw(b), sw(w))
    assert np.array_equal(d[:, [1, 0, 2]], dt)
    assert np.allclose(n, nt, rtol=0, atol=1e-12)


def test_shift_inside_window_recovered_exactly():
    ref = synth.gen_random(5, (20, 18, 16), "f32", smooth=1.0).ref
    shift = (2, 1, 0)
    flt = np.roll(ref, (shift[2], shift[1], shift[0]), axis=(0, 1, 2))
    cen = np.array([[8, 8, 8], [10, 7, 6], [9, 9, 9]], np.int32)
    d, n, _ = oracle.match_aniso(ref, flt, cen, (5, 3, 3), (3, 1, 0))
    assert np.all(d == shift) and np.allclose(n, 1.0, atol=1e-12)
    # a z shift cannot be found with a zero half window along z
    flt_z = np.roll(ref, 1, axis=0)
    d, _, _ = oracle.match_aniso(ref, flt_z, cen, (5, 3, 3), (3, 1, 0))
    assert np.all(d[:, 2] == 0)


def test_flat_volume_takes_smallest_shift_index():
    """Every NCC is 0 on a flat moving volume, so the first valid shift in
    shift-index order (dz, then dy, then dx, each from its lowest) wins."""
    ref = synth.gen_random(6, (12, 10, 9), "f32").ref
    flt = np.full_like(ref, 7.0)
    cen = np.array([[5, 5, 4], [1, 2, 1], [10, 7, 7]], np.int32)
    b, w = (3, 5, 3), (2, 1, 3)
    d, n, f = oracle.match_aniso(ref, flt, cen, b, w)
    h = np.array([1, 2, 1])
    dims = np.array([12, 10, 9])
    lo = np.maximum(-np.array(w), h - cen)
    assert np.array_equal(d, lo) and np.all(n == 0.0) and np.all(f == 0.0)
    assert np.all(cen + h <= dims - 1)


def test_ncc_at_agrees_with_the_search():
    """The NCC at the search's displacement is the reported one, every valid
    displacement in the window scores no higher, and leaving the volume
    gives NaN."""
    p = synth.gen_random(8, (14, 12, 11), "f32", smooth=1.0)
    b, w = (5, 3, 3), (2, 1, 2)
    cen = np.array([[6, 5, 5], [2, 1, 1], [9, 8, 7]], np.int32)
    d, n, _ = oracle.match_aniso(p.ref, p.flt, cen, b, w)
    assert np.array_equal(oracle.ncc_aniso_at(p.ref, p.flt, cen, d, b), n)
    for dz in range(-w[2], w[2] + 1):
        for dy in range(-w[1], w[1] + 1):
            for dx in range(-w[0], w[0] + 1):
                v = oracle.ncc_aniso_at(p.ref, p.flt, cen, np.tile([dx, dy, dz], (3, 1)), b)
                ok = ~np.isnan(v)
                assert np.all(v[ok] <= n[ok])
    far = oracle.ncc_aniso_at(p.ref, p.flt, cen, np.tile([0, 0, 9], (3, 1)), b)
    assert np.all(np.isnan(far))


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_ncc_aniso_at_is_the_correlation_of_the_two_blocks(dtype):
    """oracle.ncc_aniso_at against numpy.corrcoef of the two blocks sliced
    out directly (ref block at c - h, flt block displaced by d), NaN where a
    block leaves the volume, on an anisotropic block."""
    p = synth.gen_random(41, (21, 17, 13), dtype, smooth=1.0)
    b = np.array([5, 3, 7])  # x, y, z
    h = (b - 1) // 2
    dims = np.array(p.dims)
    rng = np.random.default_rng(5)
    centers = np.stack([rng.integers(0, dims[a], 120) for a in range(3)], axis=1).astype(np.int32)
    disp = rng.integers(-4, 5, size=(120, 3)).astype(np.int32)
    got = oracle.ncc_aniso_at(p.ref, p.flt, centers, disp, tuple(b))
    inside = 0
    for k in range(120):
        lo_r = centers[k] - h
        lo_f = lo_r + disp[k]
        if np.any(lo_r < 0) or np.any(lo_r + b > dims) or np.any(lo_f < 0) or \
                np.any(lo_f + b > dims):
            assert np.isnan(got[k]), k
            continue
        inside += 1
        t = p.ref[lo_r[2]:lo_r[2] + b[2], lo_r[1]:lo_r[1] + b[1], lo_r[0]:lo_r[0] + b[0]]
        f = p.flt[lo_f[2]:lo_f[2] + b[2], lo_f[1]:lo_f[1] + b[1], lo_f[0]:lo_f[0] + b[0]]
        want = np.corrcoef(t.astype(np.float64).ravel(), f.astype(np.float64).ravel())[0, 1]
        assert abs(got[k] - want) <= 1e-12, (k, got[k], want)
    assert inside >= 20
