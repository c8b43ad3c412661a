"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retype the oracle's own formula: each compares it with a
library routine (numpy.corrcoef, numpy.lexsort), a closed form, an invariant,
a hand-derived worked example (tests/golden/), or the independent NumPy twin.
"""

import json
import os

import numpy as np
import pytest

from paper_2308_10868_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- NCC formula

@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_ncc_equals_corrcoef(oracle_mod, dtype):
    """NCC (Pearson reading of the NCC equation) == numpy.corrcoef on blocks."""
    p = synth.gen_random(11, (13, 12, 11), dtype, smooth=1.0)
    b, w = 5, 2
    h = 2
    rng = np.random.default_rng(3)
    centers = np.stack([rng.integers(h + w, n - h - w, size=6) for n in (13, 12, 11)], 1)
    srf = oracle_mod.ncc_surface(p.ref, p.flt, centers, b, w)
    for k, (cx, cy, cz) in enumerate(centers):
        t = p.ref[cz - h:cz + h + 1, cy - h:cy + h + 1, cx - h:cx + h + 1].astype(np.float64).ravel()
        for dz in range(-w, w + 1):
            for dy in range(-w, w + 1):
                for dx in range(-w, w + 1):
                    f = p.flt[cz + dz - h:cz + dz + h + 1, cy + dy - h:cy + dy + h + 1,
                              cx + dx - h:cx + dx + h + 1].astype(np.float64).ravel()
                    ref_val = np.corrcoef(t, f)[0, 1]
                    assert abs(srf[k, dz + w, dy + w, dx + w] - ref_val) <= 1e-12


def test_self_match_is_exactly_one(oracle_mod):
    p = synth.gen_random(5, (14, 11, 9), "u16", smooth=1.5)
    centers, _ = oracle_mod.select(p.ref, 3, 2, 0.3)
    disp, ncc, conf = oracle_mod.match(p.ref, p.ref, centers, 3, 2)
    assert np.all(ncc == 1.0)
    assert np.all(conf == 1.0)
    assert np.all(disp == 0)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_ncc_bounded(oracle_mod, dtype):
    p = synth.gen_random(7, (12, 10, 9), dtype)
    centers, _ = oracle_mod.select(p.ref, 3, 1, 0.5)
    srf = oracle_mod.ncc_surface(p.ref, p.flt, centers, 3, 2)
    v = srf[~np.isnan(srf)]
    assert v.size > 0 and np.all(np.abs(v) <= 1.0 + 1e-15)


# ------------------------------------------------------------ affine changes

def test_scale_by_power_of_two_is_bit_identical(oracle_mod):
    p = synth.gen_random(21, (12, 11, 10), "f32", smooth=1.0)
    centers, _ = oracle_mod.select(p.ref, 3, 1, 0.4)
    d0, n0, _ = oracle_mod.match(p.ref, p.flt, centers, 3, 2)
    d1, n1, _ = oracle_mod.match(p.ref, (p.flt * np.float32(4.0)).astype(np.float32), centers, 3, 2)
    assert np.array_equal(d0, d1) and np.array_equal(n0, n1)
    # selection is scale-invariant too (exactly, for 2^k)
    c2, _ = oracle_mod.select((p.ref * np.float32(0.5)).astype(np.float32), 3, 1, 0.4)
    assert np.array_equal(centers, c2)


def test_integer_affine_and_negation_u16(oracle_mod):
    p = synth.gen_random(22, (12, 11, 10), "u16", smooth=1.0)
    small = (p.flt // 3).astype(np.uint16)  # <= 1365
    centers, _ = oracle_mod.select(p.ref, 3, 1, 0.4)
    s0 = oracle_mod.ncc_surface(p.ref, small, centers, 3, 2)
    s1 = oracle_mod.ncc_surface(p.ref, (3 * small.astype(np.int64) + 5).astype(np.uint16), centers, 3, 2)
    s2 = oracle_mod.ncc_surface(p.ref, (4095 - small.astype(np.int64)).astype(np.uint16), centers, 3, 2)
    m = ~np.isnan(s0)
    assert np.max(np.abs(s0[m] - s1[m])) <= 1e-12
    assert np.max(np.abs(s0[m] + s2[m])) <= 1e-12


# ------------------------------------------------- known integer translation

def test_translation_recovered():
    """64^3 blob volumes, flt = ref translated by (3,-2,1) + fresh N(0, 0.02^2)
    noise.  With smooth blobs the NCC peak is flat relative to the noise, so
    exact recovery is not guaranteed per block: most reachable blocks return
    (3,-2,1) exactly and none is off by more than two voxels per axis.  (The
    exact pin is the noise-free test below.)"""
    import oracle

    p = synth.gen_translation_f32(seed=0)
    centers, _ = oracle.select(p.ref, 7, 7, 0.2)
    assert len(centers) == 146
    disp, ncc, _ = oracle.match(p.ref, p.flt, centers, 7, 5)
    s = np.array([3, -2, 1])
    h = 3
    reach = np.all((centers + s - h >= 0) & (centers + s + h <= 63), axis=1)
    assert reach.sum() == 113
    exact = np.all(disp[reach] == s, axis=1)
    assert exact.mean() > 0.7
    assert np.max(np.abs(disp[reach] - s)) <= 2
    assert np.all(ncc[reach] > 0.9)


def test_translation_noise_free_ncc_one_and_role_swap(oracle_mod):
    p = synth.gen_translation_f32(seed=4, n=40, n_blobs=12, shift=(2, 1, -3), noise=0.0)
    centers, _ = oracle_mod.select(p.ref, 5, 5, 0.5)
    s = np.array([2, 1, -3])
    h = 2
    reach = np.all((centers + s - h >= 0) & (centers + s + h <= 39), axis=1)
    disp, ncc, _ = oracle_mod.match(p.ref, p.flt, centers[reach], 5, 4)
    assert np.all(disp == s)
    assert np.max(np.abs(ncc - 1.0)) <= 1e-12
    # role swap: blocks of flt searched in ref move by -s
    c2 = centers[reach] + s
    d2, n2, _ = oracle_mod.match(p.flt, p.ref, c2, 5, 4)
    assert np.all(d2 == -s)


def test_translation_nonsquare_axes(oracle_mod):
    """A non-cubic volume with distinct shifts per axis catches any swap of
    the (x, y, z) conventions."""
    from paper_2308_10868_amd.synth import _blob_field

    rng = np.random.default_rng(9)
    shape = (18, 23, 29)  # nz, ny, nx
    cen = rng.uniform(0, 1, (25, 3)) * np.array([29, 23, 18])
    sig = rng.uniform(2, 4, 25)
    amp = rng.uniform(0.2, 1, 25)
    s = (3, -1, 2)
    ref = _blob_field(shape, cen, sig, amp).astype(np.float32)
    flt = _blob_field(shape, cen, sig, amp, offset=s).astype(np.float32)
    centers, _ = oracle_mod.select(ref, 5, 3, 0.5)
    h = 2
    dims = np.array([29, 23, 18])
    reach = np.all((centers + np.array(s) - h >= 0) & (centers + np.array(s) + h <= dims - 1), axis=1)
    disp, ncc, _ = oracle_mod.match(ref, flt, centers[reach], 5, 3)
    assert np.all(disp == np.array(s)) and np.all(ncc > 1 - 1e-9)


# ---------------------------------------------------------------- tie-breaks

def test_periodic_tie_takes_lowest_shift_index(oracle_mod):
    rng = np.random.default_rng(5)
    period = 3
    base = rng.integers(0, 4096, size=(10, 11, period))
    vol = np.tile(base, (1, 1, 6))[:, :, :17].astype(np.uint16)  # nz=10, ny=11, nx=17
    b, w, h = 3, 4, 1
    centers = np.array([[8, 5, 5], [3, 4, 4], [13, 6, 5]], dtype=np.int32)
    disp, ncc, _ = oracle_mod.match(vol, vol, centers, b, w)
    for (cx, cy, cz), d in zip(centers, disp):
        lx = max(-w, h - cx)
        # data repeat every `period` voxels along x: every dx = 0 mod 3 is a
        # perfect match, the smallest valid one wins (dy = dz = 0 only)
        cands = [dx for dx in range(lx, w + 1) if dx % period == 0 and cx + dx + h <= 16]
        assert d[0] == min(cands) and d[1] == 0 and d[2] == 0
    assert np.all(ncc == 1.0)


def test_flat_window_gives_zero_and_lowest_valid_shift(oracle_mod):
    p = synth.gen_random(2, (12, 12, 12), "u16")
    flt = np.full_like(p.flt, 1234)
    centers = np.array([[5, 6, 4], [2, 2, 2], [9, 9, 9]], dtype=np.int32)
    disp, ncc, conf = oracle_mod.match(p.ref, flt, centers, 3, 3)
    for c, d in zip(centers, disp):
        lo = [max(-3, 1 - int(v)) for v in c]
        assert list(d) == lo
    assert np.all(ncc == 0.0) and np.all(conf == 0.0)


def test_golden_triangle_wave(oracle_mod):
    g = _load_golden("triangle_wave.json")
    nx, ny, nz = g["dims"]
    row = np.array(g["g"], dtype=np.uint16)
    vol = np.broadcast_to(row[None, None, :], (nz, ny, nx)).copy()
    c = np.array([g["center"]], dtype=np.int32)
    b, w = g["block"], g["window"]
    srf = oracle_mod.ncc_surface(vol, vol, c, b, w)[0]
    for dx, val in g["ncc_by_dx"].items():
        col = srf[:, :, int(dx) + w]
        valid = col[~np.isnan(col)]
        assert valid.size == 9  # dy, dz in -1..1
        assert np.max(np.abs(valid - val)) <= 1e-12
    for dx in (-4, -3):
        assert np.all(np.isnan(srf[:, :, dx + w]))
    disp, ncc, conf = oracle_mod.match(vol, vol, c, b, w)
    assert list(disp[0]) == g["argmax"]["disp"] and abs(ncc[0] - g["argmax"]["ncc"]) <= 1e-12


def test_golden_short_row(oracle_mod):
    g = _load_golden("short_row.json")
    nx, ny, nz = g["dims"]
    row = np.array(g["g"], dtype=np.uint16)
    vol = np.broadcast_to(row[None, None, :], (nz, ny, nx)).copy()
    c = np.array([g["center"]], dtype=np.int32)
    b, w = g["block"], g["window"]
    srf = oracle_mod.ncc_surface(vol, vol, c, b, w)[0]
    for dx, val in g["ncc_by_dx"].items():
        assert abs(srf[w, w, int(dx) + w] - val) <= 1e-12
    assert np.sum(~np.isnan(srf)) == len(g["ncc_by_dx"])
    disp, ncc, _ = oracle_mod.match(vol, vol, c, b, w)
    assert list(disp[0]) == g["argmax"]["disp"] and ncc[0] == g["argmax"]["ncc"]


# ---------------------------------------------------------------- selection

def test_selection_counts_closed_form(oracle_mod):
    g = _load_golden("selection_counts.json")
    for case in g["cases"]:
        grid = oracle_mod.grid_shape(case["dims"], case["block"], case["stride"])
        assert list(grid) == case["grid"]
        n = int(np.prod(grid))
        assert n == case["n"]
        assert oracle_mod.select_count(n, case["fraction"]) == case["k"]


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("dims,b,stride,frac", [((10, 9, 8), 3, 1, 0.3), ((13, 7, 11), 5, 2, 0.5),
                                                 ((12, 12, 12), 3, 3, 1.0), ((9, 9, 9), 5, 1, 0.07)])
def test_selection_vs_lexsort(oracle_mod, dtype, dims, b, stride, frac):
    from oracle import twin

    p = synth.gen_random(31, dims, dtype, smooth=0.8)
    got, _ = oracle_mod.select(p.ref, b, stride, frac)
    exp = twin.select(p.ref, b, stride, frac)
    assert np.array_equal(got, exp)


def test_selection_ties_lower_index_first(oracle_mod):
    vol = np.zeros((9, 9, 9), dtype=np.uint16)  # every block flat: all keys equal
    got, _ = oracle_mod.select(vol, 3, 3, 0.5)  # 27 blocks, K = 14
    assert len(got) == 14
    gx, gy, gz = (got[:, 0] - 1) // 3, (got[:, 1] - 1) // 3, (got[:, 2] - 1) // 3
    assert np.array_equal((gz * 3 + gy) * 3 + gx, np.arange(14))


# ------------------------------------------------------ oracle vs NumPy twin

@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("dims,b,w,stride", [((10, 9, 8), 3, 1, 1), ((13, 7, 11), 3, 3, 2),
                                              ((13, 12, 11), 5, 2, 2), ((11, 14, 9), 5, 3, 3)])
def test_oracle_vs_twin(oracle_mod, dtype, dims, b, w, stride):
    from oracle import twin

    p = synth.gen_random(41, dims, dtype, smooth=0.7)
    centers, _ = oracle_mod.select(p.ref, b, stride, 0.6)
    d0, n0, c0 = oracle_mod.match(p.ref, p.flt, centers, b, w)
    d1, n1, c1 = twin.match(p.ref, p.flt, centers, b, w)
    srf = oracle_mod.ncc_surface(p.ref, p.flt, centers, b, w)
    for k in range(len(centers)):
        t = twin.surface(p.ref, p.flt, centers[k], b, w)
        m = ~np.isnan(t)
        assert np.array_equal(m, ~np.isnan(srf[k]))
        assert np.max(np.abs(t[m] - srf[k][m])) <= 1e-12
    assert np.max(np.abs(n0 - n1)) <= 1e-12
    # displacements agree except where the twin's own surface has a near-tie
    for k in range(len(centers)):
        if not np.array_equal(d0[k], d1[k]):
            t = twin.surface(p.ref, p.flt, centers[k], b, w)
            dd = d0[k] + w
            assert abs(t[dd[2], dd[1], dd[0]] - n1[k]) <= 1e-12


def test_out_of_volume_centre(oracle_mod):
    p = synth.gen_random(1, (10, 10, 10), "u16")
    c = np.array([[0, 5, 5], [5, 5, 5], [5, 9, 5]], dtype=np.int32)
    disp, ncc, conf = oracle_mod.match(p.ref, p.flt, c, 3, 2)
    assert np.isnan(ncc[0]) and np.isnan(ncc[2]) and not np.isnan(ncc[1])
    assert conf[0] == 0 and conf[2] == 0 and np.all(disp[[0, 2]] == 0)


def test_valid_shift_counts(oracle_mod):
    dims = (64, 64, 64)
    c = np.array([[3, 3, 3], [31, 31, 31], [59, 10, 60]], dtype=np.int32)
    v = oracle_mod.valid_shifts(dims, c, 7, 5)
    # per axis: centre 3 -> dx in [0, 5] (6); 31 -> 11; 59/60 -> [-5, 1] / [-5, 0]
    assert list(v) == [6 ** 3, 11 ** 3, 7 * 11 * 6]
