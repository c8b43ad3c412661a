"""Pins of the oracle's selection variants (connectivity pattern, candidate
mask): hand-derived cases, an independent NumPy twin, and the properties that
define a greedy rank-order selection under a separation rule."""

import json
import os

import numpy as np
import pytest

import oracle
from oracle import twin
from paper_2308_10868_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_volume(case):
    nx, ny, nz = case["dims"]
    vol = np.zeros((nz, ny, nx), dtype=np.uint16)
    gx = nx // 3
    for g, a in enumerate(case["a"]):
        x, y = g % gx, g // gx
        vol[1, 3 * y + 1, 3 * x + 1] = a
    mask = None
    if case["mask_blocks"] is not None:
        mask = np.zeros_like(vol, dtype=np.uint8)
        for g in case["mask_blocks"]:
            x, y = g % gx, g // gx
            mask[1, 3 * y + 1, 3 * x + 1] = 1
    return vol, mask


@pytest.mark.parametrize("i", range(7))
def test_golden_cases(i):
    case = json.load(open(os.path.join(HERE, "golden", "select_connectivity.json")))["cases"][i]
    vol, mask = golden_volume(case)
    got, _ = oracle.select_ex(vol, 3, 3, case["fraction"], mask, case["connectivity"])
    gx = case["dims"][0] // 3
    want = np.array([[3 * (g % gx) + 1, 3 * (g // gx) + 1, 1] for g in case["taken"]], dtype=np.int32)
    assert np.array_equal(got, want.reshape(-1, 3)), (case["why"], got)
    tw = twin.select_ex(vol, 3, 3, case["fraction"], mask, case["connectivity"])
    assert np.array_equal(tw, want.reshape(-1, 3))


def test_plain_rule_is_the_special_case():
    p = synth.gen_random(3, (21, 18, 15), "u16", smooth=1.0)
    for b, s, f in [(3, 2, 0.3), (5, 3, 0.5), (3, 1, 0.1)]:
        a, va = oracle.select(p.ref, b, s, f)
        c, vc = oracle.select_ex(p.ref, b, s, f)
        assert np.array_equal(a, c) and np.array_equal(va, vc)


@pytest.mark.parametrize("conn", [6, 18, 26])
@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_twin_agrees(conn, dtype):
    for seed in range(3):
        p = synth.gen_random(10 + seed, (17, 14, 12), dtype, smooth=1.0)
        rng = np.random.default_rng(seed)
        mask = (rng.random(p.ref.shape) < 0.6).astype(np.uint8) if seed == 2 else None
        for b, s, f in [(3, 2, 0.4), (3, 1, 0.15), (5, 3, 0.9)]:
            a, _ = oracle.select_ex(p.ref, b, s, f, mask, conn)
            t = twin.select_ex(p.ref, b, s, f, mask, conn)
            assert np.array_equal(a, t), (conn, dtype, seed, b, s, f)


def _grid_index(c, b, s):
    h = (b - 1) // 2
    return (c - h) // s


@pytest.mark.parametrize("conn", [6, 18, 26])
def test_separation_and_greedy_maximality(conn):
    p = synth.gen_random(21, (24, 20, 16), "u16", smooth=1.5)
    b, s, f = 3, 2, 1.0  # K = N: the visit runs through every candidate
    taken, _ = oracle.select_ex(p.ref, b, s, f, None, conn)
    g = _grid_index(taken, b, s)
    limit = {6: 1, 18: 2, 26: 3}[conn]
    # no two taken blocks are neighbours
    for i in range(len(g)):
        d = np.abs(g - g[i])
        near = (d.max(axis=1) == 1) & (d.sum(axis=1) <= limit)
        assert not near.any(), i
    # every block left out has a taken neighbour ranked above it
    key, _ = oracle.block_variance(p.ref, b, s)
    G = oracle.grid_shape(p.dims, b, s)
    taken_set = {tuple(x) for x in g}
    rank = np.lexsort((np.arange(len(key)), -key))
    pos = np.empty(len(key), dtype=np.int64)
    pos[rank] = np.arange(len(key))
    for idx in range(len(key)):
        gx, gy, gz = idx % G[0], (idx // G[0]) % G[1], idx // (G[0] * G[1])
        if (gx, gy, gz) in taken_set:
            continue
        ok = False
        for (tx, ty, tz) in taken_set:
            d = (abs(tx - gx), abs(ty - gy), abs(tz - gz))
            if max(d) == 1 and sum(d) <= limit:
                tidx = (tz * G[1] + ty) * G[0] + tx
                ok = ok or pos[tidx] < pos[idx]
        assert ok, idx


def test_mask_count_rule():
    p = synth.gen_random(4, (20, 20, 20), "f32", smooth=1.0)
    mask = np.zeros(p.ref.shape, dtype=np.uint8)
    mask[:, :, :10] = 1  # left half of x
    b, s, f = 3, 2, 0.5
    c, _ = oracle.select_ex(p.ref, b, s, f, mask, 0)
    G = oracle.grid_shape(p.dims, b, s)
    centres_x = np.arange(G[0]) * s + 1
    n_in = int((centres_x < 10).sum()) * G[1] * G[2]
    assert len(c) == oracle.select_count(n_in, f)
    assert (c[:, 0] < 10).all()


# ---- the variants with per-axis block edges and strides (oracle.select_aniso_ex)

ANISO_SHAPES = [((3, 5, 1), (2, 3, 1), 0.5), ((5, 3, 3), (1, 2, 3), 0.9),
                ((1, 3, 5), (2, 1, 2), 0.3), ((3, 3, 3), (2, 1, 3), 1.0)]


@pytest.mark.parametrize("conn", [0, 6, 18, 26])
@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_aniso_twin_agrees(conn, dtype):
    p = synth.gen_random(31, (17, 14, 12), dtype, smooth=1.0)
    rng = np.random.default_rng(3)
    for mask in (None, (rng.random(p.ref.shape) < 0.7).astype(np.uint8)):
        for b, s, f in ANISO_SHAPES:
            a, _ = oracle.select_aniso_ex(p.ref, b, s, f, mask, conn)
            t = twin.select_aniso_ex(p.ref, b, s, f, mask, conn)
            assert np.array_equal(a, t), (conn, dtype, b, s, f)


@pytest.mark.parametrize("conn", [0, 6, 18, 26])
def test_aniso_equal_sizes_are_the_cubic_variants(conn):
    """Equal per-axis sizes give what the separately written cubic function
    gives, with and without a mask."""
    p = synth.gen_random(32, (20, 17, 15), "u16", smooth=1.2)
    mask = (np.random.default_rng(4).random(p.ref.shape) < 0.6).astype(np.uint8)
    for m in (None, mask):
        for b, s, f in [(3, 2, 0.6), (5, 1, 0.3), (3, 3, 1.0)]:
            a, va = oracle.select_aniso_ex(p.ref, (b, b, b), (s, s, s), f, m, conn)
            c, vc = oracle.select_ex(p.ref, b, s, f, m, conn)
            assert np.array_equal(a, c) and np.array_equal(va, vc), (conn, b, s, f)


def test_aniso_plain_rule_is_the_special_case():
    p = synth.gen_random(33, (19, 16, 13), "f32", smooth=1.0)
    for b, s, f in ANISO_SHAPES:
        a, _ = oracle.select_aniso_ex(p.ref, b, s, f, None, 0)
        c, _ = oracle.select_aniso(p.ref, b, s, f)
        assert np.array_equal(a, c), (b, s, f)


def _row_of_three(amps, along):
    """A volume of three 3x3x3 blocks in a row along x or z, block i a
    checkerboard of amplitude amps[i] (its variance rises with it)."""
    shape = (3, 3, 9) if along == "x" else (9, 3, 3)  # (nz, ny, nx)
    z, y, x = np.indices(shape)
    i = (x if along == "x" else z) // 3
    return (((x + y + z) % 2) * np.asarray(amps)[i]).astype(np.uint16)


@pytest.mark.parametrize("along", ["x", "z"])
def test_aniso_hand_case_neighbours_along_each_axis(along):
    """Three candidates in a row; the middle one varies most.  With any
    pattern its two neighbours are blocked; without one all three are taken.
    Per-axis edges (3, 3, 3) with strides 3 along the row and 1 across it."""
    vol = _row_of_three((10, 100, 50), along)
    s = (3, 1, 1) if along == "x" else (1, 1, 3)
    mid = [4, 1, 1] if along == "x" else [1, 1, 4]
    for conn in (6, 18, 26):
        got, _ = oracle.select_aniso_ex(vol, (3, 3, 3), s, 1.0, None, conn)
        assert got.tolist() == [mid], (along, conn, got)
    got, _ = oracle.select_aniso_ex(vol, (3, 3, 3), s, 1.0, None, 0)
    assert len(got) == 3


def test_aniso_mask_read_at_the_centre():
    """The mask is read at the candidate's centre, origin + (edge - 1) / 2 on
    each axis: a mask of one voxel per allowed block admits exactly those."""
    p = synth.gen_random(34, (15, 12, 9), "u16", smooth=1.0)
    b, s = (5, 3, 3), (5, 3, 3)
    mask = np.zeros(p.ref.shape, dtype=np.uint8)
    allowed = [(2, 1, 1), (7, 4, 4), (12, 10, 7)]  # centres (x, y, z)
    for x, y, z in allowed:
        mask[z, y, x] = 1
    mask[0, 0, 0] = 1  # a block's corner, not a centre
    got, _ = oracle.select_aniso_ex(p.ref, b, s, 1.0, mask, 0)
    assert sorted(map(tuple, got.tolist())) == sorted(allowed)
