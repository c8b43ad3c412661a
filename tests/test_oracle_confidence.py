"""Pins of the oracle's directional confidence (structure tensor of the
pre-operative block, scaled to trace = conf)."""

import numpy as np
import pytest

import oracle
from oracle import twin
from paper_2308_10868_amd import synth


def centres_inside(dims, b, n, seed):
    rng = np.random.default_rng(seed)
    h = (b - 1) // 2
    return np.stack([rng.integers(h, d - h, size=n) for d in dims], axis=1).astype(np.int32)


def test_ramp_along_one_axis_gives_that_axis():
    nz, ny, nx = 12, 11, 10
    for axis in range(3):
        coords = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="xy")
        z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
        vol = [x, y, z][axis].astype(np.float32) * 3.0 + 1.0
        c = np.array([[5, 5, 5], [4, 6, 7]], dtype=np.int32)
        s = oracle.structure_confidence(vol, c, 3, np.array([0.8, 0.5]))
        want = np.zeros((2, 6))
        want[:, axis] = [0.8, 0.5]
        assert np.allclose(s, want, atol=1e-15), axis


def test_symmetric_psd_trace_equals_conf():
    p = synth.gen_random(5, (20, 18, 16), "u16", smooth=1.0)
    c = centres_inside(p.dims, 5, 30, 1)
    conf = np.linspace(0.0, 1.0, 30)
    s = oracle.structure_confidence(p.ref, c, 5, conf)
    assert np.allclose(s[:, :3].sum(axis=1), conf, atol=1e-12)
    for row in s:
        m = np.array([[row[0], row[3], row[4]], [row[3], row[1], row[5]], [row[4], row[5], row[2]]])
        assert np.linalg.eigvalsh(m).min() > -1e-12


def test_axis_permutation_permutes_the_tensor():
    p = synth.gen_random(6, (14, 14, 14), "f32", smooth=1.0)
    c = centres_inside(p.dims, 5, 10, 2)
    conf = np.ones(10)
    s = oracle.structure_confidence(p.ref, c, 5, conf)
    vt = np.ascontiguousarray(np.transpose(p.ref, (2, 1, 0)))  # swap x and z
    ct = c[:, ::-1].copy()
    st = oracle.structure_confidence(vt, ct, 5, conf)
    # xx <-> zz, xy <-> yz (y fixed), xz unchanged
    assert np.allclose(st[:, [2, 1, 0, 5, 4, 3]], s, atol=1e-12)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_twin_agrees_including_border_planes(dtype):
    p = synth.gen_random(7, (15, 13, 11), dtype, smooth=0.8)
    h = 2
    c = np.array([[h, h, h], [15 - 1 - h, 13 - 1 - h, 11 - 1 - h], [7, 6, 5], [2, 10, 3]],
                 dtype=np.int32)
    conf = np.array([1.0, 0.3, 0.7, 0.2])
    assert np.allclose(oracle.structure_confidence(p.ref, c, 5, conf),
                       twin.structure_confidence(p.ref, c, 5, conf), rtol=1e-12, atol=1e-14)


def test_outside_or_flat_blocks_give_zero():
    vol = np.full((9, 9, 9), 7.0, dtype=np.float32)
    s = oracle.structure_confidence(vol, np.array([[4, 4, 4], [0, 4, 4]], dtype=np.int32), 3,
                                    np.array([1.0, 1.0]))
    assert np.all(s == 0.0)
