"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Selection must be bit-exact (same centres, same order).  Matching follows the
parity rule in gpu_util.check_match (argmax within 1e-5 of the oracle's best
NCC, NCC and confidence within 1e-5 absolute).
"""

import sys

import numpy as np
import pytest

import oracle
import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import NCC_TOL, check_match, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, params=["fma", "dot2", "mfma"])
def arith(request, monkeypatch):
    """Every case runs with each form of the cross-term arithmetic: FP32 FMA,
    the exact int16 dot2 form and the fp16 matrix-core form (the last two for
    12-bit data only; float data always use FMA, and block edges or windows
    the matrix-core form does not serve fall back to dot2)."""
    monkeypatch.setenv("NRR_ARITH", request.param)
    return request.param


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    nrr.load()
    return torch


@pytest.fixture(scope="module")
def c1():
    return synth.gen_translation_f32(seed=0)


@pytest.fixture(scope="module")
def c2():
    return synth.gen_mri_u16(seed=0)


def gpu_select(vol, b, stride, frac):
    import torch

    c = nrr.select_blocks(to_dev(vol), b, stride, frac)
    torch.cuda.synchronize()
    return to_host(c)


def gpu_match(ref, flt, centers, b, w):
    import torch

    cd = torch.from_numpy(np.ascontiguousarray(centers, dtype=np.int32)).cuda()
    d, n, c = nrr.block_match(to_dev(ref), to_dev(flt), cd, b, w)
    torch.cuda.synchronize()
    return to_host(d), to_host(n), to_host(c)


# ------------------------------------------------------------ selection

def test_select_translation_f32(torch_dev, c1):
    say("select translation_f32 64^3 b7 s7 f0.2")
    got = gpu_select(c1.ref, 7, 7, 0.2)
    exp, _ = oracle.select(c1.ref, 7, 7, 0.2)
    assert got.shape == (146, 3) and np.array_equal(got, exp)


def test_select_mri_u16(torch_dev, c2):
    say("select mri_u16 256x256x124 b7 s7 f0.25")
    got = gpu_select(c2.ref, 7, 7, 0.25)
    exp, _ = oracle.select(c2.ref, 7, 7, 0.25)
    assert got.shape == (5508, 3) and np.array_equal(got, exp)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("dims,b,stride,frac", [
    ((10, 9, 8), 3, 1, 0.3), ((13, 7, 11), 5, 2, 0.5), ((40, 33, 21), 7, 3, 0.15),
    ((31, 29, 23), 9, 2, 0.7), ((20, 20, 20), 3, 1, 1.0), ((17, 17, 16), 15, 1, 0.5),
    ((70, 9, 9), 3, 1, 0.02)])
def test_select_tiny(torch_dev, dtype, dims, b, stride, frac):
    say("select random", dtype, dims, b, stride, frac)
    p = synth.gen_random(5, dims, dtype, smooth=0.8)
    got = gpu_select(p.ref, b, stride, frac)
    exp, _ = oracle.select(p.ref, b, stride, frac)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_select_ties_take_lower_index(torch_dev, dtype):
    say("select flat volume ties", dtype)
    vol = np.zeros((12, 11, 10), dtype=np.uint16 if dtype == "u16" else np.float32)
    vol[8:, 8:, 7:] = 100  # a few non-flat blocks at high indices, the rest tie at 0
    got = gpu_select(vol, 3, 1, 0.4)
    exp, _ = oracle.select(vol, 3, 1, 0.4)
    assert np.array_equal(got, exp)


def test_select_large_grid_radix_paths(torch_dev):
    """Many candidates with many equal keys spread over several compaction
    tiles (exercises the multi-tile prefix and the equal-key quota)."""
    say("select 120x100x60 stride 1 with plateaus")
    rng = np.random.default_rng(8)
    vol = (rng.integers(0, 4, size=(60, 100, 120)) * 1000).astype(np.uint16)
    vol[:, :50, :] = 7
    got = gpu_select(vol, 3, 1, 0.37)
    exp, _ = oracle.select(vol, 3, 1, 0.37)
    assert np.array_equal(got, exp)


# ------------------------------------------------------------- matching

def test_match_translation_full(torch_dev, c1):
    say("match translation_f32 all 146 blocks W5")
    centers, _ = oracle.select(c1.ref, 7, 7, 0.2)
    d, n, c = gpu_match(c1.ref, c1.flt, centers, 7, 5)
    gap, err, differ = check_match(c1.ref, c1.flt, centers, 7, 5, d, n, c, "c1")
    say("c1 gap %.2e err %.2e differ %d" % (gap, err, differ))


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("dims,b,w", [
    ((10, 9, 8), 3, 1), ((13, 7, 11), 3, 3), ((13, 12, 11), 5, 2), ((19, 17, 15), 5, 4),
    ((24, 21, 19), 7, 5), ((30, 26, 23), 7, 6), ((29, 27, 25), 9, 4), ((33, 31, 29), 9, 7),
    ((27, 25, 23), 11, 3), ((29, 28, 27), 13, 3), ((31, 30, 29), 15, 2), ((16, 15, 14), 7, 0)])
def test_match_tiny(torch_dev, dtype, dims, b, w):
    say("match random", dtype, dims, b, w)
    p = synth.gen_random(17, dims, dtype, smooth=1.0)
    centers, _ = oracle.select(p.ref, b, 2, 0.5)
    d, n, c = gpu_match(p.ref, p.flt, centers, b, w)
    check_match(p.ref, p.flt, centers, b, w, d, n, c, "tiny")


def test_match_mri_full_launch_all_blocks(torch_dev, c2):
    """All 5508 selected blocks of the 256x256x124 workload in one launch (the
    benchmark's configuration), every one checked against the oracle,
    including the 1696 whose windows the volume clips."""
    say("match mri_u16 5508 blocks W10 (all checked)")
    centers, _ = oracle.select(c2.ref, 7, 7, 0.25)
    d, n, c = gpu_match(c2.ref, c2.flt, centers, 7, 10)
    dims = np.array(c2.dims)
    border = np.any((centers - 3 - 10 < 0) | (centers + 3 + 10 > dims - 1), axis=1)
    assert border.sum() > 1000
    gap, err, differ = check_match(c2.ref, c2.flt, centers, 7, 10, d, n, c, "c2")
    say("c2 gap %.2e err %.2e differ %d of %d" % (gap, err, differ, len(centers)))


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("b", [5, 7, 9])
@pytest.mark.parametrize("w", [13, 14, 15])
def test_match_large_windows(torch_dev, dtype, b, w):
    """Windows of 13-15 voxels (the serving range's top) with blocks near
    every face, so windows are clipped on each side, and interior blocks."""
    say("match large window", dtype, b, w)
    dims = (2 * w + b + 9, 2 * w + b + 7, 2 * w + b + 5)
    p = synth.gen_random(100 + 10 * b + w, dims, dtype, smooth=1.5)
    h = b // 2
    rng = np.random.default_rng(w * 31 + b)
    cs = [[rng.integers(h, dims[0] - h), rng.integers(h, dims[1] - h),
           rng.integers(h, dims[2] - h)] for _ in range(14)]
    cs += [[h, h, h], [dims[0] - 1 - h, dims[1] - 1 - h, dims[2] - 1 - h],
           [dims[0] // 2, h, dims[2] - 1 - h], [h + w, h + w, h + w]]
    centers = np.array(cs, dtype=np.int32)
    d, n, c = gpu_match(p.ref, p.flt, centers, b, w)
    check_match(p.ref, p.flt, centers, b, w, d, n, c, "large window")


# ----------------------------------------------------------- invariants

@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_self_match(torch_dev, dtype):
    say("self match", dtype)
    p = synth.gen_random(3, (30, 28, 26), dtype, smooth=1.2)
    centers, _ = oracle.select(p.ref, 7, 3, 0.3)
    d, n, c = gpu_match(p.ref, p.ref, centers, 7, 4)
    assert np.all(d == 0)
    assert np.all(np.abs(n - 1.0) <= 1e-6) and np.all(n <= 1.0 + 1e-6)


def test_scale_by_two(torch_dev, arith):
    """x2 intensities: selection is bit-identical (exact integer keys); the
    exact dot2 form also gives bit-identical displacements and NCC (every
    rounding step scales by a power of two); the FMA and matrix-core forms
    centre the block on a rounded integer, which does not scale with the data,
    so they are held to the parity rule instead."""
    say("u16 x2 scale", arith)
    p = synth.gen_random(4, (28, 27, 26), "u16", smooth=1.0)
    ref = (p.ref // 2).astype(np.uint16)
    flt = (p.flt // 2).astype(np.uint16)
    ref2, flt2 = (ref * 2).astype(np.uint16), (flt * 2).astype(np.uint16)
    centers = gpu_select(ref, 5, 2, 0.4)
    centers2 = gpu_select(ref2, 5, 2, 0.4)
    assert np.array_equal(centers, centers2)
    d1, n1, c1_ = gpu_match(ref, flt, centers, 5, 4)
    d2, n2, c2_ = gpu_match(ref2, flt2, centers, 5, 4)
    if arith == "dot2":
        assert np.array_equal(d1, d2) and np.array_equal(n1, n2)
    else:
        check_match(ref, flt, centers, 5, 4, d1, n1, c1_, "x1")
        check_match(ref2, flt2, centers, 5, 4, d2, n2, c2_, "x2")


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_periodic_tie_lowest_index(torch_dev, dtype, arith):
    say("periodic tie", dtype)
    rng = np.random.default_rng(5)
    base = rng.integers(0, 4096, size=(20, 21, 3))
    vol = np.tile(base, (1, 1, 9))[:, :, :25]
    vol = vol.astype(np.uint16) if dtype == "u16" else vol.astype(np.float32) / 4096
    centers = np.array([[12, 10, 9], [5, 6, 7], [19, 14, 12], [3, 3, 3]], dtype=np.int32)
    d, n, c = gpu_match(vol, vol, centers, 3, 4)
    do, no, _ = oracle.match(vol, vol, centers, 3, 4)
    if arith == "mfma" and dtype == "u16":
        # the FP32 sums of the matrix-core form round in a position-dependent
        # order, so shifts whose exact NCCs are equal need not rank equal:
        # the winner must be one of the exactly tied shifts
        srf = oracle.ncc_surface(vol, vol, centers, 3, 4)
        for k in range(len(centers)):
            assert srf[k, d[k, 2] + 4, d[k, 1] + 4, d[k, 0] + 4] == no[k]
    else:
        assert np.array_equal(d, do)  # exact ties -> smallest shift index on both sides
    assert np.all(np.abs(n - 1) <= 1e-6)


def test_flat_window_and_flat_block(torch_dev):
    say("flat window / flat block")
    p = synth.gen_random(2, (20, 20, 20), "u16")
    flt = np.full_like(p.flt, 1234)
    centers = np.array([[5, 6, 4], [2, 2, 2], [16, 16, 16], [10, 10, 10]], dtype=np.int32)
    d, n, c = gpu_match(p.ref, flt, centers, 3, 3)
    do, no, _ = oracle.match(p.ref, flt, centers, 3, 3)
    assert np.array_equal(d, do) and np.all(n == 0) and np.all(c == 0)
    ref = p.ref.copy()
    ref[:10, :10, :10] = 77  # block at (5,5,5) flat
    d, n, c = gpu_match(ref, p.flt, np.array([[5, 5, 5]], np.int32), 3, 2)
    assert list(d[0]) == [-2, -2, -2] and n[0] == 0


def test_out_of_volume_centres(torch_dev):
    say("out-of-volume centres")
    p = synth.gen_random(1, (16, 15, 14), "u16", smooth=1.0)
    centers = np.array([[0, 5, 5], [7, 7, 7], [7, 14, 7], [7, 7, -3], [8, 8, 8]], np.int32)
    d, n, c = gpu_match(p.ref, p.flt, centers, 3, 2)
    assert np.isnan(n[0]) and np.isnan(n[2]) and np.isnan(n[3])
    assert c[0] == 0 and np.all(d[[0, 2, 3]] == 0)
    check_match(p.ref, p.flt, centers, 3, 2, d, n, c, "oov")


def test_run_twice_bitwise(torch_dev, c1):
    say("determinism")
    centers, _ = oracle.select(c1.ref, 7, 7, 0.2)
    a = gpu_match(c1.ref, c1.flt, centers, 7, 5)
    b = gpu_match(c1.ref, c1.flt, centers, 7, 5)
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)


def test_n_zero_noop(torch_dev):
    import torch

    say("n = 0")
    v = to_dev(np.zeros((10, 10, 10), np.uint16))
    d, n, c = nrr.block_match(v, v, torch.zeros((0, 3), dtype=torch.int32, device="cuda"), 3, 2)
    assert d.shape == (0, 3)


@pytest.mark.parametrize("b,w", [(7, 3), (9, 3), (11, 2), (13, 2), (15, 1)])
def test_extreme_contrast_no_overflow(torch_dev, b, w):
    """Checkerboards of 0 / 4095: the largest magnitudes the int32 groups of
    the 12-bit kernel must absorb."""
    say("extreme contrast", b, w)
    zz, yy, xx = np.meshgrid(np.arange(b + 2 * w + 6), np.arange(b + 2 * w + 5),
                             np.arange(b + 2 * w + 4), indexing="ij")
    ref = (((xx + yy + zz) % 2) * 4095).astype(np.uint16)
    rng = np.random.default_rng(b)
    flt = np.where(rng.random(ref.shape) < 0.9, ref, 4095 - ref).astype(np.uint16)
    h = b // 2
    centers = np.array([[h + w, h + w, h + w], [h + w + 1, h + w + 2, h + w + 1]], np.int32)
    d, n, c = gpu_match(ref, flt, centers, b, w)
    check_match(ref, flt, centers, b, w, d, n, c, "contrast")
