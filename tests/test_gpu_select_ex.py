"""GPU: selection with a candidate mask and a connectivity pattern, against
the oracle (bit-exact: same centres, same order)."""

import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    nrr.load()
    return torch


def gpu_ex(vol, b, s, f, mask, conn):
    import torch

    c = nrr.select_blocks_ex(to_dev(vol), b, s, f, None if mask is None else to_dev(mask), conn)
    torch.cuda.synchronize()
    return to_host(c)


@pytest.mark.parametrize("conn", [0, 6, 18, 26])
@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_tiny_random_with_masks(torch_dev, conn, dtype):
    for seed in range(3):
        p = synth.gen_random(30 + seed, (19, 15, 13), dtype, smooth=1.0)
        rng = np.random.default_rng(seed)
        mask = (rng.random(p.ref.shape) < 0.7).astype(np.uint8) if seed != 0 else None
        for b, s, f in [(3, 2, 0.4), (3, 1, 0.2), (5, 3, 0.9), (3, 3, 1.0)]:
            say("select_ex", dtype, conn, seed, b, s, f)
            want, _ = oracle.select_ex(p.ref, b, s, f, mask, conn)
            got = gpu_ex(p.ref, b, s, f, mask, conn)
            assert np.array_equal(got, want), (dtype, conn, seed, b, s, f)


def test_golden_cases(torch_dev):
    from tests.test_oracle_select_ex import golden_volume

    for case in json.load(open(os.path.join(HERE, "golden", "select_connectivity.json")))["cases"]:
        vol, mask = golden_volume(case)
        got = gpu_ex(vol, 3, 3, case["fraction"], mask, case["connectivity"])
        gx = case["dims"][0] // 3
        want = np.array([[3 * (g % gx) + 1, 3 * (g // gx) + 1, 1] for g in case["taken"]],
                        dtype=np.int32).reshape(-1, 3)
        assert np.array_equal(got, want), case["why"]


@pytest.mark.parametrize("conn", [6, 26])
def test_mri_workload_with_region_mask(torch_dev, conn):
    p = synth.gen_mri_u16(seed=0)
    nz, ny, nx = p.ref.shape
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    # an ellipsoidal region (a stand-in for the intracranial cavity)
    mask = (((x - nx / 2) / (0.42 * nx)) ** 2 + ((y - ny / 2) / (0.45 * ny)) ** 2 +
            ((z - nz / 2) / (0.48 * nz)) ** 2 <= 1.0).astype(np.uint8)
    say("select_ex mri", conn)
    want, _ = oracle.select_ex(p.ref, 7, 7, 0.25, mask, conn)
    got = gpu_ex(p.ref, 7, 7, 0.25, mask, conn)
    assert len(want) > 300  # a nontrivial set (26-connectivity leaves about 800)
    assert np.array_equal(got, want)


def test_plain_special_case_equals_select_blocks(torch_dev):
    p = synth.gen_translation_f32(seed=0)
    a = to_host(nrr.select_blocks(to_dev(p.ref), 7, 7, 0.2))
    b = gpu_ex(p.ref, 7, 7, 0.2, None, 0)
    assert np.array_equal(a, b)


# Grids above 24,576 candidates take the round-launch path.
@pytest.mark.parametrize("conn", [0, 6, 18, 26])
@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_large_grids_every_pattern(torch_dev, conn, dtype):
    p = synth.gen_random(50, (66, 60, 52), dtype, smooth=1.5)  # b 3, stride 1: 184,800
    rng = np.random.default_rng(7)
    for mask in (None, (rng.random(p.ref.shape) < 0.8).astype(np.uint8)):
        for b, s, f in [(3, 1, 0.3), (5, 2, 0.9)]:
            say("select_ex large", dtype, conn, mask is not None, b, s, f)
            want, _ = oracle.select_ex(p.ref, b, s, f, mask, conn)
            got = gpu_ex(p.ref, b, s, f, mask, conn)
            assert np.array_equal(got, want), (dtype, conn, b, s, f)


def test_large_grid_with_long_decision_chains(torch_dev):
    """Block variance rising along x and y (a checkerboard of growing
    amplitude): every candidate's decision waits for its neighbour's, so the
    chains run across the whole grid and through many tiles."""
    nz, ny, nx = 12, 90, 300
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    vol = (((x + y + z) % 2) * (10 * x + 3 * y + 1)).astype(np.uint16)
    vol = np.minimum(vol, 4095).astype(np.uint16)
    for conn in (6, 26):
        say("select_ex chains", conn)
        want, _ = oracle.select_ex(vol, 3, 1, 1.0, None, conn)
        got = gpu_ex(vol, 3, 1, 1.0, None, conn)
        assert len(want) > 1000
        assert np.array_equal(got, want), conn


@pytest.mark.parametrize("conn", [6, 26])
def test_dense_grid_with_region_mask(torch_dev, conn):
    """The dense 512x512x256 workload's grid (9^3 blocks, stride 5: 510,050
    candidates), a region mask and a pattern, against the oracle."""
    import time

    import torch

    p = synth.gen_blobs_u16(seed=0)
    nz, ny, nx = p.ref.shape
    z, y, x = np.ogrid[0:nz, 0:ny, 0:nx]
    mask = (((x - nx / 2) / (0.42 * nx)) ** 2 + ((y - ny / 2) / (0.45 * ny)) ** 2 +
            ((z - nz / 2) / (0.48 * nz)) ** 2 <= 1.0).astype(np.uint8)
    say("select_ex dense", conn)
    want, _ = oracle.select_ex(p.ref, 9, 5, 0.7, mask, conn)
    ref, md = to_dev(p.ref), to_dev(mask)
    nrr.select_blocks_ex(ref, 9, 5, 0.7, md, conn)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    c = nrr.select_blocks_ex(ref, 9, 5, 0.7, md, conn)
    torch.cuda.synchronize()
    say("select_ex dense %d: %d taken, %.2f ms" % (conn, len(c), (time.perf_counter() - t) * 1e3))
    assert len(want) > 10000  # 6: about 77,000; 26: about 19,000
    assert np.array_equal(to_host(c), want)


# Per-axis block edges and strides with the variants.
@pytest.mark.parametrize("conn", [0, 6, 18, 26])
@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_aniso_variants_small(torch_dev, conn, dtype):
    import torch

    p = synth.gen_random(60, (23, 19, 15), dtype, smooth=1.0)
    rng = np.random.default_rng(8)
    for mask in (None, (rng.random(p.ref.shape) < 0.7).astype(np.uint8)):
        for b, s, f in [((3, 5, 1), (2, 3, 1), 0.5), ((5, 3, 3), (1, 2, 3), 0.9),
                        ((1, 3, 5), (2, 1, 2), 0.3), ((7, 3, 3), (3, 3, 1), 1.0)]:
            say("select_aniso_ex", dtype, conn, mask is not None, b, s, f)
            want, _ = oracle.select_aniso_ex(p.ref, b, s, f, mask, conn)
            c = nrr.select_blocks_aniso_ex(to_dev(p.ref), b, s, f,
                                           None if mask is None else to_dev(mask), conn)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(c), want), (dtype, conn, b, s, f)


@pytest.mark.parametrize("conn", [6, 26])
def test_aniso_variants_mri_slices(torch_dev, conn):
    """The MRI pair with blocks thinner along the slice axis (7 x 7 x 3,
    stride 7 x 7 x 3: 53,136 candidates, the round-launch path) inside an
    ellipsoidal region."""
    import torch

    p = synth.gen_mri_u16(seed=0)
    nz, ny, nx = p.ref.shape
    z, y, x = np.ogrid[0:nz, 0:ny, 0:nx]
    mask = (((x - nx / 2) / (0.42 * nx)) ** 2 + ((y - ny / 2) / (0.45 * ny)) ** 2 +
            ((z - nz / 2) / (0.48 * nz)) ** 2 <= 1.0).astype(np.uint8)
    say("select_aniso_ex mri", conn)
    want, _ = oracle.select_aniso_ex(p.ref, (7, 7, 3), (7, 7, 3), 0.25, mask, conn)
    c = nrr.select_blocks_aniso_ex(to_dev(p.ref), (7, 7, 3), (7, 7, 3), 0.25, to_dev(mask), conn)
    torch.cuda.synchronize()
    assert len(want) > 1000
    assert np.array_equal(to_host(c), want)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_plain_selection_large_grid_with_ties(torch_dev, dtype):
    """Grids above 32,768 candidates take the multi-workgroup radix select,
    smaller ones the one-workgroup select with its keys in registers: half
    the volume is flat, so thousands of candidates share the key 0 and the
    K-th key falls among them (ties to the lower grid index)."""
    import torch

    p = synth.gen_random(70, (120, 100, 90), dtype, smooth=1.0)
    ref = p.ref.copy()
    ref[:, :, :60] = ref[0, 0, 0]  # flat half
    for b, s, f in [(3, 2, 0.7), (5, 1, 0.55), (3, 1, 0.05), (15, 8, 0.3)]:
        say("plain selection large", dtype, b, s, f)
        want, _ = oracle.select(ref, b, s, f)
        got = nrr.select_blocks(to_dev(ref), b, s, f)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(got), want), (dtype, b, s, f)
    small = ref[:64, :64, :64].copy()  # b 3, stride 2: 29,791 candidates (one workgroup)
    for f in (0.6, 0.999):
        want, _ = oracle.select(small, 3, 2, f)
        got = nrr.select_blocks(to_dev(small), 3, 2, f)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(got), want), (dtype, "29,791", f)
