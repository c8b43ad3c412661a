"""GPU: the plain selection's code paths against the oracle, bit for bit:
keys read by candidate rows (stride >= edge in x and y, the row chunks of a
workgroup ragged at the end, gaps between candidates, full 16-bit values),
and the one-workgroup radix select near its 32,768-candidate limit, with
few and with many keys equal to the K-th (the LDS-list path and the
register path)."""

import sys

import numpy as np
import pytest

import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import to_dev
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    nrr.load()
    return torch


def gpu_select(vol, b, stride, frac):
    import torch

    c = nrr.select_blocks(to_dev(vol), b, stride, frac)
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("dims,b,stride,frac,full16", [
    ((200, 37, 30), 5, 5, 0.3, False),   # 40 candidates per row: chunks of 12, 12, 12, 4
    ((150, 40, 33), 7, 9, 0.25, False),  # gaps of 2 voxels between candidates
    ((255, 20, 12), 3, 3, 0.5, True),    # 85 per row, values over the whole 16-bit range
    ((100, 46, 31), 15, 15, 0.6, False),  # the largest edge: 4 candidates per chunk
    ((64, 64, 64), 7, 11, 0.1, True),
])
def test_row_keys_against_the_oracle(torch_dev, dims, b, stride, frac, full16):
    say("select by candidate rows", dims, b, stride, frac, full16)
    if full16:
        rng = np.random.default_rng(b * 31 + stride)
        vol = rng.integers(0, 65536, size=dims[::-1]).astype(np.uint16)
    else:
        vol = synth.gen_mri_u16(seed=b + stride, dims=dims).ref
    got = gpu_select(vol, b, stride, frac)
    exp, _ = oracle.select(vol, b, stride, frac)
    assert np.array_equal(got, exp)


def test_one_workgroup_select_near_its_limit(torch_dev):
    """32 x 32 x 32 = 32,768 candidates (the most one workgroup takes), keys
    mostly distinct: the matching keys move to the LDS list."""
    say("select 32768 candidates, distinct keys")
    vol = synth.gen_random(11, (96, 96, 96), "u16", smooth=0.6).ref
    got = gpu_select(vol, 3, 3, 0.37)
    exp, _ = oracle.select(vol, 3, 3, 0.37)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("levels,frac", [(3, 0.5), (2, 0.9), (40, 0.33)])
def test_one_workgroup_select_with_many_equal_keys(torch_dev, levels, frac):
    """Blocks built from a few patterns: thousands of keys equal the K-th,
    so the passes stay on the registers and the equal keys are taken by
    lowest grid index."""
    say("select equal keys", levels, frac)
    rng = np.random.default_rng(levels)
    b = 5
    g = (30, 28, 26)  # 21,840 candidates
    pats = [rng.integers(0, 4096, size=(b, b, b)).astype(np.uint16) for _ in range(levels)]
    pick = rng.integers(0, levels, size=g[::-1])
    vol = np.zeros((g[2] * b, g[1] * b, g[0] * b), np.uint16)
    for z in range(g[2]):
        for y in range(g[1]):
            for x in range(g[0]):
                vol[z * b:(z + 1) * b, y * b:(y + 1) * b, x * b:(x + 1) * b] = pats[pick[z, y, x]]
    got = gpu_select(vol, b, b, frac)
    exp, _ = oracle.select(vol, b, b, frac)
    assert np.array_equal(got, exp)


def test_float_select_one_workgroup(torch_dev):
    """Float keys (bit patterns of FP64 variances) through the same select."""
    say("select f32 stride = edge")
    vol = synth.gen_random(12, (120, 90, 60), "f32", smooth=0.7).ref
    got = gpu_select(vol, 5, 5, 0.2)
    exp, _ = oracle.select(vol, 5, 5, 0.2)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("dims,frac", [((18, 18, 18), 0.37), ((19, 18, 18), 0.37),
                                       ((18, 18, 18), 1.0)])
def test_select_around_the_small_grid_bound(torch_dev, dtype, dims, frac):
    """Grids of 4096 candidates take the select with 4 key slots per thread,
    4352 candidates the one with 32: both against the oracle, with plateaus of
    equal keys around the K-th."""
    say("select around 4096 candidates", dtype, dims, frac)
    rng = np.random.default_rng(sum(dims))
    vol = rng.integers(0, 6, size=dims[::-1]) * 500
    vol = vol.astype(np.uint16) if dtype == "u16" else vol.astype(np.float32) * 0.37
    got = gpu_select(vol, 3, 1, frac)
    exp, _ = oracle.select(vol, 3, 1, frac)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("dims,b,stride,wide", [
    ((40, 33, 21), 3, 1, False),   # 27 voxels: nine rows of three
    ((31, 29, 23), 5, 2, True),    # 125: 25 rows, a ring of four row buffers
    ((40, 36, 30), 9, 3, True),    # 729: 81 rows
    ((17, 17, 16), 15, 1, True),   # 3375: the largest edge
    ((30, 28, 26), 7, 2, True),    # the other row lengths of the row walk
    ((33, 31, 29), 11, 3, True),
    ((27, 26, 25), 13, 2, False),
])
def test_float_keys_bitwise_against_the_oracle(torch_dev, dims, b, stride, wide):
    """Every candidate's float key (the FP64 two-pass variance summed in z, y,
    x order, left by the plain selection at the start of its workspace) equals
    the oracle's bit for bit.  With values spread over many binades a sum
    taken in another order would round differently."""
    torch = torch_dev
    say("float keys", dims, b, stride, wide)
    vol = synth.gen_random(b + stride, dims, "f32", smooth=0.0 if wide else 0.8).ref
    if wide:
        rng = np.random.default_rng(b * 7 + stride)
        vol = (vol * 10.0 ** rng.uniform(-4, 4, size=vol.shape)).astype(np.float32)
    ws = torch.zeros(nrr.select_workspace_bytes(dims, b, stride), dtype=torch.uint8,
                     device="cuda")
    nrr.select_blocks(to_dev(vol), b, stride, 0.3, workspace=ws)
    torch.cuda.synchronize()
    key, _ = oracle.block_variance(vol, b, stride)
    got = ws[:key.size * 8].view(torch.int64).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, key.view(np.uint64))
