"""GPU: the window-statistics table and the plane-pair volume that the
12-bit search reads, against their plain definitions computed here with
NumPy (white box: the workspace holds the table of one record per block
origin, 16 rows of slack, 256-byte alignment, then one pair word per voxel).

A record is {int32 s = sum over the block at that origin of (F - 2048),
float32 r = 1/sqrt(N sum (F - 2048)^2 - s^2), 0 for a flat block}; a pair
word is (F(z) - 2048) | (F(z + 1) - 2048) << 16 as two int16, the upper half
0 on the last plane.  The volumes span several 64 x 4 origin tiles and
several z-runs, with ragged edges on every axis."""

import sys

import numpy as np
import pytest

import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu

TILE_SLACK = 16


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def box_sum(v, b):
    """Sum over every b x b x b box of v ([z][y][x]), indexed by its lowest corner."""
    c = np.zeros(tuple(n + 1 for n in v.shape), np.int64)
    c[1:, 1:, 1:] = v.cumsum(0).cumsum(1).cumsum(2)
    return (c[b:, b:, b:] - c[:-b, b:, b:] - c[b:, :-b, b:] - c[b:, b:, :-b]
            + c[:-b, :-b, b:] + c[:-b, b:, :-b] + c[b:, :-b, :-b] - c[:-b, :-b, :-b])


@pytest.mark.parametrize("dims,b,seed", [((70, 9, 12), 3, 1), ((23, 19, 17), 5, 2),
                                         ((130, 21, 40), 7, 3), ((66, 13, 50), 9, 4),
                                         ((20, 20, 20), 15, 5)])
def test_statistics_table_and_pair_volume(dims, b, seed):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    p = synth.gen_random(seed, dims, "u16", smooth=1.0)
    p.flt[0, 0, :5] = [0, 4095, 0, 4095, 2048]  # the extremes of the 12-bit range
    say("stats table", dims, b)
    ws = nrr.window_stats(to_dev(p.flt), b)
    torch.cuda.synchronize()
    raw = ws.cpu().numpy()
    nx, ny, nz = dims
    ox, oy, oz = nx - b + 1, ny - b + 1, nz - b + 1
    f = p.flt.astype(np.int64) - 2048
    s_want = box_sum(f, b)
    q_want = box_sum(f * f, b)
    n_rec = ox * oy * oz
    rec = raw[:n_rec * 8].view(np.int32).reshape(oz, oy, ox, 2)
    assert np.array_equal(rec[..., 0], s_want)
    var = b ** 3 * q_want - s_want * s_want
    r_want = np.zeros(var.shape)
    r_want[var > 0] = 1.0 / np.sqrt(var[var > 0].astype(np.float64))
    r_got = rec[..., 1].copy().view(np.float32).astype(np.float64)
    assert np.all((r_got == 0) == (r_want == 0))
    assert np.allclose(r_got, r_want, rtol=2e-6, atol=0)
    table = ((n_rec + TILE_SLACK * (ox + 1)) * 8 + 255) // 256 * 256
    nvox = nx * ny * nz
    pairs = raw[table:table + 4 * nvox].view(np.uint32).reshape(nz, ny, nx)
    lo = (f & 0xFFFF).astype(np.uint32)
    hi = np.zeros_like(lo)
    hi[:-1] = lo[1:]
    assert np.array_equal(pairs, lo | hi << 16)


def test_check_volume_counts_voxels_outside_the_contract():
    """nrr_check_volume: 12-bit voxels above 4095 and non-finite floats."""
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    nrr.load()
    v = np.random.default_rng(0).integers(0, 4096, size=(9, 10, 11)).astype(np.uint16)
    assert nrr.check_volume(to_dev(v)) == 0
    v[3, 4, 5] = 4096
    v[8, 9, 10] = 65535
    assert nrr.check_volume(to_dev(v)) == 2
    f = np.random.default_rng(1).standard_normal((5, 6, 7)).astype(np.float32)
    assert nrr.check_volume(to_dev(f)) == 0
    f[0, 0, 0], f[4, 5, 6], f[2, 2, 2] = np.nan, np.inf, -np.inf
    assert nrr.check_volume(to_dev(f)) == 3
