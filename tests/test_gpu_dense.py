"""GPU parity on the large dense workload (512 x 512 x 256 u16 blob volumes,
blocks 9^3 on an overlapping stride-5 grid, F = 0.70 -> K = 357,035, window
+-12), in the launch the benchmark times: the selection compared whole
against the oracle, the search on a seeded sample of 2048 selected blocks
(about a quarter of them near a face, with clipped windows) under the parity
rule of the other GPU tests, with each form of the cross-term arithmetic."""

import sys

import numpy as np
import pytest

import oracle
import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import check_match, to_dev, to_host

pytestmark = pytest.mark.gpu

B, STRIDE, FRAC, W = 9, 5, 0.70, 12


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dense():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    nrr.load()
    say("generating the 512x512x256 blob pair (about a minute)")
    p = synth.gen_blobs_u16(seed=0)
    want, _ = oracle.select(p.ref, B, STRIDE, FRAC)
    return p, want


def test_select_whole(dense):
    import torch

    p, want = dense
    say("dense select", len(want))
    got = to_host(nrr.select_blocks(to_dev(p.ref), B, STRIDE, FRAC))
    torch.cuda.synchronize()
    assert len(want) == 357035
    assert np.array_equal(got, want)


@pytest.mark.parametrize("arith", ["dot2", "fma", "mfma"])
def test_match_sampled(dense, monkeypatch, arith):
    import torch

    monkeypatch.setenv("NRR_ARITH", arith)
    p, want = dense
    r, f = to_dev(p.ref), to_dev(p.flt)
    c = torch.from_numpy(want).cuda()
    say("dense match", arith, len(want))
    d, n, cf = nrr.block_match(r, f, c, B, W)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(5).choice(len(want), 2048, replace=False))
    dims = np.array(p.dims)
    near = np.any((want[idx] - (B - 1) // 2 - W < 0) | (want[idx] + (B - 1) // 2 + W > dims - 1),
                  axis=1)
    assert near.sum() > 200  # clipped windows are part of the sample
    say("dense oracle", len(idx), "blocks,", int(near.sum()), "near a face")
    check_match(p.ref, p.flt, want[idx], B, W, to_host(d)[idx], to_host(n)[idx],
                to_host(cf)[idx], "dense " + arith)
