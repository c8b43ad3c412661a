"""GPU: every compiled search shape against the oracle.

Each shape the library compiles (the plain search's tile shapes, with their
planned z-chunk and the finer splits the tuner times, the matrix-core form,
and the batched search's shapes) is pinned through the C ABI
(nrr_set_tuned_shape), confirmed as the one a launch would use
(nrr_match_plan, nrr_batch_shapes), and run on a small volume with blocks on
every face and in the interior; the results must hold the oracle's parity
rule.
"""

import sys

import numpy as np
import pytest

import oracle
import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import check_match, to_dev, to_host

pytestmark = pytest.mark.gpu

W = 4  # window: 9 displacement planes, so the finer z-chunk splits exist
KEYS = ("arith", "rx", "ry", "nt", "pf")

# The batched search's compiled shapes (256 threads, no record prefetch
# unless pf = 1): float data with the FMA form, 12-bit data with dot2.
BATCH_SHAPES = {
    "f32": [(5, 4, 4, 0), (7, 4, 4, 0), (9, 4, 4, 0), (5, 3, 3, 0), (7, 3, 3, 0), (9, 3, 3, 0)],
    "u16": [(5, 4, 4, 0), (7, 3, 7, 1), (7, 4, 4, 0), (9, 4, 4, 0), (9, 5, 5, 0), (5, 3, 3, 0)],
}


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def clean_tuning(monkeypatch):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    monkeypatch.delenv("NRR_ARITH", raising=False)
    monkeypatch.delenv("NRR_TILE", raising=False)
    monkeypatch.delenv("NRR_CZ", raising=False)
    nrr.load()
    nrr.clear_tuning()
    yield
    nrr.clear_tuning()


def case(dtype, b, w, seed):
    dims = (2 * w + b + 6, 2 * w + b + 5, 2 * w + b + 4)
    p = synth.gen_random(seed, dims, dtype, smooth=1.2)
    h = b // 2
    rng = np.random.default_rng(seed)
    cs = [[rng.integers(h, dims[0] - h), rng.integers(h, dims[1] - h),
           rng.integers(h, dims[2] - h)] for _ in range(10)]
    cs += [[h, h, h], [dims[0] - 1 - h, dims[1] - 1 - h, dims[2] - 1 - h],
           [dims[0] // 2, h, dims[2] // 2], [h, dims[1] // 2, dims[2] - 1 - h],
           [h + w, h + w, h + w]]
    return p, dims, np.array(cs, dtype=np.int32)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
@pytest.mark.parametrize("b", [3, 5, 7, 9, 11, 13, 15])
def test_every_plain_shape(dtype, b):
    import torch

    dt = nrr.U16 if dtype == "u16" else nrr.F32
    shapes = nrr.match_shapes(dt, b, W)
    assert shapes, (dtype, b)
    forms = {s["arith"] for s in shapes}
    assert (dtype == "f32") == (forms == {1}), forms  # 12-bit data have dot2 (and mfma)
    p, dims, centers = case(dtype, b, W, 40 + b)
    ref, flt = to_dev(p.ref), to_dev(p.flt)
    cd = torch.from_numpy(centers).cuda()
    for sh in shapes:
        say("shape", dtype, b, sh)
        nrr.set_tuned_shape(dt, b, W, sh)
        plan = nrr.match_plan(dt, dims, b, W)
        assert all(plan[k] == sh[k] for k in KEYS + ("cz",)), (sh, plan)
        d, n, c = nrr.block_match(ref, flt, cd, b, W)
        torch.cuda.synchronize()
        check_match(p.ref, p.flt, centers, b, W, to_host(d), to_host(n), to_host(c),
                    "%s b%d %s" % (dtype, b, sh))
    nrr.clear_tuning()


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_every_batched_shape(dtype):
    import torch

    dt = nrr.U16 if dtype == "u16" else nrr.F32
    for b, rx, ry, pf in BATCH_SHAPES[dtype]:
        sh = {"arith": 0 if dtype == "u16" else 1, "rx": rx, "ry": ry, "nt": 256, "pf": pf,
              "cz": 0}
        p, dims, _ = case(dtype, b, W, 70 + b + rx)
        sets = [(b, W, b, 0.5), (b, W, max(1, b - 2), 0.3)]
        say("batched shape", dtype, sh, sets)
        nrr.set_tuned_shape(dt, b, W, sh)
        got = nrr.batch_shapes(dt, dims, sets)
        for g in got:
            assert all(g[k] == sh[k] for k in KEYS), (sh, g)
        plan = nrr.BatchPlan(to_dev(p.ref), to_dev(p.flt), sets, use_graph=False)
        plan.run()
        torch.cuda.synchronize()
        for i, (q, (c, d, n, cf)) in enumerate(zip(sets, plan.results())):
            bb, w, stride, frac = q
            c_o, _ = oracle.select(p.ref, bb, stride, frac)
            assert np.array_equal(to_host(c), c_o), (sh, i)
            check_match(p.ref, p.flt, c_o, bb, w, to_host(d), to_host(n), to_host(cf),
                        "batched %s %s set%d" % (dtype, sh, i))
        plan.close()
        nrr.clear_tuning()


def test_unknown_shape_is_rejected():
    with pytest.raises(nrr.NrrError):
        nrr.set_tuned_shape(nrr.F32, 7, W, {"arith": 1, "rx": 6, "ry": 6, "nt": 256, "pf": 0})
    with pytest.raises(nrr.NrrError):  # the matrix-core form serves 12-bit data only
        nrr.set_tuned_shape(nrr.F32, 7, W, {"arith": 2, "rx": 0, "ry": 0, "nt": 256, "pf": -1})


def test_statistics_for_a_window_then_another_plan(monkeypatch):
    """nrr_window_stats_for writes the plane-pair volume only when the planned
    search reads it (not for the matrix-core form); a prepared search whose
    plan has changed since (here to dot2) adds it itself."""
    import torch

    p = synth.gen_mri_u16(seed=3, dims=(64, 64, 48))
    b, w = 7, 5
    ref, flt = to_dev(p.ref), to_dev(p.flt)
    centers = nrr.select_blocks(ref, b, b, 0.3)
    assert nrr.match_plan(nrr.U16, p.dims, b, w)["arith"] == 2
    want = [to_host(t) for t in nrr.block_match(ref, flt, centers, b, w)]
    ws = nrr.window_stats(flt, b, window=w)  # no pair volume
    got = [to_host(t) for t in nrr.block_match(ref, flt, centers, b, w, workspace=ws,
                                               prepared=True)]
    for x, y in zip(want, got):
        assert np.array_equal(x, y)
    monkeypatch.setenv("NRR_ARITH", "dot2")
    assert nrr.match_plan(nrr.U16, p.dims, b, w)["arith"] == 0
    d, n, c = nrr.block_match(ref, flt, centers, b, w, workspace=ws, prepared=True)
    torch.cuda.synchronize()
    check_match(p.ref, p.flt, to_host(centers), b, w, to_host(d), to_host(n), to_host(c),
                "dot2 after statistics made for the matrix-core form")
    ws2 = nrr.window_stats(flt, b, window=w)  # planned for dot2: with the pair volume
    d2, n2, c2 = nrr.block_match(ref, flt, centers, b, w, workspace=ws2, prepared=True)
    assert np.array_equal(to_host(d2), to_host(d)) and np.array_equal(to_host(n2), to_host(n))
