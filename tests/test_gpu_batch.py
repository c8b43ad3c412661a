"""GPU: the batched parametric search and the tile tuner, through the C ABI.

Every set of a batch must give exactly what the plain calls (selection then
exhaustive search with that set's parameters) give, and hold the oracle's
parity rule; a graph-captured plan must reproduce the eager plan on every
replay.
"""

import sys

import numpy as np
import pytest

import oracle
import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import check_match, to_dev, to_host

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


@pytest.fixture(scope="module")
def c1():
    return synth.gen_translation_f32(seed=0)


@pytest.fixture(scope="module")
def u16_pair():
    # a 64 x 56 x 48 crop of the MRI-shaped pair (12-bit, anisotropic dims)
    p = synth.gen_mri_u16(seed=3, dims=(64, 56, 48))
    return p


def run_plan(torch, ref_d, flt_d, sets, use_graph):
    plan = nrr.BatchPlan(ref_d, flt_d, sets, use_graph=use_graph)
    plan.run()
    torch.cuda.synchronize()
    return plan


def plain(torch, ref_d, flt_d, q):
    b, w, stride, frac = q
    c = nrr.select_blocks(ref_d, b, stride, frac)
    d, n, cf = nrr.block_match(ref_d, flt_d, c, b, w)
    torch.cuda.synchronize()
    return to_host(c), to_host(d), to_host(n), to_host(cf)


def same_or_tied(dp, np_, db, nb):
    """Same displacement and NCC, or (differently rounded ranking keys) a
    displacement whose NCC is within 1e-5 of the other's."""
    for k in range(len(dp)):
        if np.array_equal(dp[k], db[k]):
            assert np.isclose(np_[k], nb[k], atol=1e-6, equal_nan=True), k
        else:
            assert abs(float(np_[k]) - float(nb[k])) < 1e-5, (k, dp[k], db[k])


SMALL_SETS = [(5, 2, 5, 0.05), (7, 3, 7, 0.1), (9, 2, 9, 0.25), (5, 3, 5, 0.1),
              (7, 2, 7, 0.5), (9, 3, 9, 0.001), (7, 1, 4, 0.05)]


def test_batch_f32_matches_oracle_per_set(torch_dev, c1):
    torch = torch_dev
    say("batch f32 vs oracle", SMALL_SETS)
    plan = run_plan(torch, to_dev(c1.ref), to_dev(c1.flt), SMALL_SETS, use_graph=False)
    for i, (q, (c, d, n, cf)) in enumerate(zip(SMALL_SETS, plan.results())):
        b, w, stride, frac = q
        c_o, _ = oracle.select(c1.ref, b, stride, frac)
        c_g = to_host(c)
        assert c_g.shape == c_o.shape and np.array_equal(c_g, c_o), (i, q)
        if len(c_o) == 0:
            continue
        check_match(c1.ref, c1.flt, c_o, b, w, to_host(d), to_host(n), to_host(cf),
                    label="set%d" % i)
    plan.close()


def test_batch_f32_config_sets_equal_plain_calls(torch_dev, c1):
    torch = torch_dev
    sets = synth.gen_param_sets(32, seed=1)
    say("batch f32 32 sets vs plain calls")
    ref_d, flt_d = to_dev(c1.ref), to_dev(c1.flt)
    plan = run_plan(torch, ref_d, flt_d, sets, use_graph=False)
    for i, (q, (c, d, n, cf)) in enumerate(zip(sets, plan.results())):
        cp, dp, np_, cfp = plain(torch, ref_d, flt_d, q)
        assert np.array_equal(to_host(c), cp), (i, q)
        same_or_tied(dp, np_, to_host(d), to_host(n))
        assert np.allclose(to_host(cf), np.maximum(to_host(n), 0), atol=0), i
    plan.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_f32_config_sets_match_oracle_per_set(torch_dev, c1, use_graph):
    """The 32 parameter sets of the batched workload (64^3 float pair, block
    {5,7,9}, window {5,8,12}, fraction {0.05..0.5}, stride = block), each set
    against the oracle: bit-exact selection, the parity rule for the search;
    eager and graph-replayed (the graph plan checked on two replays)."""
    torch = torch_dev
    sets = synth.gen_param_sets(32, seed=1)
    say("batch f32 32 sets vs oracle, graph" if use_graph else "batch f32 32 sets vs oracle")
    plan = run_plan(torch, to_dev(c1.ref), to_dev(c1.flt), sets, use_graph=use_graph)
    for rep in range(2 if use_graph else 1):
        if rep:
            plan.ncc.fill_(-7.0)  # stale values must not survive the replay
            plan.run()
            torch.cuda.synchronize()
        for i, (q, (c, d, n, cf)) in enumerate(zip(sets, plan.results())):
            b, w, stride, frac = q
            c_o, _ = oracle.select(c1.ref, b, stride, frac)
            assert np.array_equal(to_host(c), c_o), (rep, i, q)
            check_match(c1.ref, c1.flt, c_o, b, w, to_host(d), to_host(n), to_host(cf),
                        label="rep%d set%d" % (rep, i))
    plan.close()


def test_batch_u16_equals_plain_and_oracle(torch_dev, u16_pair, monkeypatch):
    torch = torch_dev
    monkeypatch.setenv("NRR_ARITH", "dot2")
    p = u16_pair
    sets = [(5, 3, 5, 0.1), (7, 4, 7, 0.25), (9, 2, 9, 0.5), (7, 2, 4, 0.05), (5, 5, 5, 0.02)]
    say("batch u16", sets)
    ref_d, flt_d = to_dev(p.ref), to_dev(p.flt)
    plan = run_plan(torch, ref_d, flt_d, sets, use_graph=False)
    for i, (q, (c, d, n, cf)) in enumerate(zip(sets, plan.results())):
        cp, dp, np_, cfp = plain(torch, ref_d, flt_d, q)
        assert np.array_equal(to_host(c), cp), (i, q)
        # 12-bit data: exact integer cross terms, so the same argmax and NCC
        assert np.array_equal(to_host(d), dp), (i, q)
        assert np.array_equal(to_host(n), np_), (i, q)
        b, w, stride, frac = q
        check_match(p.ref, p.flt, cp, b, w, to_host(d), to_host(n), to_host(cf), label="u%d" % i)
    plan.close()


def test_batch_graph_replays_match_eager(torch_dev, c1):
    torch = torch_dev
    sets = SMALL_SETS + [(5, 5, 5, 0.25), (9, 5, 9, 0.1)]
    ref_d, flt_d = to_dev(c1.ref), to_dev(c1.flt)
    say("batch graph replays")
    eager = run_plan(torch, ref_d, flt_d, sets, use_graph=False)
    want = [tuple(to_host(x).copy() for x in r) for r in eager.results()]
    eager.close()
    g = nrr.BatchPlan(ref_d, flt_d, sets, use_graph=True)
    for rep in range(3):
        g.ncc.fill_(-7.0)  # stale values must not survive a replay
        g.run()
        torch.cuda.synchronize()
        for i, r in enumerate(g.results()):
            got = [to_host(x) for x in r]
            for a, b in zip(got, want[i]):
                assert np.array_equal(a, b, equal_nan=True), (rep, i)
        # eager work of the program between replays
        c = nrr.select_blocks(ref_d, 7, 7, 0.2)
        nrr.block_match(ref_d, flt_d, c, 7, 3)
        torch.cuda.synchronize()
    g.close()


def test_batch_rejects_bad_sets(torch_dev, c1):
    ref_d, flt_d = to_dev(c1.ref), to_dev(c1.flt)
    with pytest.raises(nrr.NrrError):
        nrr.BatchPlan(ref_d, flt_d, [(6, 3, 6, 0.1)])      # even block
    with pytest.raises(nrr.NrrError):
        nrr.BatchPlan(ref_d, flt_d, [(5, 3, 1, 0.1)])      # 60^3 candidates > batched limit


def test_tuner_keeps_results_and_records_shape(torch_dev, u16_pair):
    torch = torch_dev
    p = u16_pair
    ref_d, flt_d = to_dev(p.ref), to_dev(p.flt)
    nrr.clear_tuning()
    c = nrr.select_blocks(ref_d, 7, 7, 0.3)
    d0, n0, f0 = nrr.block_match(ref_d, flt_d, c, 7, 6)
    torch.cuda.synchronize()
    say("tuner u16 b7 w6")
    shape, us = nrr.tune_match(ref_d, flt_d, c, 7, 6, reps=2)
    assert us > 0 and (shape["rx"] > 0 or shape["arith"] == 2)  # 2: matrix-core form
    assert nrr.tuned_shape(nrr.U16, 7, 6) == shape
    d1, n1, f1 = nrr.block_match(ref_d, flt_d, c, 7, 6)
    torch.cuda.synchronize()
    same_or_tied(to_host(d0), to_host(n0), to_host(d1), to_host(n1))
    check_match(p.ref, p.flt, to_host(c), 7, 6, to_host(d1), to_host(n1), to_host(f1), "tuned")
    nrr.clear_tuning()
    assert nrr.tuned_shape(nrr.U16, 7, 6) is None
