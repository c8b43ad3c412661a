"""GPU: nrr_select_and_window_stats (selection and window statistics side by
side: in one launch for 12-bit data and block edges up to 9 on grids the
one-workgroup select takes, else on two streams) gives exactly what the two
separate calls give, eagerly and replayed from a captured HIP graph."""

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


def defined_bytes(ws, dims, b, dtype, pairs):
    """The written parts of a match workspace: the table's records, then the
    plane-pair words when the plan reads them."""
    nx, ny, nz = dims
    ox, oy, oz = nx - b + 1, ny - b + 1, nz - b + 1
    rec = 8 if dtype == "u16" else 16
    parts = [ws[:ox * oy * oz * rec]]
    if pairs:
        table = ((ox * oy * oz + TILE_SLACK * (ox + 1)) * rec + 255) // 256 * 256
        parts.append(ws[table:table + 4 * nx * ny * nz])
    return parts


@pytest.mark.parametrize("kind,dims,b,w,frac,seed", [
    ("u16", (96, 80, 64), 7, 6, 0.25, 1),     # matrix-core plan: no pair words
    ("u16", (70, 66, 60), 11, 4, 0.3, 2),     # dot2 plan: pair words
    ("f32", (60, 52, 40), 5, 5, 0.2, 3),
    ("u16", (40, 40, 40), 5, 3, 1e-6, 4),     # K = 0: statistics only
    ("u16", (130, 70, 50), 3, 2, 0.2, 7),     # one launch for both, many statistics workgroups
    ("u16", (96, 96, 96), 3, 4, 0.37, 8),     # 32,768 candidates: the most the one launch takes
    ("u16", (12, 9, 8), 3, 2, 0.5, 9),        # one statistics wavefront, a ragged select
    ("u16", (80, 70, 60), 9, 5, 0.25, 10),    # the largest edge of the one launch
])
def test_combined_call_equals_separate_calls(kind, dims, b, w, frac, seed):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    p = synth.gen_mri_u16(seed=seed, dims=dims) if kind == "u16" else \
        synth.gen_random(seed, dims, "f32", smooth=1.0)
    ref, flt = to_dev(p.ref), to_dev(p.flt)
    dt = nrr.U16 if kind == "u16" else nrr.F32
    pairs = kind == "u16" and nrr.match_plan(dt, dims, b, w)["form"] == "dot2"
    say("select_and_window_stats", kind, dims, b, w, frac)
    want_c = nrr.select_blocks(ref, b, b, frac).clone()
    want_ws = nrr.window_stats(flt, b, window=w).clone()
    for _ in range(2):  # the second call reuses the library's stream and events
        got_c, got_ws = nrr.select_and_window_stats(ref, flt, b, b, frac, w)
        torch.cuda.synchronize()
        assert torch.equal(got_c, want_c)
        for g, e in zip(defined_bytes(got_ws, dims, b, kind, pairs),
                        defined_bytes(want_ws, dims, b, kind, pairs)):
            assert torch.equal(g, e)


def test_combined_call_against_the_oracle_and_box_sums():
    """The one-launch path checked directly: centres against oracle.select,
    the table's records against box sums of flt computed here."""
    import torch
    import oracle
    from tests.test_gpu_stats_table import check_u16_records

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    dims, b, w, frac = (120, 100, 70), 7, 6, 0.25
    p = synth.gen_mri_u16(seed=12, dims=dims)
    say("select_and_window_stats against the oracle", dims, b, w, frac)
    c, ws = nrr.select_and_window_stats(to_dev(p.ref), to_dev(p.flt), b, b, frac, w)
    torch.cuda.synchronize()
    exp, _ = oracle.select(p.ref, b, b, frac)
    assert np.array_equal(c.cpu().numpy(), exp)
    check_u16_records(ws.cpu().numpy(), p.flt, (b, b, b))


def test_combined_call_one_launch_then_pair_words(monkeypatch):
    """The dot2 form forced for a block edge the one-launch path takes: the
    pair words follow as a pass of their own."""
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    monkeypatch.setenv("NRR_ARITH", "dot2")
    dims, b, w, frac = (70, 60, 40), 5, 4, 0.3
    assert nrr.match_plan(nrr.U16, dims, b, w)["form"] == "dot2"
    p = synth.gen_mri_u16(seed=6, dims=dims)
    ref, flt = to_dev(p.ref), to_dev(p.flt)
    say("select_and_window_stats, dot2 forced", dims, b, w)
    want_c = nrr.select_blocks(ref, b, b, frac).clone()
    want_ws = nrr.window_stats(flt, b, window=w).clone()
    got_c, got_ws = nrr.select_and_window_stats(ref, flt, b, b, frac, w)
    torch.cuda.synchronize()
    assert torch.equal(got_c, want_c)
    for g, e in zip(defined_bytes(got_ws, dims, b, "u16", True),
                    defined_bytes(want_ws, dims, b, "u16", True)):
        assert torch.equal(g, e)


def test_combined_call_replayed_from_a_graph():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    dims, b, w, frac = (96, 80, 64), 7, 6, 0.25
    p = synth.gen_mri_u16(seed=5, dims=dims)
    ref, flt = to_dev(p.ref), to_dev(p.flt)
    sel_ws = torch.empty(nrr.select_workspace_bytes(dims, b, b), dtype=torch.uint8, device="cuda")
    mat_ws = torch.empty(nrr.match_workspace_bytes(nrr.U16, dims, b), dtype=torch.uint8,
                         device="cuda")
    say("select_and_window_stats under graph capture", dims, b, w)
    want_c, _ = nrr.select_and_window_stats(ref, flt, b, b, frac, w, sel_ws, mat_ws)
    want_c = want_c.clone()
    want_t = defined_bytes(mat_ws, dims, b, "u16", False)[0].clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        g_c, _ = nrr.select_and_window_stats(ref, flt, b, b, frac, w, sel_ws, mat_ws)
    torch.cuda.synchronize()
    for rep in range(3):
        mat_ws.fill_(7)  # eager work between the replays
        g_c.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(g_c, want_c), rep
        assert torch.equal(defined_bytes(mat_ws, dims, b, "u16", False)[0], want_t), rep
