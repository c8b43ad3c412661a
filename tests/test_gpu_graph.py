"""GPU: the hot path captured as a HIP graph (selection on one stream, window
statistics on a second, then the search) gives the eager results on every
replay, with other eager work on the device between the replays."""

import sys

import numpy as np
import pytest

import paper_2308_10868_amd as nrr
from paper_2308_10868_amd import synth
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_graph_replays_equal_eager(dtype):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    nrr.load()
    p = synth.gen_random(81, (48, 40, 36), dtype, smooth=1.2)
    q = synth.gen_random(82, (48, 40, 36), dtype, smooth=1.2)
    ref, flt = to_dev(p.ref), to_dev(p.flt)
    b, s, f, w = 5, 4, 0.3, 4
    dims = p.dims
    dt = nrr.U16 if dtype == "u16" else nrr.F32
    sel_ws = torch.empty(nrr.select_workspace_bytes(dims, b, s), dtype=torch.uint8, device="cuda")
    mat_ws = torch.empty(nrr.match_workspace_bytes(dt, dims, b), dtype=torch.uint8, device="cuda")
    say("graph eager", dtype)
    c_e = nrr.select_blocks(ref, b, s, f)
    d_e, n_e, cf_e = nrr.block_match(ref, flt, c_e, b, w)
    torch.cuda.synchronize()
    k = c_e.shape[0]
    disp = torch.empty((k, 3), dtype=torch.int32, device="cuda")
    ncc = torch.empty(k, dtype=torch.float32, device="cuda")
    conf = torch.empty(k, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    say("graph capture", dtype)
    with torch.cuda.graph(g):
        cap = torch.cuda.current_stream()
        side.wait_stream(cap)
        with torch.cuda.stream(side):
            nrr.window_stats(flt, b, workspace=mat_ws)
        c_g = nrr.select_blocks(ref, b, s, f, workspace=sel_ws)
        cap.wait_stream(side)
        nrr.block_match(ref, flt, c_g, b, w, workspace=mat_ws, out=(disp, ncc, conf),
                        prepared=True)
    torch.cuda.synchronize()
    other = (to_dev(q.ref), to_dev(q.flt))
    for rep in range(4):
        disp.zero_()
        ncc.zero_()
        conf.zero_()
        say("graph replay", dtype, rep)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(c_g), to_host(c_e)), rep
        assert np.array_equal(to_host(disp), to_host(d_e)), rep
        assert np.array_equal(to_host(ncc), to_host(n_e)), rep
        assert np.array_equal(to_host(conf), to_host(cf_e)), rep
        # eager work on other volumes between replays (it reuses no graph memory)
        c_o = nrr.select_blocks(other[0], b, s, f)
        nrr.block_match(other[0], other[1], c_o, b, w)
        torch.cuda.synchronize()
