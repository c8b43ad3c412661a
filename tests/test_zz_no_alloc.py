"""The allocation-free selection (nrr_select_blocks_static, scratch in a
fixed device array of the library) against nrr_select_blocks with a caller
workspace, through the C ABI: bit-identical centres and count on two calls in
a row, the second on a smaller input (the array keeps the first call's
contents), and a clear error for grids beyond the array."""

import ctypes
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


def call_static(lib, vol, dims, b, stride, frac, capacity):
    import torch

    centers = torch.full((max(capacity, 1), 3), -1, dtype=torch.int32, device=vol.device)
    k = ctypes.c_int64(-1)
    dt = nrr.U16 if vol.dtype == torch.uint16 else nrr.F32
    st = lib.nrr_select_blocks_static(
        ctypes.c_void_p(vol.data_ptr()), dt, (ctypes.c_int32 * 3)(*dims), b, stride, frac,
        ctypes.c_void_p(centers.data_ptr()), capacity, ctypes.byref(k),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, k.value, centers


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_selection_matches_workspace_selection(order):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    lib = nrr.load()
    mri = synth.gen_mri_u16(seed=0)
    tiny = synth.gen_translation_f32(seed=0)
    cases = [(mri.ref, 7, 7, 0.25, 5508), (tiny.ref, 7, 7, 0.2, 146)]
    for vol_h, b, stride, frac, k_want in cases:  # second call: smaller input
        say("static selection", vol_h.shape, b, stride, frac)
        vol = to_dev(vol_h)
        dims = (vol_h.shape[2], vol_h.shape[1], vol_h.shape[0])
        st, k, got = call_static(lib, vol, dims, b, stride, frac, k_want)
        torch.cuda.synchronize()
        assert st == 0, nrr.load().nrr_last_error()
        want = nrr.select_blocks(vol, b, stride, frac)
        torch.cuda.synchronize()
        assert k == k_want == want.shape[0]
        assert np.array_equal(to_host(got[:k]), to_host(want))


def test_static_selection_rejects_grids_beyond_the_array():
    import torch

    lib = nrr.load()
    dims = (512, 512, 256)  # stride 1, b 3: 66 million candidates
    vol = torch.zeros((1, 1, 1), dtype=torch.uint16, device="cuda")  # never read
    st, k, _ = call_static(lib, vol, dims, 3, 1, 0.1, 1)
    assert st == 4  # NRR_ERR_UNSUPPORTED, before any device work
    assert b"allocation-free" in lib.nrr_last_error()
