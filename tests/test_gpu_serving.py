"""GPU: the registration server (continuous batching over HIP streams).

Each served request must give exactly what it gives when served alone (and
what the plain calls give), whatever else is admitted beside it; admission
must respect the server's device memory.
"""

import sys

import numpy as np
import pytest

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
    nrr.clear_tuning()
    return torch


def pinned(a, torch):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        t = torch.from_numpy(a.view(np.int16)).view(torch.uint16)
    else:
        t = torch.from_numpy(a)
    return t.pin_memory()


@pytest.fixture(scope="module")
def mix(torch_dev):
    """Eight requests of four sizes and mixed parameters (12-bit pairs)."""
    torch = torch_dev
    sizes = [(64, 64, 64), (96, 80, 64), (112, 96, 72), (80, 72, 56)]
    reqs = []
    for i in range(8):
        p = synth.gen_mri_u16(seed=20 + i, dims=sizes[i % 4])
        b = (5, 7, 9)[i % 3]
        reqs.append(dict(ref=pinned(p.ref, torch), flt=pinned(p.flt, torch), block=b, stride=b,
                         window=(3, 5, 6, 4)[i % 4], fraction=(0.1, 0.2, 0.3)[i % 3], pair=p))
    return reqs


def serve(reqs, slots, device_bytes, one_at_a_time=False):
    srv = nrr.Server(device_bytes=device_bytes, slots=slots)
    jobs, infos = [], []
    for q in reqs:
        j = srv.submit(q["ref"], q["flt"], q["block"], q["stride"], q["window"], q["fraction"])
        if one_at_a_time:
            infos.append(j.wait())
        jobs.append(j)
    if not one_at_a_time:
        infos = [j.wait() for j in jobs]
    stats = srv.stats()
    srv.close()
    out = [tuple(to_host(t).copy() for t in (j.centers, j.disp, j.ncc, j.conf)) for j in jobs]
    return out, infos, stats


def test_served_results_same_alone_and_in_the_mix(torch_dev, mix):
    say("serving: alone vs mixed, 8 requests")
    alone, _, st1 = serve(mix, slots=1, device_bytes=1 << 30, one_at_a_time=True)
    mixed, infos, st4 = serve(mix, slots=4, device_bytes=1 << 30)
    assert st4["max_running"] >= 2, st4  # requests really overlapped
    for i, (a, m) in enumerate(zip(alone, mixed)):
        for x, y in zip(a, m):
            assert np.array_equal(x, y, equal_nan=True), i
        assert infos[i]["state"] == 2 and infos[i]["k"] == len(a[0])


def test_served_equals_plain_calls_and_oracle(torch_dev, mix):
    torch = torch_dev
    say("serving vs plain calls and oracle")
    out, _, _ = serve(mix[:3], slots=3, device_bytes=1 << 30)
    for q, (c, d, n, f) in zip(mix[:3], out):
        ref_d, flt_d = to_dev(q["pair"].ref), to_dev(q["pair"].flt)
        cp = nrr.select_blocks(ref_d, q["block"], q["stride"], q["fraction"])
        dp, np_, fp = nrr.block_match(ref_d, flt_d, cp, q["block"], q["window"])
        torch.cuda.synchronize()
        assert np.array_equal(c, to_host(cp))
        assert np.array_equal(d, to_host(dp)) and np.array_equal(n, to_host(np_))
    q, (c, d, n, f) = mix[0], out[0]
    check_match(q["pair"].ref, q["pair"].flt, c, q["block"], q["window"], d, n, f, "served")


def test_admission_respects_device_memory(torch_dev, mix):
    fp = [nrr.request_footprint(q["ref"], q["flt"], q["block"], q["stride"], q["window"],
                                q["fraction"]) for q in mix]
    budget = int(sorted(fp)[-1] + sorted(fp)[-2] + 4096)  # room for about two requests
    say("serving: memory-bound admission, budget", budget)
    out, infos, st = serve(mix, slots=6, device_bytes=budget)
    assert st["completed"] == len(mix) and st["pending"] == 0
    assert st["peak_bytes"] <= budget
    assert 1 <= st["max_running"] <= 3, st
    alone, _, _ = serve(mix, slots=1, device_bytes=1 << 30, one_at_a_time=True)
    for a, m in zip(alone, out):
        for x, y in zip(a, m):
            assert np.array_equal(x, y, equal_nan=True)


def test_oversize_request_is_rejected(torch_dev, mix):
    q = mix[2]
    srv = nrr.Server(device_bytes=1 << 20, slots=2)
    with pytest.raises(nrr.NrrError) as e:
        srv.submit(q["ref"], q["flt"], q["block"], q["stride"], q["window"], q["fraction"])
    assert e.value.status == 4
    srv.close()
