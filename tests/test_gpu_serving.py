"""GPU: the registration server (continuous batching over HIP streams).

Each served request must give exactly what it gives when served alone (and
what the plain calls give), whatever else is admitted beside it; admission
must respect the server's device memory.
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



def test_every_served_request_meets_the_oracle(torch_dev, mix):
    say("serving: all 8 requests of the mix vs oracle")
    out, _, _ = serve(mix, slots=4, device_bytes=1 << 30)
    for i, (q, (c, d, n, f)) in enumerate(zip(mix, out)):
        c_o, _ = oracle.select(q["pair"].ref, q["block"], q["stride"], q["fraction"])
        assert np.array_equal(c, c_o), i
        check_match(q["pair"].ref, q["pair"].flt, c, q["block"], q["window"], d, n, f,
                    "served %d" % i)


@pytest.mark.parametrize("size,block", [((192, 192, 96), 7), ((384, 384, 160), 9)])
def test_large_served_requests_with_window_15(torch_dev, size, block):
    """Clinical-size requests with the largest served window, beside a small
    one, against the oracle on 160 seeded blocks (a quarter near a face)."""
    torch = torch_dev
    w = 15
    p = synth.gen_blobs_u16(seed=1000, dims=size, peak=(4.0, 10.0))
    small = synth.gen_mri_u16(seed=30, dims=(64, 64, 64))
    say("serving: %s b%d W%d" % (size, block, w))
    srv = nrr.Server(device_bytes=4 << 30, slots=2)
    big = srv.submit(pinned(p.ref, torch), pinned(p.flt, torch), block, block, w, 0.2)
    other = srv.submit(pinned(small.ref, torch), pinned(small.flt, torch), 5, 5, 6, 0.2)
    big.wait()
    other.wait()
    srv.close()
    c, d, n, f = (to_host(t) for t in (big.centers, big.disp, big.ncc, big.conf))
    c_o, _ = oracle.select(p.ref, block, block, 0.2)
    assert np.array_equal(c, c_o)
    h = block // 2
    dims = np.array(size)
    near = np.flatnonzero(np.any((c - h - w < 0) | (c + h + w > dims - 1), axis=1))
    far = np.setdiff1d(np.arange(len(c)), near)
    rng = np.random.default_rng(5)
    idx = np.sort(np.concatenate([rng.choice(near, min(40, len(near)), replace=False),
                                  rng.choice(far, 120, replace=False)]))
    check_match(p.ref, p.flt, c[idx], block, w, d[idx], n[idx], f[idx],
                "served %s b%d W%d" % (size, block, w))


def test_resident_volumes_and_cached_selection(torch_dev, mix):
    """Requests naming resident volumes give the uploaded requests' results;
    a resident ref's selection is computed once per parameter set and then
    shared; finished records are released; a volume in use cannot go."""
    torch = torch_dev
    say("serving: resident volumes")
    q0, q1 = mix[0], mix[1]
    base, _, _ = serve([q0, q1, q0, q1], slots=1, device_bytes=1 << 30, one_at_a_time=True)
    srv = nrr.Server(device_bytes=1 << 30, slots=3)
    vols = {}
    for i, q in enumerate((q0, q1)):
        dev_ref = to_dev(q["pair"].ref)  # one from device memory, one from host memory
        vols[i] = (srv.add_volume(dev_ref if i == 0 else q["ref"]), srv.add_volume(q["flt"]))
    assert srv.stats()["volumes"] == 4
    jobs = []
    for rep in range(3):  # the same parameters again: the kept selection serves them
        for i, q in enumerate((q0, q1)):
            jobs.append((i, srv.submit(vols[i][0], vols[i][1], q["block"], q["stride"],
                                       q["window"], q["fraction"])))
    # a resident ref with an uploaded flt
    jobs.append((0, srv.submit(vols[0][0], q0["flt"], q0["block"], q0["stride"], q0["window"],
                               q0["fraction"])))
    for i, j in jobs:
        info = j.wait()
        assert info["state"] == 2
        got = tuple(to_host(t) for t in (j.centers, j.disp, j.ncc, j.conf))
        for x, y in zip(base[i], got):
            assert np.array_equal(x, y, equal_nan=True), i
    st = srv.stats()
    assert st["records"] == 0, st  # every waited request was released
    assert 0.0 < st["busy_ms"] <= st["wall_ms"], st
    # the library checks a named volume against the request's dtype and dims
    import ctypes

    outs = (torch.empty((4096, 3), dtype=torch.int32), torch.empty((4096, 3), dtype=torch.int32),
            torch.empty(4096), torch.empty(4096))
    r, _, _ = nrr._make_request(q1["ref"], q1["flt"], 5, 5, 3, 0.1, outs)
    t = ctypes.c_int64()
    assert nrr.load().nrr_server_submit_resident(srv._h, ctypes.byref(r), vols[0][0].id, 0,
                                                 ctypes.byref(t)) == 1
    assert nrr.load().nrr_server_submit_resident(srv._h, ctypes.byref(r), 0, 999,
                                                 ctypes.byref(t)) == 1
    for r, f in vols.values():
        r.remove()
        f.remove()
    assert srv.stats()["volumes"] == 0
    assert srv.stats()["used_bytes"] == 0
    srv.close()


def test_volume_in_use_cannot_be_removed(torch_dev, mix):
    torch = torch_dev
    say("serving: removing a volume in use")
    big = synth.gen_blobs_u16(seed=1001, dims=(192, 192, 96), peak=(4.0, 10.0))
    q = mix[0]
    srv = nrr.Server(device_bytes=1 << 30, slots=1)
    vol = srv.add_volume(q["ref"])
    # one slot: the request naming the volume queues behind a long one
    blocker = srv.submit(pinned(big.ref, torch), pinned(big.flt, torch), 7, 7, 15, 0.3)
    j = srv.submit(vol, q["flt"], q["block"], q["stride"], q["window"], q["fraction"])
    with pytest.raises(nrr.NrrError):
        vol.remove()
    blocker.wait()
    j.wait()
    vol.remove()
    assert srv.stats()["used_bytes"] == 0
    srv.close()


def test_admission_respects_device_memory(torch_dev, mix):
    fp = [nrr.request_footprint(q["ref"], q["flt"], q["block"], q["stride"], q["window"],
                                q["fraction"]) for q in mix]
    budget = int(sorted(fp)[-1] + sorted(fp)[-2] + 4096)  # room for about two requests
    say("serving: memory-bound admission, budget", budget)
    out, infos, st = serve(mix, slots=6, device_bytes=budget)
    assert st["completed"] == len(mix) and st["pending"] == 0
    assert st["peak_bytes"] <= budget
    # most requests that fit the budget at once: the smallest footprints first
    fit, used = 0, 0
    for b in sorted(fp):
        if used + b > budget:
            break
        fit, used = fit + 1, used + b
    assert fit < len(mix)  # the budget does bound admission
    assert 1 <= st["max_running"] <= fit, st
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
