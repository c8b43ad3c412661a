"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/nrr.h declares, and the host-side helpers and argument
validation behave as documented (no call here reaches a kernel launch)."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2308_10868_amd as nrr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nrr.library_path()):
        pytest.skip("libnrr.so not built")
    return nrr.load()


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "nrr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nrr_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = _declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_strings(lib):
    assert lib.nrr_version() == 10000
    for s, text in [(0, b"ok"), (1, b"invalid argument"), (2, b"buffer too small"),
                    (3, b"HIP runtime error"), (4, b"unsupported")]:
        assert lib.nrr_status_string(s) == text


def test_grid_and_count_closed_forms(lib):
    import json

    g = json.load(open(os.path.join(ROOT, "tests", "golden", "selection_counts.json")))
    for case in g["cases"]:
        assert list(nrr.grid_shape(case["dims"], case["block"], case["stride"])) == case["grid"]
        assert nrr.select_count(case["dims"], case["block"], case["stride"], case["fraction"]) \
            == case["k"]


def test_count_rule_rounding(lib):
    # N = 10 (10x1x1 grid of 3-blocks along x with stride 1 on a 12x3x3 volume)
    dims = (12, 3, 3)
    assert nrr.grid_shape(dims, 3, 1) == (10, 1, 1)
    assert nrr.select_count(dims, 3, 1, 0.25) == 3   # 2.5 + 0.5 -> 3
    assert nrr.select_count(dims, 3, 1, 0.24) == 2   # 2.4 + 0.5 -> 2
    assert nrr.select_count(dims, 3, 1, 1.0) == 10
    assert nrr.select_count(dims, 3, 1, 0.01) == 0   # 0.1 + 0.5 -> 0


@pytest.mark.parametrize("block,stride,fraction,dims", [
    (4, 1, 0.5, (10, 10, 10)),   # even block
    (1, 1, 0.5, (10, 10, 10)),   # block < 3
    (3, 0, 0.5, (10, 10, 10)),   # stride < 1
    (3, 1, 0.0, (10, 10, 10)),   # fraction <= 0
    (3, 1, 1.5, (10, 10, 10)),   # fraction > 1
    (5, 1, 0.5, (10, 4, 10)),    # dims < block
])
def test_select_invalid_args(lib, block, stride, fraction, dims):
    k = ctypes.c_int64(-1)
    d = (ctypes.c_int32 * 3)(*dims)
    s = lib.nrr_select_blocks(None, 0, d, block, stride, fraction, None, 1000, ctypes.byref(k),
                              None, 0, None)
    assert s == 1
    assert len(lib.nrr_last_error()) > 0


def test_select_capacity_too_small_reports_k(lib):
    k = ctypes.c_int64(-1)
    d = (ctypes.c_int32 * 3)(64, 64, 64)
    s = lib.nrr_select_blocks(ctypes.c_void_p(1), 0, d, 7, 7, 0.2, ctypes.c_void_p(1), 100,
                              ctypes.byref(k), ctypes.c_void_p(1), 1 << 30, None)
    assert s == 2 and k.value == 146
    assert b"capacity" in lib.nrr_last_error()


def test_select_workspace_too_small(lib):
    k = ctypes.c_int64(-1)
    d = (ctypes.c_int32 * 3)(64, 64, 64)
    s = lib.nrr_select_blocks(ctypes.c_void_p(1), 0, d, 7, 7, 0.2, ctypes.c_void_p(1), 146,
                              ctypes.byref(k), ctypes.c_void_p(1), 16, None)
    assert s == 2 and b"workspace" in lib.nrr_last_error()


def test_select_k_zero_is_noop(lib):
    k = ctypes.c_int64(-1)
    d = (ctypes.c_int32 * 3)(12, 3, 3)
    s = lib.nrr_select_blocks(None, 0, d, 3, 1, 0.01, None, 0, ctypes.byref(k), None, 0, None)
    assert s == 0 and k.value == 0


def test_match_invalid_args(lib):
    d = (ctypes.c_int32 * 3)(32, 32, 32)
    P = ctypes.c_void_p(1)
    call = lambda **kw: lib.nrr_block_match(
        kw.get("ref", P), kw.get("flt", P), kw.get("dtype", 0), kw.get("dims", d),
        kw.get("centers", P), kw.get("n", 4), kw.get("block", 7), kw.get("window", 5), P, P, P,
        P, kw.get("ws", 1 << 30), None)
    assert call(block=6) == 1
    assert call(window=-1) == 1
    assert call(n=-1) == 1
    assert call(dtype=7) == 1
    assert call(centers=None) == 1
    assert call(dims=(ctypes.c_int32 * 3)(32, 5, 32)) == 1
    assert call(n=0, centers=None, ref=None) == 0       # n == 0: no-op
    assert call(ws=16) == 2                              # workspace too small
    assert call(block=17) == 4                           # not built


def test_match_workspace_size(lib):
    assert nrr.match_workspace_bytes(nrr.U16, (256, 256, 124), 7) >= 250 * 250 * 118 * 8
    assert nrr.match_workspace_bytes(nrr.F32, (64, 64, 64), 7) >= 58 ** 3 * 16
    assert lib.nrr_match_supported(0, 17, 3) == 4
    assert lib.nrr_match_supported(0, 8, 3) == 1
    assert lib.nrr_match_supported(0, 7, -1) == 1


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setenv("NRR_LIBRARY", str(tmp_path / "missing.so"))
    monkeypatch.setattr(nrr, "_lib", None)
    with pytest.raises(nrr.NrrError):
        nrr.load()


def test_batch_layout_offsets_and_errors(lib):
    import ctypes

    import paper_2308_10868_amd as nrr

    dims = (64, 64, 64)
    sets = [(5, 5, 5, 0.05), (7, 8, 7, 0.5), (9, 12, 9, 0.25), (9, 5, 9, 0.001)]
    offs, nbytes = nrr.batch_layout(nrr.F32, dims, sets)
    ks = [nrr.select_count(dims, b, s, f) for b, w, s, f in sets]
    assert offs == list(np.cumsum([0] + ks)) and nbytes > 0
    assert ks[-1] == 0  # an empty set is allowed
    with pytest.raises(nrr.NrrError) as e:
        nrr.batch_layout(nrr.F32, dims, [(5, 3, 1, 0.1)])  # 60^3 candidates
    assert e.value.status == 4
    for bad in [(6, 3, 6, 0.1), (5, -1, 5, 0.1), (5, 3, 0, 0.1), (5, 3, 5, 0.0), (99, 3, 5, 0.5)]:
        with pytest.raises(nrr.NrrError) as e:
            nrr.batch_layout(nrr.F32, dims, [bad])
        assert e.value.status == 1, bad
    assert nrr.batch_layout(nrr.U16, dims, []) [0] == [0]


def test_tuning_table_host_calls(lib):
    import paper_2308_10868_amd as nrr

    nrr.clear_tuning()
    assert nrr.tuned_shape(nrr.U16, 7, 10) is None


def test_param_sets_generator():
    from paper_2308_10868_amd import synth

    a = synth.gen_param_sets(32, seed=1)
    assert a == synth.gen_param_sets(32, seed=1) and len(a) == 32
    for b, w, s, f in a:
        assert b in (5, 7, 9) and w in (5, 8, 12) and s == b and f in (0.05, 0.1, 0.25, 0.5)
    assert len({(b, w, f) for b, w, s, f in a}) > 10


def test_request_footprint_closed_form(lib):
    import torch

    import paper_2308_10868_amd as nrr

    ref = torch.zeros((48, 56, 64), dtype=torch.uint16)
    flt = torch.zeros((48, 56, 64), dtype=torch.uint16)
    fp = nrr.request_footprint(ref, flt, 7, 7, 5, 0.25)
    up = lambda v: (v + 255) // 256 * 256
    dims = (64, 56, 48)
    k = nrr.select_count(dims, 7, 7, 0.25)
    vb = 64 * 56 * 48 * 2
    want = (2 * up(vb) + up(nrr.select_workspace_bytes(dims, 7, 7))
            + up(nrr.match_workspace_bytes(nrr.U16, dims, 7)) + 2 * up(12 * k) + 2 * up(4 * k))
    assert fp == want
    with pytest.raises(nrr.NrrError):
        nrr.request_footprint(ref, flt, 6, 7, 5, 0.25)


def test_select_ex_validation(lib):
    import ctypes

    buf = (ctypes.c_byte * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    dims = (ctypes.c_int32 * 3)(64, 64, 64)
    f = lib.nrr_select_blocks_ex
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_double, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                  ctypes.c_void_p]
    assert f(p, 0, dims, 7, 7, 0.2, None, 5, p, 1000, p, p, 1 << 30, None) == 1  # bad pattern
    assert f(p, 0, dims, 7, 7, 1.5, None, 6, p, 1000, p, p, 1 << 30, None) == 1  # bad fraction
    big = (ctypes.c_int32 * 3)(1302, 1302, 1302)  # block 3, stride 1: 2.2e9 candidates
    assert f(p, 0, big, 3, 1, 0.2, None, 6, p, 10 ** 6, p, p, 1 << 30, None) == 4
    assert f(p, 0, dims, 7, 7, 0.2, None, 6, p, 1, p, p, 1 << 30, None) == 2  # capacity
    # large grids (62^3 candidates) need the variants' extra workspace
    need = nrr.select_workspace_bytes((64, 64, 64), 3, 1)
    plain = nrr.select_workspace_bytes((64, 64, 64), 3, 3)
    assert need >= 62 ** 3 * (8 + 5)
    assert f(p, 0, dims, 3, 1, 0.2, None, 6, p, 10 ** 6, p, p, need - 256, None) == 2
    assert plain >= 21 ** 3 * 8  # 9,261 candidates: no extra


def test_structure_confidence_validation(lib):
    import ctypes

    buf = (ctypes.c_byte * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    dims = (ctypes.c_int32 * 3)(32, 32, 32)
    f = lib.nrr_structure_confidence
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert f(p, 0, dims, p, 4, 6, p, p, None) == 1      # even block
    assert f(p, 7, dims, p, 4, 7, p, p, None) == 1      # unknown dtype
    assert f(p, 0, dims, p, -1, 7, p, p, None) == 1     # negative count
    assert f(p, 0, dims, None, 4, 7, p, p, None) == 1   # null centres
    assert f(None, 0, dims, None, 0, 7, None, None, None) == 0  # n == 0: no-op


def test_aniso_validation(lib):
    import ctypes

    buf = (ctypes.c_byte * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    t3 = lambda *v: (ctypes.c_int32 * 3)(*v)  # noqa: E731
    dims = t3(40, 30, 20)
    ws = lib.nrr_aniso_workspace_bytes
    ws.restype = ctypes.c_int
    ws.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p]
    sb, mb = ctypes.c_size_t(), ctypes.c_size_t()
    assert ws(0, dims, t3(5, 3, 7), t3(5, 3, 7), ctypes.byref(sb), ctypes.byref(mb)) == 0
    # u16 search table: one 8-byte record per origin plus the tile slack rows
    ox, oy, oz = 40 - 5 + 1, 30 - 3 + 1, 20 - 7 + 1
    assert mb.value >= (ox * oy * oz) * 8 and mb.value % 256 == 0
    assert sb.value >= (8 * 10 * 2) * 8  # one 8-byte key per candidate
    assert ws(0, dims, t3(4, 3, 3), None, None, None) == 1     # even edge
    assert ws(0, dims, t3(17, 3, 3), None, None, None) == 4    # edge above 15
    assert ws(0, t3(40, 30, 9), t3(3, 3, 11), None, None, None) == 1  # larger than the volume
    m = lib.nrr_block_match_aniso
    m.restype = ctypes.c_int
    m.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_size_t, ctypes.c_void_p]
    assert m(p, p, 0, dims, p, 4, t3(5, 3, 3), t3(2, -1, 2), p, p, p, p, 1 << 30, None) == 1
    assert m(p, p, 0, dims, p, 4, t3(5, 3, 3), t3(2, 16, 2), p, p, p, p, 1 << 30, None) == 4
    assert m(p, p, 0, dims, p, 4, t3(5, 3, 3), t3(2, 1, 2), p, p, p, p, 16, None) == 2
    assert m(None, None, 0, dims, None, 0, t3(5, 3, 3), t3(2, 1, 2), None, None, None, None, 0,
             None) == 0  # n == 0: no-op
    sel = lib.nrr_select_blocks_aniso
    sel.restype = ctypes.c_int
    sel.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                    ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    k = ctypes.c_int64()
    assert sel(p, 0, dims, t3(5, 3, 7), t3(5, 3, 0), 0.5, p, 1000, ctypes.byref(k), p, 1 << 30,
               None) == 1  # zero stride
    assert sel(p, 0, dims, t3(5, 3, 7), t3(5, 3, 7), 0.5, p, 1, ctypes.byref(k), p, 1 << 30,
               None) == 2  # capacity
    assert k.value == int(0.5 + 8 * 10 * 2 * 0.5)


def test_select_count_aniso_matches_the_rule():
    import ctypes

    import oracle

    for dims, b, st, f in [((256, 256, 124), (7, 7, 3), (7, 7, 3), 0.25),
                           ((19, 15, 13), (3, 5, 1), (2, 3, 1), 0.5),
                           ((64, 64, 64), (9, 1, 5), (4, 1, 5), 0.07)]:
        k = nrr.select_count_aniso(dims, b, st, f)
        grid = [(dims[a] - b[a]) // st[a] + 1 for a in range(3)]
        assert k == oracle.select_count(grid[0] * grid[1] * grid[2], f)
        g = (ctypes.c_int32 * 3)()
        kk = ctypes.c_int64()
        assert nrr.load().nrr_select_count_aniso(nrr._dims3(dims), nrr._triple(b),
                                                 nrr._triple(st), f, g, ctypes.byref(kk)) == 0
        assert list(g) == grid and kk.value == k
    with pytest.raises(nrr.NrrError):
        nrr.select_count_aniso((10, 10, 10), (4, 3, 3), (1, 1, 1), 0.5)  # even edge


def test_select_and_window_stats_validation(lib):
    """nrr_select_and_window_stats checks its arguments before any launch:
    K is reported even when the call fails on capacity."""
    d = (ctypes.c_int32 * 3)(64, 64, 64)
    k = ctypes.c_int64(-1)
    P = ctypes.c_void_p
    call = lambda **kw: lib.nrr_select_and_window_stats(
        kw.get("ref", P(1)), kw.get("flt", P(1)), kw.get("dtype", 0), d, kw.get("block", 7),
        kw.get("stride", 7), kw.get("fraction", 0.2), kw.get("window", 3),
        kw.get("centers", P(1)), kw.get("capacity", 1000), kw.get("k_out", ctypes.byref(k)),
        kw.get("sws", P(1)), kw.get("sbytes", 1 << 30), kw.get("mws", P(1)),
        kw.get("mbytes", 1 << 30), None)
    assert call(k_out=None) == 1
    assert call(fraction=0.0) == 1 and call(fraction=1.5) == 1
    assert call(window=-1) == 1
    assert call(block=8) == 1            # even edge
    assert call(block=17) == 4           # not built
    assert call(dtype=7) == 1
    assert call(ref=None) == 1 and call(mws=None) == 1
    assert call(capacity=10) == 2        # K = floor(0.5 + 729 * 0.2) = 146
    assert k.value == 146
    assert call(sbytes=16) == 2 and b"selection workspace" in lib.nrr_last_error()
    assert call(mbytes=16) == 2 and b"match workspace" in lib.nrr_last_error()
