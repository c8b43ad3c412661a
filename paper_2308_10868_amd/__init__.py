"""GPU block matching for physics-based non-rigid registration (MI355X).

Thin Python binding over ``libnrr.so`` (C ABI in ``include/nrr.h``): argument
marshalling only -- every step of selection and matching runs in the HIP
kernels of the library.  PyTorch provides device memory and the current HIP
stream.  Importing this package does not load the library; the first compute
call does, and raises ``NrrError`` if it is missing or no GPU is visible.

    import torch, paper_2308_10868_amd as nrr
    centers = nrr.select_blocks(ref, block=7, stride=7, fraction=0.25)
    disp, ncc, conf = nrr.block_match(ref, flt, centers, block=7, window=10)

Volumes are ``[nz, ny, nx]`` tensors (uint16 with 12-bit values, or
float32) on a HIP device; centres and displacements are ``(x, y, z)`` int32.
"""

from __future__ import annotations

import ctypes
import os

__all__ = [
    "NrrError",
    "library_path",
    "load",
    "grid_shape",
    "select_count",
    "select_workspace_bytes",
    "match_workspace_bytes",
    "match_supported",
    "select_blocks",
    "select_blocks_ex",
    "block_match",
    "window_stats",
    "structure_confidence",
    "aniso_workspace_bytes",
    "select_blocks_aniso",
    "block_match_aniso",
    "window_stats_aniso",
    "tune_match",
    "tuned_shape",
    "clear_tuning",
    "ParamSet",
    "batch_layout",
    "BatchPlan",
    "Server",
    "request_footprint",
    "U16",
    "F32",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
U16, F32 = 0, 1
_STATUS = {0: "NRR_OK", 1: "NRR_ERR_INVALID_ARG", 2: "NRR_ERR_BUFFER_TOO_SMALL", 3: "NRR_ERR_HIP",
           4: "NRR_ERR_UNSUPPORTED"}
_lib = None


class TileShape(ctypes.Structure):
    _fields_ = [("arith", ctypes.c_int32), ("rx", ctypes.c_int32), ("ry", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("pf", ctypes.c_int32), ("cz", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ParamSet(ctypes.Structure):
    """One parameter set of the batched search (block, window, stride, fraction)."""
    _fields_ = [("block", ctypes.c_int32), ("window", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("fraction", ctypes.c_double)]


class _Request(ctypes.Structure):
    _fields_ = [("ref", ctypes.c_void_p), ("flt", ctypes.c_void_p), ("dtype", ctypes.c_int),
                ("dims", ctypes.c_int32 * 3), ("block", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("window", ctypes.c_int32), ("fraction", ctypes.c_double),
                ("centers", ctypes.c_void_p), ("disp", ctypes.c_void_p), ("ncc", ctypes.c_void_p),
                ("conf", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("k", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("queued_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _ServerInfo(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("used_bytes", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("max_running", ctypes.c_int32), ("submitted", ctypes.c_int64),
                ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("pending", ctypes.c_int64), ("wall_ms", ctypes.c_double),
                ("busy_ms", ctypes.c_double), ("volumes", ctypes.c_int64),
                ("records", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NrrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


def library_path() -> str:
    return os.environ.get("NRR_LIBRARY") or os.path.join(_HERE, "libnrr.so")


def load():
    """Load libnrr.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise NrrError(3, "libnrr.so not built at %s (run __graft_entry__.build())" % path)
    lib = ctypes.CDLL(path)
    P, I32, I64, F64, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                            ctypes.c_size_t)
    st = ctypes.c_int
    sig = {
        "nrr_grid_shape": (st, [P, I32, I32, P]),
        "nrr_select_count": (st, [P, I32, I32, F64, P]),
        "nrr_select_workspace_bytes": (st, [P, I32, I32, P]),
        "nrr_match_workspace_bytes": (st, [ctypes.c_int, P, I32, P]),
        "nrr_match_supported": (st, [ctypes.c_int, I32, I32]),
        "nrr_match_plan": (st, [ctypes.c_int, P, I32, I32, P]),
        "nrr_block_match_surface": (st, [P, P, ctypes.c_int, P, P, I64, I32, I32, I32, P, P, P,
                                         P, P, SZ, P]),
        "nrr_match_shapes": (st, [ctypes.c_int, I32, I32, P, I32, P]),
        "nrr_set_tuned_shape": (st, [ctypes.c_int, I32, I32, P]),
        "nrr_batch_shapes": (st, [ctypes.c_int, P, P, I32, P]),
        "nrr_select_blocks": (st, [P, ctypes.c_int, P, I32, I32, F64, P, I64, P, P, SZ, P]),
        "nrr_block_match": (st, [P, P, ctypes.c_int, P, P, I64, I32, I32, P, P, P, P, SZ, P]),
        "nrr_select_blocks_ex": (st, [P, ctypes.c_int, P, I32, I32, F64, P, I32, P, I64, P, P, SZ,
                                      P]),
        "nrr_select_blocks_static": (st, [P, ctypes.c_int, P, I32, I32, F64, P, I64, P, P]),
        "nrr_window_stats": (st, [P, ctypes.c_int, P, I32, P, SZ, P]),
        "nrr_window_stats_for": (st, [P, ctypes.c_int, P, I32, I32, P, SZ, P]),
        "nrr_select_and_window_stats": (st, [P, P, ctypes.c_int, P, I32, I32, F64, I32, P, I64,
                                             P, P, SZ, P, SZ, P]),
        "nrr_check_volume": (st, [P, ctypes.c_int, P, P, P]),
        "nrr_block_match_prepared": (st, [P, P, ctypes.c_int, P, P, I64, I32, I32, P, P, P, P, SZ,
                                          P]),
        "nrr_aniso_workspace_bytes": (st, [ctypes.c_int, P, P, P, P, P]),
        "nrr_select_blocks_aniso": (st, [P, ctypes.c_int, P, P, P, ctypes.c_double, P, I64, P, P,
                                         ctypes.c_size_t, P]),
        "nrr_select_count_aniso": (st, [P, P, P, F64, P, P]),
        "nrr_select_blocks_aniso_ex": (st, [P, ctypes.c_int, P, P, P, F64, P, I32, P, I64, P, P,
                                            SZ, P]),
        "nrr_block_match_aniso": (st, [P, P, ctypes.c_int, P, P, I64, P, P, P, P, P, P,
                                       ctypes.c_size_t, P]),
        "nrr_block_match_aniso_prepared": (st, [P, P, ctypes.c_int, P, P, I64, P, P, P, P, P, P,
                                                ctypes.c_size_t, P]),
        "nrr_window_stats_aniso": (st, [P, ctypes.c_int, P, P, P, ctypes.c_size_t, P]),
        "nrr_structure_confidence": (st, [P, ctypes.c_int, P, P, I64, I32, P, P, P]),
        "nrr_tune_match": (st, [P, P, ctypes.c_int, P, P, I64, I32, I32, P, P, P, P, SZ, I32, P, P,
                                P]),
        "nrr_tuned_shape": (st, [ctypes.c_int, I32, I32, P]),
        "nrr_clear_tuning": (st, []),
        "nrr_batch_layout": (st, [ctypes.c_int, P, P, I32, P, P]),
        "nrr_batch_plan_create": (st, [P, P, ctypes.c_int, P, P, I32, P, P, P, P, P, SZ, I32, P,
                                       P]),
        "nrr_batch_plan_run": (st, [P, P]),
        "nrr_batch_plan_destroy": (st, [P]),
        "nrr_request_footprint": (st, [P, P]),
        "nrr_server_create": (st, [SZ, I32, P]),
        "nrr_server_submit": (st, [P, P, P]),
        "nrr_server_submit_resident": (st, [P, P, I64, I64, P]),
        "nrr_server_add_volume": (st, [P, P, I32, P, P]),
        "nrr_server_remove_volume": (st, [P, I64]),
        "nrr_server_release": (st, [P, I64]),
        "nrr_server_poll": (st, [P, I64, P]),
        "nrr_server_wait": (st, [P, I64, P]),
        "nrr_server_stats": (st, [P, P]),
        "nrr_server_destroy": (st, [P]),
        "nrr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "nrr_last_error": (ctypes.c_char_p, []),
        "nrr_version": (I32, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise NrrError(status, load().nrr_last_error().decode())


def _dims3(dims) -> ctypes.Array:
    return (ctypes.c_int32 * 3)(*[int(v) for v in dims])


def grid_shape(dims, block: int, stride: int):
    g = (ctypes.c_int32 * 3)()
    _check(load().nrr_grid_shape(_dims3(dims), block, stride, g))
    return tuple(g)


def select_count(dims, block: int, stride: int, fraction: float) -> int:
    k = ctypes.c_int64()
    _check(load().nrr_select_count(_dims3(dims), block, stride, float(fraction), ctypes.byref(k)))
    return k.value


def select_workspace_bytes(dims, block: int, stride: int) -> int:
    b = ctypes.c_size_t()
    _check(load().nrr_select_workspace_bytes(_dims3(dims), block, stride, ctypes.byref(b)))
    return b.value


def match_workspace_bytes(dtype: int, dims, block: int) -> int:
    b = ctypes.c_size_t()
    _check(load().nrr_match_workspace_bytes(dtype, _dims3(dims), block, ctypes.byref(b)))
    return b.value


def match_supported(dtype: int, block: int, window: int) -> bool:
    return load().nrr_match_supported(dtype, block, window) == 0


# --------------------------------------------------------------- tensors

ARITH_NAMES = {0: "dot2", 1: "fma", 2: "mfma"}


def match_plan(dtype: int, dims, block: int, window: int) -> dict:
    """The shape nrr_block_match would launch now (environment overrides and
    tuned shapes included), as a dict with 'form' = 'dot2', 'fma' or 'mfma'."""
    out = TileShape()
    _check(load().nrr_match_plan(dtype, _dims3(dims), block, window, ctypes.byref(out)))
    d = out.as_dict()
    d["form"] = ARITH_NAMES.get(d["arith"], str(d["arith"]))
    return d


def match_shapes(dtype: int, block: int, window: int) -> list:
    """The compiled shapes the tuner times for (dtype, block, window)."""
    lib = load()
    arr = (TileShape * 64)()
    n = ctypes.c_int32()
    _check(lib.nrr_match_shapes(dtype, block, window, arr, 64, ctypes.byref(n)))
    return [arr[i].as_dict() for i in range(min(n.value, 64))]


def set_tuned_shape(dtype: int, block: int, window: int, shape: dict):
    """Pin a compiled shape for later searches of (dtype, block, window)."""
    t = TileShape(*[int(shape.get(k, 0)) for k, _ in TileShape._fields_])
    _check(load().nrr_set_tuned_shape(dtype, block, window, ctypes.byref(t)))


def _torch():
    import torch

    return torch


def _vol_info(t):
    torch = _torch()
    if not t.is_cuda:
        raise NrrError(1, "volumes must be device tensors")
    if t.dim() != 3 or not t.is_contiguous():
        raise NrrError(1, "volumes must be contiguous [nz, ny, nx] tensors")
    if t.dtype == torch.uint16:
        dt = U16
    elif t.dtype == torch.float32:
        dt = F32
    else:
        raise NrrError(1, "volume dtype must be uint16 or float32, got %s" % t.dtype)
    nz, ny, nx = t.shape
    return dt, (nx, ny, nz)


def _stream(t):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _workspace(nbytes: int, device, workspace):
    torch = _torch()
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise NrrError(2, "workspace of %d bytes < %d" % (workspace.numel(), nbytes))
        return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def select_blocks(vol, block: int, stride: int, fraction: float, workspace=None):
    """Variance-ranked selection: int32 [K, 3] centres (x, y, z) in ascending
    grid index, on vol's device (asynchronous on the current stream)."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(vol)
    k = select_count(dims, block, stride, fraction)
    out = torch.empty((max(k, 1), 3), dtype=torch.int32, device=vol.device)
    ws = _workspace(select_workspace_bytes(dims, block, stride), vol.device, workspace)
    kout = ctypes.c_int64()
    _check(lib.nrr_select_blocks(ctypes.c_void_p(vol.data_ptr()), dt, _dims3(dims), block, stride,
                                 float(fraction), ctypes.c_void_p(out.data_ptr()), out.shape[0],
                                 ctypes.byref(kout), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream(vol)))
    return out[:kout.value]


def select_and_window_stats(ref, flt, block: int, stride: int, fraction: float, window: int,
                            select_workspace=None, match_workspace=None):
    """select_blocks(ref, ...) and window_stats(flt, block, window=window) in
    one call, side by side on two streams (nrr_select_and_window_stats).
    Returns (centres int32 [K, 3], the match workspace) on the current
    stream, which has joined the statistics' stream."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(ref)
    dt2, dims2 = _vol_info(flt)
    if dt != dt2 or dims != dims2 or ref.device != flt.device:
        raise NrrError(1, "ref and flt must share dtype, shape and device")
    k = select_count(dims, block, stride, fraction)
    out = torch.empty((max(k, 1), 3), dtype=torch.int32, device=ref.device)
    sws = _workspace(select_workspace_bytes(dims, block, stride), ref.device, select_workspace)
    mws = _workspace(match_workspace_bytes(dt, dims, block), ref.device, match_workspace)
    kout = ctypes.c_int64()
    _check(lib.nrr_select_and_window_stats(
        ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(flt.data_ptr()), dt, _dims3(dims),
        block, stride, float(fraction), int(window), ctypes.c_void_p(out.data_ptr()),
        out.shape[0], ctypes.byref(kout), ctypes.c_void_p(sws.data_ptr()), sws.numel(),
        ctypes.c_void_p(mws.data_ptr()), mws.numel(), _stream(ref)))
    return out[:kout.value], mws


def select_blocks_ex(vol, block: int, stride: int, fraction: float, mask=None,
                     connectivity: int = 0, workspace=None):
    """Selection restricted to a mask (uint8 device tensor like `vol`; nonzero
    = candidate centre allowed) with a connectivity pattern (0, 6, 18, 26).
    Returns int32 [k, 3] centres in ascending grid index.  Synchronises the
    stream to read k."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(vol)
    kmax = select_count(dims, block, stride, fraction)
    out = torch.empty((max(kmax, 1), 3), dtype=torch.int32, device=vol.device)
    kd = torch.zeros(1, dtype=torch.int64, device=vol.device)
    ws = _workspace(select_workspace_bytes(dims, block, stride), vol.device, workspace)
    mp = None
    if mask is not None:
        if mask.dtype != torch.uint8 or tuple(mask.shape) != tuple(vol.shape) \
                or not mask.is_contiguous() or mask.device != vol.device:
            raise NrrError(1, "mask must be a contiguous uint8 tensor shaped like vol")
        mp = ctypes.c_void_p(mask.data_ptr())
    _check(lib.nrr_select_blocks_ex(ctypes.c_void_p(vol.data_ptr()), dt, _dims3(dims), block,
                                    stride, float(fraction), mp, int(connectivity),
                                    ctypes.c_void_p(out.data_ptr()), out.shape[0],
                                    ctypes.c_void_p(kd.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                    ws.numel(), _stream(vol)))
    return out[:int(kd.item())]


def check_volume(vol) -> int:
    """Number of voxels of a device volume outside its dtype's contract
    (12-bit data above 4095, float data not finite); synchronises the
    stream.  The other calls do not check: such data give undefined
    results."""
    torch = _torch()
    dt, dims = _vol_info(vol)
    bad = torch.zeros(1, dtype=torch.int64, device=vol.device)
    _check(load().nrr_check_volume(ctypes.c_void_p(vol.data_ptr()), dt, _dims3(dims),
                                   ctypes.c_void_p(bad.data_ptr()), _stream(vol)))
    return int(bad.item())


def window_stats(flt, block: int, workspace=None, window=None):
    """Per-voxel window statistics of `flt` for this block size (the table
    block_match(..., prepared=True) reads).  With `window`, only what the
    planned search for that window reads (nrr_window_stats_for).  Returns the
    workspace tensor."""
    lib = load()
    dt, dims = _vol_info(flt)
    ws = _workspace(match_workspace_bytes(dt, dims, block), flt.device, workspace)
    if window is None:
        _check(lib.nrr_window_stats(ctypes.c_void_p(flt.data_ptr()), dt, _dims3(dims), block,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(flt)))
    else:
        _check(lib.nrr_window_stats_for(ctypes.c_void_p(flt.data_ptr()), dt, _dims3(dims), block,
                                        int(window), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream(flt)))
    return ws


def block_match(ref, flt, centers, block: int, window: int, workspace=None, out=None,
                prepared: bool = False):
    """Exhaustive NCC search; returns (disp int32 [n,3], ncc f32 [n], conf f32 [n]).

    With ``prepared=True`` the window-statistics pass is skipped and
    ``workspace`` must be the table ``window_stats(flt, block)`` returned."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(ref)
    dt2, dims2 = _vol_info(flt)
    if dt != dt2 or dims != dims2 or ref.device != flt.device:
        raise NrrError(1, "ref and flt must share dtype, shape and device")
    if centers.dtype != torch.int32 or centers.dim() != 2 or centers.shape[1] != 3 \
            or not centers.is_contiguous() or centers.device != ref.device:
        raise NrrError(1, "centers must be a contiguous int32 [n, 3] tensor on ref's device")
    n = centers.shape[0]
    if out is None:
        disp = torch.empty((n, 3), dtype=torch.int32, device=ref.device)
        ncc = torch.empty(n, dtype=torch.float32, device=ref.device)
        conf = torch.empty(n, dtype=torch.float32, device=ref.device)
    else:
        disp, ncc, conf = out
    if n == 0:
        return disp, ncc, conf
    if prepared and workspace is None:
        raise NrrError(1, "prepared=True needs the workspace window_stats() filled")
    ws = _workspace(match_workspace_bytes(dt, dims, block), ref.device, workspace)
    fn = lib.nrr_block_match_prepared if prepared else lib.nrr_block_match
    _check(fn(ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(flt.data_ptr()),
                               dt, _dims3(dims), ctypes.c_void_p(centers.data_ptr()), n, block,
                               window, ctypes.c_void_p(disp.data_ptr()),
                               ctypes.c_void_p(ncc.data_ptr()), ctypes.c_void_p(conf.data_ptr()),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(ref)))
    return disp, ncc, conf


def block_match_surface(ref, flt, centers, block: int, window: int, arith: str = "default"):
    """The search plus the ranking NCC of every valid displacement:
    (disp, ncc, conf, surface[n, 2W+1, 2W+1, 2W+1] indexed [dz][dy][dx], NaN
    where a displacement is invalid).  arith: 'default', 'dot2', 'fma' or
    'mfma'.  A diagnostic of the ranking arithmetic."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(ref)
    n = centers.shape[0]
    side = 2 * window + 1
    dev = ref.device
    disp = torch.empty((max(n, 1), 3), dtype=torch.int32, device=dev)
    ncc = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    conf = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    surf = torch.empty((max(n, 1), side, side, side), dtype=torch.float32, device=dev)
    ws = _workspace(match_workspace_bytes(dt, dims, block), dev, None)
    code = {"default": -1, "dot2": 0, "fma": 1, "mfma": 2}[arith]
    _check(lib.nrr_block_match_surface(
        ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(flt.data_ptr()), dt, _dims3(dims),
        ctypes.c_void_p(centers.data_ptr()), n, block, window, code,
        ctypes.c_void_p(disp.data_ptr()), ctypes.c_void_p(ncc.data_ptr()),
        ctypes.c_void_p(conf.data_ptr()), ctypes.c_void_p(surf.data_ptr()),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(ref)))
    return disp[:n], ncc[:n], conf[:n], surf[:n]


def _triple(v) -> ctypes.Array:
    t = (ctypes.c_int32 * 3)()
    vals = [int(v)] * 3 if isinstance(v, int) else [int(x) for x in v]
    if len(vals) != 3:
        raise NrrError(1, "per-axis sizes are (x, y, z) triples")
    for i in range(3):
        t[i] = vals[i]
    return t


def aniso_workspace_bytes(dtype, dims, block, stride=None):
    """(selection bytes, search bytes) for per-axis block edges and strides."""
    lib = load()
    sb, mb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.nrr_aniso_workspace_bytes(dtype, _dims3(dims), _triple(block),
                                         None if stride is None else _triple(stride),
                                         ctypes.byref(sb), ctypes.byref(mb)))
    return sb.value, mb.value


def select_count_aniso(dims, block, stride, fraction: float) -> int:
    """K for per-axis sizes (the library's count rule over its grid)."""
    k = ctypes.c_int64()
    _check(load().nrr_select_count_aniso(_dims3(dims), _triple(block), _triple(stride),
                                         float(fraction), None, ctypes.byref(k)))
    return k.value


def select_blocks_aniso(vol, block, stride, fraction: float, workspace=None):
    """Variance-ranked selection with per-axis block edges and strides
    ((x, y, z) triples): int32 [K, 3] centres in ascending grid index."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(vol)
    b3, s3 = _triple(block), _triple(stride)
    kmax = max(select_count_aniso(dims, block, stride, fraction), 1)
    out = torch.empty((kmax, 3), dtype=torch.int32, device=vol.device)
    sel_bytes, _ = aniso_workspace_bytes(dt, dims, block, stride)
    ws = _workspace(sel_bytes, vol.device, workspace)
    kout = ctypes.c_int64()
    _check(lib.nrr_select_blocks_aniso(ctypes.c_void_p(vol.data_ptr()), dt, _dims3(dims), b3, s3,
                                       float(fraction), ctypes.c_void_p(out.data_ptr()),
                                       out.shape[0], ctypes.byref(kout),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(vol)))
    return out[:kout.value]


def select_blocks_aniso_ex(vol, block, stride, fraction: float, mask=None,
                           connectivity: int = 0, workspace=None):
    """select_blocks_ex with per-axis block edges and strides ((x, y, z)
    triples).  Synchronises the stream to read k."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(vol)
    kmax = max(select_count_aniso(dims, block, stride, fraction), 1)
    out = torch.empty((kmax, 3), dtype=torch.int32, device=vol.device)
    kd = torch.zeros(1, dtype=torch.int64, device=vol.device)
    sel_bytes, _ = aniso_workspace_bytes(dt, dims, block, stride)
    ws = _workspace(sel_bytes, vol.device, workspace)
    mp = None
    if mask is not None:
        if mask.dtype != torch.uint8 or tuple(mask.shape) != tuple(vol.shape) \
                or not mask.is_contiguous() or mask.device != vol.device:
            raise NrrError(1, "mask must be a contiguous uint8 tensor shaped like vol")
        mp = ctypes.c_void_p(mask.data_ptr())
    _check(lib.nrr_select_blocks_aniso_ex(ctypes.c_void_p(vol.data_ptr()), dt, _dims3(dims),
                                          _triple(block), _triple(stride), float(fraction), mp,
                                          int(connectivity), ctypes.c_void_p(out.data_ptr()),
                                          out.shape[0], ctypes.c_void_p(kd.data_ptr()),
                                          ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          _stream(vol)))
    return out[:int(kd.item())]


def window_stats_aniso(flt, block, workspace=None):
    """Window statistics of the per-axis block of `flt` into a workspace for
    ``block_match_aniso(..., prepared=True)``; returns the workspace."""
    lib = load()
    dt, dims = _vol_info(flt)
    _, match_bytes = aniso_workspace_bytes(dt, dims, block)
    ws = _workspace(match_bytes, flt.device, workspace)
    _check(lib.nrr_window_stats_aniso(ctypes.c_void_p(flt.data_ptr()), dt, _dims3(dims),
                                      _triple(block), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream(flt)))
    return ws


def block_match_aniso(ref, flt, centers, block, window, workspace=None, out=None,
                      prepared: bool = False):
    """Exhaustive NCC search with per-axis block edges and half windows;
    returns (disp int32 [n,3], ncc f32 [n], conf f32 [n]).  With
    ``prepared=True`` ``workspace`` must hold ``window_stats_aniso(flt, block)``."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(ref)
    dt2, dims2 = _vol_info(flt)
    if dt != dt2 or dims != dims2 or ref.device != flt.device:
        raise NrrError(1, "ref and flt must share dtype, shape and device")
    if centers.dtype != torch.int32 or centers.dim() != 2 or centers.shape[1] != 3 \
            or not centers.is_contiguous() or centers.device != ref.device:
        raise NrrError(1, "centers must be a contiguous int32 [n, 3] tensor on ref's device")
    n = centers.shape[0]
    if out is None:
        disp = torch.empty((n, 3), dtype=torch.int32, device=ref.device)
        ncc = torch.empty(n, dtype=torch.float32, device=ref.device)
        conf = torch.empty(n, dtype=torch.float32, device=ref.device)
    else:
        disp, ncc, conf = out
    if prepared and workspace is None:
        raise NrrError(1, "prepared=True needs the workspace window_stats_aniso() filled")
    _, match_bytes = aniso_workspace_bytes(dt, dims, block)
    ws = _workspace(match_bytes, ref.device, workspace)
    fn = lib.nrr_block_match_aniso_prepared if prepared else lib.nrr_block_match_aniso
    _check(fn(ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(flt.data_ptr()), dt,
              _dims3(dims), ctypes.c_void_p(centers.data_ptr()), n, _triple(block),
              _triple(window), ctypes.c_void_p(disp.data_ptr()), ctypes.c_void_p(ncc.data_ptr()),
              ctypes.c_void_p(conf.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
              _stream(ref)))
    return disp, ncc, conf


def structure_confidence(ref, centers, block: int, conf):
    """Directional confidence S per block (float32 [n, 6]: xx, yy, zz, xy, xz,
    yz) = conf * structure tensor / its trace (see include/nrr.h)."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(ref)
    n = centers.shape[0]
    out = torch.zeros((max(n, 1), 6), dtype=torch.float32, device=ref.device)
    if n == 0:
        return out[:0]
    conf = conf.contiguous().to(torch.float32)
    _check(lib.nrr_structure_confidence(ctypes.c_void_p(ref.data_ptr()), dt, _dims3(dims),
                                        ctypes.c_void_p(centers.data_ptr()), n, block,
                                        ctypes.c_void_p(conf.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream(ref)))
    return out[:n]


# ------------------------------------------------------------------ tuning

def tune_match(ref, flt, centers, block: int, window: int, workspace=None, reps: int = 3):
    """Time every compiled search shape for (dtype, block, window) on these
    inputs and keep the fastest for later searches in this process.
    Returns (shape dict, mean microseconds).  Synchronises the stream."""
    torch = _torch()
    lib = load()
    dt, dims = _vol_info(ref)
    n = centers.shape[0]
    disp = torch.empty((max(n, 1), 3), dtype=torch.int32, device=ref.device)
    ncc = torch.empty(max(n, 1), dtype=torch.float32, device=ref.device)
    conf = torch.empty(max(n, 1), dtype=torch.float32, device=ref.device)
    ws = workspace if workspace is not None else window_stats(flt, block)
    best = TileShape()
    us = ctypes.c_double()
    _check(lib.nrr_tune_match(ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(flt.data_ptr()),
                              dt, _dims3(dims), ctypes.c_void_p(centers.data_ptr()), n, block,
                              window, ctypes.c_void_p(disp.data_ptr()),
                              ctypes.c_void_p(ncc.data_ptr()), ctypes.c_void_p(conf.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), int(reps),
                              ctypes.byref(best), ctypes.byref(us), _stream(ref)))
    return best.as_dict(), us.value


def tuned_shape(dtype: int, block: int, window: int):
    """The tuned shape for (dtype, block, window) as a dict, or None."""
    out = TileShape()
    st = load().nrr_tuned_shape(dtype, block, window, ctypes.byref(out))
    return out.as_dict() if st == 0 else None


def clear_tuning():
    _check(load().nrr_clear_tuning())


# ---------------------------------------------------------- batched search

def _param_array(sets):
    arr = (ParamSet * max(len(sets), 1))()
    for i, q in enumerate(sets):
        if isinstance(q, ParamSet):
            arr[i] = q
        else:
            b, w, stride, frac = q
            arr[i] = ParamSet(int(b), int(w), int(stride), float(frac))
    return arr


def batch_layout(dtype: int, dims, sets):
    """(row offsets per set [nsets+1], workspace bytes) of a batched search."""
    arr = _param_array(sets)
    offs = (ctypes.c_int64 * (len(sets) + 1))()
    nb = ctypes.c_size_t()
    _check(load().nrr_batch_layout(dtype, _dims3(dims), arr, len(sets), offs, ctypes.byref(nb)))
    return list(offs), nb.value


def batch_shapes(dtype: int, dims, sets) -> list:
    """The shape each parameter set of a batched plan would run with."""
    arr = _param_array(sets)
    out = (TileShape * max(len(sets), 1))()
    _check(load().nrr_batch_shapes(dtype, _dims3(dims), arr, len(sets), out))
    return [out[i].as_dict() for i in range(len(sets))]


class BatchPlan:
    """A batched parametric search over one volume pair.

    ``sets`` are (block, window, stride, fraction) tuples.  ``run()`` enqueues
    one batch on the current stream (a HIP graph replay with ``use_graph``);
    ``results()`` splits the outputs into per-set (centers, disp, ncc, conf)
    views.  Inputs must stay alive and unchanged in shape while the plan
    lives (the plan reads them on every run)."""

    def __init__(self, ref, flt, sets, use_graph: bool = True):
        torch = _torch()
        lib = load()
        dt, dims = _vol_info(ref)
        dt2, dims2 = _vol_info(flt)
        if dt != dt2 or dims != dims2 or ref.device != flt.device:
            raise NrrError(1, "ref and flt must share dtype, shape and device")
        self.ref, self.flt, self.sets = ref, flt, list(sets)
        self.offsets, nbytes = batch_layout(dt, dims, self.sets)
        rows = max(self.offsets[-1], 1)
        dev = ref.device
        self.centers = torch.empty((rows, 3), dtype=torch.int32, device=dev)
        self.disp = torch.empty((rows, 3), dtype=torch.int32, device=dev)
        self.ncc = torch.empty(rows, dtype=torch.float32, device=dev)
        self.conf = torch.empty(rows, dtype=torch.float32, device=dev)
        self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        arr = _param_array(self.sets)
        h = ctypes.c_void_p()
        torch.cuda.synchronize(dev)
        _check(lib.nrr_batch_plan_create(
            ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(flt.data_ptr()), dt, _dims3(dims),
            arr, len(self.sets), ctypes.c_void_p(self.centers.data_ptr()),
            ctypes.c_void_p(self.disp.data_ptr()), ctypes.c_void_p(self.ncc.data_ptr()),
            ctypes.c_void_p(self.conf.data_ptr()), ctypes.c_void_p(self.workspace.data_ptr()),
            self.workspace.numel(), 1 if use_graph else 0, _stream(ref), ctypes.byref(h)))
        self._h = h

    def run(self):
        if self._h is None:
            raise NrrError(1, "plan closed")
        _check(load().nrr_batch_plan_run(self._h, _stream(self.ref)))

    def results(self):
        out = []
        for i in range(len(self.sets)):
            a, b = self.offsets[i], self.offsets[i + 1]
            out.append((self.centers[a:b], self.disp[a:b], self.ncc[a:b], self.conf[a:b]))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().nrr_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving

def _host_or_dev_info(t):
    torch = _torch()
    if t.dim() != 3 or not t.is_contiguous():
        raise NrrError(1, "volumes must be contiguous [nz, ny, nx] tensors")
    if t.dtype == torch.uint16:
        dt = U16
    elif t.dtype == torch.float32:
        dt = F32
    else:
        raise NrrError(1, "volume dtype must be uint16 or float32, got %s" % t.dtype)
    nz, ny, nx = t.shape
    return dt, (nx, ny, nz)


class Volume:
    """A volume held in a server's memory (Server.add_volume); requests name
    it in place of a tensor."""

    def __init__(self, server, vid, dtype, dims):
        self.server, self.id, self.dtype, self.dims = server, vid, dtype, dims

    def remove(self):
        """Free the volume (all requests naming it must have finished)."""
        if self.id and getattr(self.server, "_h", None) is not None:
            _check(load().nrr_server_remove_volume(self.server._h, self.id))
        self.id = 0


def _vol_or_tensor(v):
    if isinstance(v, Volume):
        return v.dtype, v.dims, None, v.id
    dt, dims = _host_or_dev_info(v)
    return dt, dims, v.data_ptr(), 0


def _make_request(ref, flt, block, stride, window, fraction, outs=None):
    dt, dims, rp, _ = _vol_or_tensor(ref)
    dt2, dims2, fp, _ = _vol_or_tensor(flt)
    if dt != dt2 or dims != dims2:
        raise NrrError(1, "ref and flt must share dtype and shape")
    r = _Request()
    r.ref, r.flt, r.dtype = rp, fp, dt
    r.dims[:] = list(dims)
    r.block, r.stride, r.window, r.fraction = int(block), int(stride), int(window), float(fraction)
    if outs is not None:
        c, d, n, f = outs
        r.centers, r.disp, r.ncc, r.conf = c.data_ptr(), d.data_ptr(), n.data_ptr(), f.data_ptr()
        r.capacity = c.shape[0]
    return r, dt, dims


def request_footprint(ref, flt, block: int, stride: int, window: int, fraction: float) -> int:
    """Device bytes one served request occupies while it runs."""
    r, _, _ = _make_request(ref, flt, block, stride, window, fraction)
    nb = ctypes.c_size_t()
    _check(load().nrr_request_footprint(ctypes.byref(r), ctypes.byref(nb)))
    return nb.value


class Job:
    """One submitted registration: poll()/wait() give its state and times;
    after wait(), centers/disp/ncc/conf hold its results (host tensors in
    page-locked memory, or the device tensors given at submission)."""

    def __init__(self, server, ticket, keep, outs, k):
        self.server, self.ticket, self._keep = server, ticket, keep
        self._info = None
        self.centers, self.disp, self.ncc, self.conf = [o[:k] for o in outs]
        self.k = k

    def poll(self):
        if self._info is not None:
            return dict(self._info)
        info = _RequestInfo()
        _check(load().nrr_server_poll(self.server._h, self.ticket, ctypes.byref(info)))
        return info.as_dict()

    def wait(self):
        """Block until the request finishes; its record is then released in
        the server (later poll()/wait() return the same information)."""
        if self._info is not None:
            return dict(self._info)
        info = _RequestInfo()
        st = load().nrr_server_wait(self.server._h, self.ticket, ctypes.byref(info))
        if st in (0, 3):  # finished (done, or failed on the device)
            _check(load().nrr_server_release(self.server._h, self.ticket))
            self._keep = None
            self._info = info.as_dict()
        _check(st)
        return dict(self._info)


class Server:
    """Registration server: admits requests as slots and device memory free
    up (continuous batching); see nrr_server_create in include/nrr.h."""

    def __init__(self, device_bytes: int = 8 << 30, slots: int = 4):
        h = ctypes.c_void_p()
        _check(load().nrr_server_create(int(device_bytes), int(slots), ctypes.byref(h)))
        self._h = h

    def add_volume(self, vol) -> Volume:
        """Copy a [nz, ny, nx] host or device tensor into the server's memory
        once; requests may then name the returned Volume in place of it."""
        torch = _torch()
        dt, dims = _host_or_dev_info(vol)
        if vol.is_cuda:
            torch.cuda.current_stream(vol.device).synchronize()  # the copy is ordered after nothing
        vid = ctypes.c_int64()
        _check(load().nrr_server_add_volume(self._h, ctypes.c_void_p(vol.data_ptr()), dt,
                                            _dims3(dims), ctypes.byref(vid)))
        return Volume(self, vid.value, dt, dims)

    def submit(self, ref, flt, block: int, stride: int, window: int, fraction: float,
               out=None) -> Job:
        """Queue one registration.  `ref`/`flt` are [nz, ny, nx] host (ideally
        page-locked) or device tensors, kept alive until the job completes,
        or Volumes added to this server.  Results go to `out` = (centers,
        disp, ncc, conf) tensors of >= K rows if given, else to new
        page-locked host tensors."""
        torch = _torch()
        dt, dims, _, ref_id = _vol_or_tensor(ref)
        flt_id = _vol_or_tensor(flt)[3]
        k = select_count(dims, block, stride, fraction)
        if out is None:
            rows = max(k, 1)
            out = (torch.empty((rows, 3), dtype=torch.int32, pin_memory=True),
                   torch.empty((rows, 3), dtype=torch.int32, pin_memory=True),
                   torch.empty(rows, dtype=torch.float32, pin_memory=True),
                   torch.empty(rows, dtype=torch.float32, pin_memory=True))
        r, _, _ = _make_request(ref, flt, block, stride, window, fraction, out)
        t = ctypes.c_int64()
        _check(load().nrr_server_submit_resident(self._h, ctypes.byref(r), ref_id, flt_id,
                                                 ctypes.byref(t)))
        return Job(self, t.value, (ref, flt), out, k)

    def stats(self):
        info = _ServerInfo()
        _check(load().nrr_server_stats(self._h, ctypes.byref(info)))
        return info.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().nrr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
