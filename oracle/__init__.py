"""Block-matching oracle (FP64, CPU) -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2308_10868_amd``) and imports nothing from it.

``nrr_oracle.c`` is the plain C implementation (FP64, plain loops, OpenMP over
blocks); ``twin.py`` is an independently written NumPy brute force for tiny
inputs.  Both follow the paper's definitions: variance-ranked block selection
with K = floor(0.5 + N*F), and an exhaustive search maximising the normalised
cross-correlation (read as the Pearson correlation over the block).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nrr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

U16, F32 = 0, 1


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no intrinsics, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        # NRR_ORACLE_LIB lets the mutation test load a deliberately broken
        # copy of this oracle (built from a modified source in a temp dir).
        path = os.environ.get("NRR_ORACLE_LIB") or build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.oracle_select.restype = i64
        lib.oracle_select.argtypes = [P, ctypes.c_int, P, i32, i32, f64, P, P, i64]
        lib.oracle_structure_confidence.restype = ctypes.c_int
        lib.oracle_structure_confidence.argtypes = [P, ctypes.c_int, P, P, i64, i32, P, P]
        lib.oracle_select_ex.restype = i64
        lib.oracle_select_ex.argtypes = [P, ctypes.c_int, P, i32, i32, f64, P, i32, P, P, i64]
        lib.oracle_block_variance.restype = ctypes.c_int
        lib.oracle_block_variance.argtypes = [P, ctypes.c_int, P, i32, i32, P, P]
        lib.oracle_match.restype = ctypes.c_int
        lib.oracle_match.argtypes = [P, P, ctypes.c_int, P, P, i64, i32, i32, P, P, P]
        lib.oracle_ncc_surface.restype = ctypes.c_int
        lib.oracle_ncc_surface.argtypes = [P, P, ctypes.c_int, P, P, i64, i32, i32, P]
        lib.oracle_valid_shifts.restype = ctypes.c_int
        lib.oracle_valid_shifts.argtypes = [P, P, i64, i32, i32, P]
        lib.oracle_select_count.restype = i64
        lib.oracle_select_count.argtypes = [i64, f64]
        lib.oracle_grid_shape.restype = ctypes.c_int
        lib.oracle_grid_shape.argtypes = [P, i32, i32, P]
        lib.oracle_select_aniso.restype = i64
        lib.oracle_select_aniso.argtypes = [P, ctypes.c_int, P, P, P, f64, P, P, i64]
        lib.oracle_select_aniso_ex.restype = i64
        lib.oracle_select_aniso_ex.argtypes = [P, ctypes.c_int, P, P, P, f64, P, i32, P, P, i64]
        lib.oracle_match_aniso.restype = ctypes.c_int
        lib.oracle_match_aniso.argtypes = [P, P, ctypes.c_int, P, P, i64, P, P, P, P, P]
        lib.oracle_ncc_aniso_at.restype = ctypes.c_int
        lib.oracle_ncc_aniso_at.argtypes = [P, P, ctypes.c_int, P, P, P, i64, P, P]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _vol(a: np.ndarray):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        return a, U16
    if a.dtype == np.float32:
        return a, F32
    raise TypeError("volume must be uint16 or float32, got %s" % a.dtype)


def _dims(a: np.ndarray) -> np.ndarray:
    nz, ny, nx = a.shape
    return np.array([nx, ny, nz], dtype=np.int32)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    """Cap the OpenMP threads of later oracle calls in this process."""
    _load().oracle_set_threads(int(n))


def threads() -> int:
    return int(_load().oracle_threads())


def grid_shape(dims, block: int, stride: int):
    g = np.zeros(3, dtype=np.int32)
    d = np.asarray(dims, dtype=np.int32)
    if _load().oracle_grid_shape(_ptr(d), block, stride, _ptr(g)):
        raise ValueError("bad grid arguments")
    return tuple(int(v) for v in g)


def select_count(n_candidates: int, fraction: float) -> int:
    return int(_load().oracle_select_count(n_candidates, fraction))


def block_variance(vol: np.ndarray, block: int, stride: int):
    """(key[N], var[N]) for every candidate block, in linear grid order."""
    vol, dt = _vol(vol)
    dims = _dims(vol)
    n = int(np.prod(grid_shape(dims, block, stride)))
    key = np.empty(n, dtype=np.float64)
    var = np.empty(n, dtype=np.float64)
    _load().oracle_block_variance(_ptr(vol), dt, _ptr(dims), block, stride, _ptr(key), _ptr(var))
    return key, var


def select(vol: np.ndarray, block: int, stride: int, fraction: float):
    """Selected centres int32[K, 3] (x, y, z) in ascending grid index, and
    their FP64 variances."""
    vol, dt = _vol(vol)
    dims = _dims(vol)
    n = int(np.prod(grid_shape(dims, block, stride)))
    cap = max(1, n)
    out = np.empty((cap, 3), dtype=np.int32)
    var = np.empty(cap, dtype=np.float64)
    k = _load().oracle_select(_ptr(vol), dt, _ptr(dims), block, stride, float(fraction),
                              _ptr(out), _ptr(var), cap)
    if k < 0:
        raise ValueError("oracle_select rejected the arguments (%d)" % k)
    return out[:k].copy(), var[:k].copy()


def select_ex(vol: np.ndarray, block: int, stride: int, fraction: float, mask=None,
              connectivity: int = 0):
    """Selection with a candidate mask (uint8 volume, nonzero = candidate
    centre allowed) and a connectivity pattern (0, 6, 18, 26): the taken
    centres int32[k, 3] in ascending grid index, and their variances."""
    vol, dt = _vol(vol)
    dims = _dims(vol)
    n = int(np.prod(grid_shape(dims, block, stride)))
    cap = max(1, n)
    out = np.empty((cap, 3), dtype=np.int32)
    var = np.empty(cap, dtype=np.float64)
    mp = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.shape == vol.shape
        mp = _ptr(mask)
    k = _load().oracle_select_ex(_ptr(vol), dt, _ptr(dims), block, stride, float(fraction), mp,
                                 int(connectivity), _ptr(out), _ptr(var), cap)
    if k < 0:
        raise ValueError("oracle_select_ex rejected the arguments (%d)" % k)
    return out[:k].copy(), var[:k].copy()


def structure_confidence(ref: np.ndarray, centers: np.ndarray, block: int, conf: np.ndarray):
    """Directional confidence S per block: f64 [n, 6] = (xx, yy, zz, xy, xz, yz)."""
    ref, dt = _vol(ref)
    c = np.ascontiguousarray(centers, dtype=np.int32).reshape(-1, 3)
    n = c.shape[0]
    cf = np.ascontiguousarray(conf, dtype=np.float64).reshape(n)
    out = np.zeros((max(n, 1), 6), dtype=np.float64)
    if _load().oracle_structure_confidence(_ptr(ref), dt, _ptr(_dims(ref)), _ptr(c), n, block,
                                           _ptr(cf), _ptr(out)):
        raise ValueError("oracle_structure_confidence rejected the arguments")
    return out[:n]


def match(ref: np.ndarray, flt: np.ndarray, centers: np.ndarray, block: int, window: int):
    """Exhaustive NCC search: (disp int32[n,3], ncc f64[n], conf f64[n])."""
    ref, dt = _vol(ref)
    flt, dt2 = _vol(flt)
    assert dt == dt2 and ref.shape == flt.shape
    c = np.ascontiguousarray(centers, dtype=np.int32).reshape(-1, 3)
    n = c.shape[0]
    disp = np.zeros((max(n, 1), 3), dtype=np.int32)
    ncc = np.zeros(max(n, 1), dtype=np.float64)
    conf = np.zeros(max(n, 1), dtype=np.float64)
    if _load().oracle_match(_ptr(ref), _ptr(flt), dt, _ptr(_dims(ref)), _ptr(c), n, block, window,
                            _ptr(disp), _ptr(ncc), _ptr(conf)):
        raise ValueError("oracle_match rejected the arguments")
    return disp[:n], ncc[:n], conf[:n]


def _triple(v) -> np.ndarray:
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.int32), (3,)))
    return t


def select_aniso(vol: np.ndarray, block, stride, fraction: float):
    """Selection with per-axis block edges and strides ((x, y, z) triples):
    centres int32[K, 3] in ascending grid index and their FP64 variances."""
    vol, dt = _vol(vol)
    dims = _dims(vol)
    b, s = _triple(block), _triple(stride)
    if np.any(b < 1) or np.any(b % 2 == 0) or np.any(s < 1) or np.any(dims < b):
        raise ValueError("bad per-axis block/stride")
    n = int(np.prod((dims - b) // s + 1))
    cap = max(select_count(n, fraction), 1)
    centers = np.zeros((cap, 3), dtype=np.int32)
    var = np.zeros(cap, dtype=np.float64)
    k = _load().oracle_select_aniso(_ptr(vol), dt, _ptr(dims), _ptr(b), _ptr(s), fraction,
                                    _ptr(centers), _ptr(var), cap)
    if k < 0:
        raise ValueError("oracle_select_aniso rejected the arguments (%d)" % k)
    return centers[:k], var[:k]


def select_aniso_ex(vol: np.ndarray, block, stride, fraction: float, mask=None,
                    connectivity: int = 0):
    """Selection variants (mask, connectivity pattern) with per-axis block
    edges and strides: centres int32[k, 3] in ascending grid index and their
    FP64 variances."""
    vol, dt = _vol(vol)
    dims = _dims(vol)
    b, s = _triple(block), _triple(stride)
    if np.any(b < 1) or np.any(b % 2 == 0) or np.any(s < 1) or np.any(dims < b):
        raise ValueError("bad per-axis block/stride")
    n = int(np.prod((dims - b) // s + 1))
    cap = max(n, 1)
    centers = np.zeros((cap, 3), dtype=np.int32)
    var = np.zeros(cap, dtype=np.float64)
    mp = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.shape == vol.shape
        mp = _ptr(mask)
    k = _load().oracle_select_aniso_ex(_ptr(vol), dt, _ptr(dims), _ptr(b), _ptr(s),
                                       float(fraction), mp, int(connectivity), _ptr(centers),
                                       _ptr(var), cap)
    if k < 0:
        raise ValueError("oracle_select_aniso_ex rejected the arguments (%d)" % k)
    return centers[:k].copy(), var[:k].copy()


def match_aniso(ref: np.ndarray, flt: np.ndarray, centers: np.ndarray, block, window):
    """Exhaustive NCC search with per-axis block edges and half windows:
    (disp int32[n,3], ncc f64[n], conf f64[n])."""
    ref, dt = _vol(ref)
    flt, dt2 = _vol(flt)
    assert dt == dt2 and ref.shape == flt.shape
    c = np.ascontiguousarray(centers, dtype=np.int32).reshape(-1, 3)
    n = c.shape[0]
    disp = np.zeros((max(n, 1), 3), dtype=np.int32)
    ncc = np.zeros(max(n, 1), dtype=np.float64)
    conf = np.zeros(max(n, 1), dtype=np.float64)
    if _load().oracle_match_aniso(_ptr(ref), _ptr(flt), dt, _ptr(_dims(ref)), _ptr(c), n,
                                  _ptr(_triple(block)), _ptr(_triple(window)), _ptr(disp),
                                  _ptr(ncc), _ptr(conf)):
        raise ValueError("oracle_match_aniso rejected the arguments")
    return disp[:n], ncc[:n], conf[:n]


def ncc_aniso_at(ref: np.ndarray, flt: np.ndarray, centers, disp, block) -> np.ndarray:
    """FP64 NCC of each ref block and its flt block displaced by disp[k]
    (per-axis block edges); NaN where a block leaves the volume."""
    ref, dt = _vol(ref)
    flt, _ = _vol(flt)
    c = np.ascontiguousarray(centers, dtype=np.int32).reshape(-1, 3)
    d = np.ascontiguousarray(disp, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(max(len(c), 1), dtype=np.float64)
    if _load().oracle_ncc_aniso_at(_ptr(ref), _ptr(flt), dt, _ptr(_dims(ref)), _ptr(c), _ptr(d),
                                   len(c), _ptr(_triple(block)), _ptr(out)):
        raise ValueError("oracle_ncc_aniso_at rejected the arguments")
    return out[:len(c)]


def ncc_surface(ref: np.ndarray, flt: np.ndarray, centers: np.ndarray, block: int, window: int):
    """NCC for every displacement: f64[n, 2W+1, 2W+1, 2W+1] indexed [dz][dy][dx]
    (offset by W); NaN where the displaced block leaves the volume."""
    ref, dt = _vol(ref)
    flt, _ = _vol(flt)
    c = np.ascontiguousarray(centers, dtype=np.int32).reshape(-1, 3)
    n = c.shape[0]
    s = 2 * window + 1
    out = np.empty((max(n, 1), s, s, s), dtype=np.float64)
    if _load().oracle_ncc_surface(_ptr(ref), _ptr(flt), dt, _ptr(_dims(ref)), _ptr(c), n, block,
                                  window, _ptr(out)):
        raise ValueError("oracle_ncc_surface rejected the arguments")
    return out[:n]


def valid_shifts(dims, centers: np.ndarray, block: int, window: int) -> np.ndarray:
    """Number of evaluated displacements per centre."""
    c = np.ascontiguousarray(centers, dtype=np.int32).reshape(-1, 3)
    d = np.asarray(dims, dtype=np.int32)
    out = np.zeros(max(c.shape[0], 1), dtype=np.int64)
    _load().oracle_valid_shifts(_ptr(d), _ptr(c), c.shape[0], block, window, _ptr(out))
    return out[: c.shape[0]]
