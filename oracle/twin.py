"""NumPy brute-force twin of the C oracle, for tiny inputs only.

Test infrastructure.  Written independently of ``nrr_oracle.c`` (vectorised
NumPy over all displacements via ``sliding_window_view`` instead of plain
loops) so that the two check each other.  Same readings of the paper:
variance-ranked selection keeping K = floor(0.5 + N*F) blocks (ties by lower
grid index, output in ascending grid index), exhaustive search maximising the
Pearson-correlation reading of the NCC equation (0 for a flat block or
window, exact ties -> smallest shift index), confidence max(0, NCC).
"""

from __future__ import annotations

import math

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def grid_origins(n: int, block: int, stride: int) -> np.ndarray:
    return np.arange(0, n - block + 1, stride)


def select(vol: np.ndarray, block: int, stride: int, fraction: float) -> np.ndarray:
    nz, ny, nx = vol.shape
    ox, oy, oz = (grid_origins(n, block, stride) for n in (nx, ny, nz))
    blocks = sliding_window_view(vol, (block, block, block))[np.ix_(oz, oy, ox)]
    blocks = blocks.reshape(len(oz) * len(oy) * len(ox), -1)
    if vol.dtype == np.uint16:
        v = blocks.astype(np.int64)
        score = block ** 3 * (v * v).sum(axis=1) - v.sum(axis=1) ** 2  # exact integers
    else:
        score = blocks.astype(np.float64).var(axis=1)
    n = score.shape[0]
    k = min(n, max(0, math.floor(0.5 + n * fraction)))
    order = np.lexsort((np.arange(n), -score))  # variance desc, grid index asc
    chosen = np.sort(order[:k])
    gz, rem = np.divmod(chosen, len(oy) * len(ox))
    gy, gx = np.divmod(rem, len(ox))
    h = (block - 1) // 2
    return np.stack([ox[gx] + h, oy[gy] + h, oz[gz] + h], axis=1).astype(np.int32)


def select_ex(vol: np.ndarray, block: int, stride: int, fraction: float, mask=None,
              connectivity: int = 0) -> np.ndarray:
    """Greedy selection in rank order with a candidate mask and a connectivity
    pattern, written independently of the C oracle (small grids only)."""
    nz, ny, nx = vol.shape
    ox, oy, oz = (grid_origins(n, block, stride) for n in (nx, ny, nz))
    blocks = sliding_window_view(vol, (block, block, block))[np.ix_(oz, oy, ox)]
    blocks = blocks.reshape(len(oz) * len(oy) * len(ox), -1)
    if vol.dtype == np.uint16:
        v = blocks.astype(np.int64)
        score = block ** 3 * (v * v).sum(axis=1) - v.sum(axis=1) ** 2
    else:
        score = blocks.astype(np.float64).var(axis=1)
    h = (block - 1) // 2
    G = (len(ox), len(oy), len(oz))
    cand = []
    for g in range(score.shape[0]):
        gz, rem = divmod(g, G[0] * G[1])
        gy, gx = divmod(rem, G[0])
        if mask is None or mask[oz[gz] + h, oy[gy] + h, ox[gx] + h]:
            cand.append(g)
    k = min(len(cand), max(0, math.floor(0.5 + len(cand) * fraction)))
    cand.sort(key=lambda g: (-score[g], g))
    limit = {0: 0, 6: 1, 18: 2, 26: 3}[connectivity]
    taken = set()
    for g in cand:
        if len(taken) == k:
            break
        gz, rem = divmod(g, G[0] * G[1])
        gy, gx = divmod(rem, G[0])
        near = False
        for q in taken:
            qz, r2 = divmod(q, G[0] * G[1])
            qy, qx = divmod(r2, G[0])
            d = (abs(qx - gx), abs(qy - gy), abs(qz - gz))
            if max(d) == 1 and sum(d) <= limit:
                near = True
                break
        if not near:
            taken.add(g)
    out = []
    for g in sorted(taken):
        gz, rem = divmod(g, G[0] * G[1])
        gy, gx = divmod(rem, G[0])
        out.append((ox[gx] + h, oy[gy] + h, oz[gz] + h))
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def surface(ref: np.ndarray, flt: np.ndarray, center, block: int, window: int) -> np.ndarray:
    """NCC over [-W, W]^3 indexed [dz+W, dy+W, dx+W]; NaN where invalid."""
    h = (block - 1) // 2
    s = 2 * window + 1
    out = np.full((s, s, s), np.nan)
    cx, cy, cz = (int(v) for v in center)
    nz, ny, nx = ref.shape
    if not (h <= cx < nx - h and h <= cy < ny - h and h <= cz < nz - h):
        return out
    t = ref[cz - h:cz + h + 1, cy - h:cy + h + 1, cx - h:cx + h + 1].astype(np.float64).ravel()
    t = t - t.mean()
    tt = float(t @ t)
    wins = sliding_window_view(flt, (block, block, block))  # [z0, y0, x0, b, b, b]
    rng = []
    for c, n in ((cz, nz), (cy, ny), (cx, nx)):
        lo = max(-window, h - c)
        hi = min(window, n - 1 - h - c)
        rng.append((lo, hi))
    (lz, hz), (ly, hy), (lx, hx) = rng
    sub = wins[cz - h + lz:cz - h + hz + 1, cy - h + ly:cy - h + hy + 1,
               cx - h + lx:cx - h + hx + 1].astype(np.float64)
    f = sub.reshape(sub.shape[:3] + (-1,))
    f = f - f.mean(axis=-1, keepdims=True)
    num = f @ t
    ff = np.einsum("...i,...i->...", f, f)
    den2 = tt * ff
    val = np.where(den2 > 0, num / np.sqrt(np.where(den2 > 0, den2, 1.0)), 0.0)
    out[lz + window:hz + window + 1, ly + window:hy + window + 1,
        lx + window:hx + window + 1] = val
    return out


def match(ref: np.ndarray, flt: np.ndarray, centers: np.ndarray, block: int, window: int):
    n = len(centers)
    disp = np.zeros((n, 3), dtype=np.int32)
    ncc = np.zeros(n)
    conf = np.zeros(n)
    for k, c in enumerate(centers):
        srf = surface(ref, flt, c, block, window)
        flat = srf.ravel()  # C order: dz slowest, dx fastest == increasing shift index
        if np.all(np.isnan(flat)):
            ncc[k] = np.nan
            continue
        best = np.nanmax(flat)
        i = int(np.flatnonzero(flat == best)[0])
        dz, rem = divmod(i, (2 * window + 1) ** 2)
        dy, dx = divmod(rem, 2 * window + 1)
        disp[k] = (dx - window, dy - window, dz - window)
        ncc[k] = best
        conf[k] = max(0.0, best)
    return disp, ncc, conf


def structure_confidence(ref: np.ndarray, centers, block: int, conf) -> np.ndarray:
    """Directional confidence by numpy.gradient (central differences inside,
    one-sided first differences on the border planes)."""
    v = ref.astype(np.float64)
    gz, gy, gx = np.gradient(v, edge_order=1)
    h = (block - 1) // 2
    out = np.zeros((len(centers), 6))
    nz, ny, nx = v.shape
    for k, (cx, cy, cz) in enumerate(np.asarray(centers).reshape(-1, 3)):
        if not (cx - h >= 0 and cy - h >= 0 and cz - h >= 0 and cx + h < nx and cy + h < ny
                and cz + h < nz):
            continue
        sl = (slice(cz - h, cz + h + 1), slice(cy - h, cy + h + 1), slice(cx - h, cx + h + 1))
        a, b, c = gx[sl].ravel(), gy[sl].ravel(), gz[sl].ravel()
        j = np.array([a @ a, b @ b, c @ c, a @ b, a @ c, b @ c])
        tr = j[:3].sum()
        out[k] = conf[k] * j / tr if tr > 0 else 0.0
    return out


def select_aniso(vol: np.ndarray, block, stride, fraction: float) -> np.ndarray:
    """Selection with per-axis block edges and strides, (x, y, z) triples."""
    bx, by, bz = (int(v) for v in block)
    sx, sy, sz = (int(v) for v in stride)
    nz, ny, nx = vol.shape
    ox, oy, oz = grid_origins(nx, bx, sx), grid_origins(ny, by, sy), grid_origins(nz, bz, sz)
    blocks = sliding_window_view(vol, (bz, by, bx))[np.ix_(oz, oy, ox)]
    blocks = blocks.reshape(len(oz) * len(oy) * len(ox), -1)
    if vol.dtype == np.uint16:
        v = blocks.astype(np.int64)
        score = bx * by * bz * (v * v).sum(axis=1) - v.sum(axis=1) ** 2
    else:
        score = blocks.astype(np.float64).var(axis=1)
    n = score.shape[0]
    k = min(n, max(0, math.floor(0.5 + n * fraction)))
    chosen = np.sort(np.lexsort((np.arange(n), -score))[:k])
    gz, rem = np.divmod(chosen, len(oy) * len(ox))
    gy, gx = np.divmod(rem, len(ox))
    return np.stack([ox[gx] + (bx - 1) // 2, oy[gy] + (by - 1) // 2, oz[gz] + (bz - 1) // 2],
                    axis=1).astype(np.int32)


def select_aniso_ex(vol: np.ndarray, block, stride, fraction: float, mask=None,
                    connectivity: int = 0) -> np.ndarray:
    """Per-axis sizes with a candidate mask and a connectivity pattern: rank
    every candidate, keep those whose centre the mask allows, then walk the
    ranking and skip any candidate with a taken grid neighbour (small grids
    only; a set of taken grid coordinates)."""
    bx, by, bz = (int(v) for v in block)
    sx, sy, sz = (int(v) for v in stride)
    nz, ny, nx = vol.shape
    ox, oy, oz = grid_origins(nx, bx, sx), grid_origins(ny, by, sy), grid_origins(nz, bz, sz)
    blocks = sliding_window_view(vol, (bz, by, bx))[np.ix_(oz, oy, ox)]
    score = blocks.reshape(len(oz), len(oy), len(ox), -1)
    if vol.dtype == np.uint16:
        v = score.astype(np.int64)
        score = bx * by * bz * (v * v).sum(axis=-1) - v.sum(axis=-1) ** 2
    else:
        score = score.astype(np.float64).var(axis=-1)
    cz, cy, cx = np.meshgrid(oz + (bz - 1) // 2, oy + (by - 1) // 2, ox + (bx - 1) // 2,
                             indexing="ij")
    inside = np.ones(score.shape, bool) if mask is None else mask[cz, cy, cx] != 0
    order = np.lexsort((np.arange(score.size), -score.ravel()))
    order = order[inside.ravel()[order]]
    k = min(len(order), max(0, math.floor(0.5 + len(order) * fraction)))
    reach = {0: 0, 6: 1, 18: 2, 26: 3}[connectivity]
    steps = [(a, b_, c) for a in (-1, 0, 1) for b_ in (-1, 0, 1) for c in (-1, 0, 1)
             if 0 < abs(a) + abs(b_) + abs(c) <= reach]
    taken = set()
    for g in order:
        if len(taken) == k:
            break
        iz, iy, ix = np.unravel_index(g, score.shape)
        if any((iz + a, iy + b_, ix + c) in taken for a, b_, c in steps):
            continue
        taken.add((int(iz), int(iy), int(ix)))
    out = sorted(taken)  # (z, y, x) order = ascending grid index
    return np.asarray([(ox[x] + (bx - 1) // 2, oy[y] + (by - 1) // 2, oz[z] + (bz - 1) // 2)
                       for z, y, x in out], dtype=np.int32).reshape(-1, 3)


def match_aniso(ref: np.ndarray, flt: np.ndarray, centers, block, window):
    """Search with per-axis block edges and half windows: every valid shift's
    Pearson correlation, argmax by (largest NCC, smallest shift index)."""
    b = np.array([int(v) for v in block])      # (x, y, z)
    w = np.array([int(v) for v in window])
    h = (b - 1) // 2
    dims = np.array(ref.shape[::-1])
    n = len(centers)
    disp = np.zeros((n, 3), dtype=np.int32)
    ncc = np.full(n, np.nan)
    conf = np.zeros(n)
    wins = sliding_window_view(flt, (b[2], b[1], b[0]))
    for k, c in enumerate(np.asarray(centers, dtype=np.int64)):
        if np.any(c - h < 0) or np.any(c + h > dims - 1):
            continue
        t = ref[c[2] - h[2]:c[2] + h[2] + 1, c[1] - h[1]:c[1] + h[1] + 1,
                c[0] - h[0]:c[0] + h[0] + 1].astype(np.float64).ravel()
        t -= t.mean()
        lo = np.maximum(-w, h - c)
        hi = np.minimum(w, dims - 1 - h - c)
        sub = wins[c[2] - h[2] + lo[2]:c[2] - h[2] + hi[2] + 1,
                   c[1] - h[1] + lo[1]:c[1] - h[1] + hi[1] + 1,
                   c[0] - h[0] + lo[0]:c[0] - h[0] + hi[0] + 1].astype(np.float64)
        f = sub.reshape(sub.shape[:3] + (-1,))
        f = f - f.mean(axis=-1, keepdims=True)
        den2 = float(t @ t) * np.einsum("...i,...i->...", f, f)
        val = np.where(den2 > 0, (f @ t) / np.sqrt(np.where(den2 > 0, den2, 1.0)), 0.0)
        # the sub-array is in increasing shift index (dz slowest, dx fastest)
        i = int(np.flatnonzero(val.ravel() == val.max())[0])
        iz, rem = divmod(i, val.shape[1] * val.shape[2])
        iy, ix = divmod(rem, val.shape[2])
        disp[k] = (lo[0] + ix, lo[1] + iy, lo[2] + iz)
        ncc[k] = val.max()
        conf[k] = max(0.0, ncc[k])
    return disp, ncc, conf
