"""Seeded synthetic volumes that stand in for the paper's clinical MRI pairs.

This module only *makes inputs*: it holds none of the block-matching
arithmetic (no variance, no selection, no correlation).  Both the oracle
under ``oracle/`` and the HIP path consume the arrays it returns, so every
comparison is made on identical bytes.

Conventions (shared by every generator):

* Arrays are C-order ``[z][y][x]``; ``dims`` is ``(nx, ny, nz)``.
* Vectors (centres, shifts, sag directions) are ``(x, y, z)``.
* ``ref`` is the undeformed pre-operative volume (blocks are taken from it);
  ``flt`` is the deformed intra-operative volume (the search window lies in
  it).  ``flt(p) = ref(p - s)`` for a pure translation ``s``, so the
  displacement the matcher should recover at a block is ``+s``.
* Randomness comes from ``numpy.random.default_rng`` over child streams of a
  ``SeedSequence(seed)``; the draw order of each generator is fixed and
  written in its docstring.

Workloads (the paper measures clinical brain MRI, which is not available; the
shapes, value ranges and deformation magnitudes below are the stand-ins):

* ``gen_translation_f32``: 64^3 float32 Gaussian-blob volumes, ``flt`` is
  ``ref`` translated by an integer shift (3, -2, 1), fresh noise.
* ``gen_mri_u16``: 256x256x124 uint16 12-bit volumes with three smooth tissue
  classes and Rician-like noise; ``flt`` is ``ref`` warped by 1-3 Gaussian
  radial "sags" (brain shift) with trilinear resampling.
* ``gen_blobs_u16``: large uint16 12-bit blob volumes (the dense 512x512x256
  case) warped by 3 sags of peak displacement up to 14 voxels.
* ``gen_random``: tiny non-cubic random volumes for brute-force parity.
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "VolumePair",
    "gen_translation_f32",
    "gen_mri_u16",
    "gen_blobs_u16",
    "gen_random",
    "sha256",
]

U16_MAX12 = 4095


@dataclass
class VolumePair:
    ref: np.ndarray  # [nz, ny, nx]
    flt: np.ndarray  # [nz, ny, nx]
    dims: tuple  # (nx, ny, nz)
    meta: dict = field(default_factory=dict)

    @property
    def dtype(self) -> str:
        return "u16" if self.ref.dtype == np.uint16 else "f32"


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _streams(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def _blob_field(shape_zyx, centres, sigmas, amps, offset=(0.0, 0.0, 0.0), support=None):
    """Sum of isotropic Gaussian blobs evaluated at voxel centres (float64).

    ``offset`` (x, y, z) evaluates the field at ``p - offset`` (a translated
    copy, computed analytically so there are no border artefacts).  With
    ``support`` = k, each blob is evaluated on its +-k*sigma box only (the
    separable factors make that an outer product).  Elementwise work runs in
    multithreaded torch CPU ops; the result is deterministic.
    """
    import torch

    nz, ny, nx = shape_zyx
    out = torch.zeros(shape_zyx, dtype=torch.float64)
    ox, oy, oz = offset
    for (cx, cy, cz), s, a in zip(centres, sigmas, amps):
        cx, cy, cz = cx + ox, cy + oy, cz + oz
        if support is None:
            x0, x1, y0, y1, z0, z1 = 0, nx, 0, ny, 0, nz
        else:
            r = support * s
            x0, x1 = max(0, int(np.floor(cx - r))), min(nx, int(np.ceil(cx + r)) + 1)
            y0, y1 = max(0, int(np.floor(cy - r))), min(ny, int(np.ceil(cy + r)) + 1)
            z0, z1 = max(0, int(np.floor(cz - r))), min(nz, int(np.ceil(cz + r)) + 1)
            if x0 >= x1 or y0 >= y1 or z0 >= z1:
                continue
        inv = 1.0 / (2.0 * s * s)
        gx = torch.from_numpy(np.exp(-((np.arange(x0, x1) - cx) ** 2) * inv))
        gy = torch.from_numpy(np.exp(-((np.arange(y0, y1) - cy) ** 2) * inv))
        gz = torch.from_numpy(a * np.exp(-((np.arange(z0, z1) - cz) ** 2) * inv))
        out[z0:z1, y0:y1, x0:x1] += gz[:, None, None] * (gy[None, :, None] * gx[None, None, :])
    return out.numpy()


def gen_translation_f32(seed: int = 0, n: int = 64, n_blobs: int = 40,
                        shift=(3, -2, 1), noise: float = 0.02) -> VolumePair:
    """Plain tiny workload: two n^3 float32 blob volumes related by a shift.

    Draw order (one child stream each): blob centres U[0, n)^3 as (x, y, z),
    sigmas U(3, 8), amplitudes U(0.2, 1), ref noise N(0, noise^2), flt noise.
    ``flt(p) = clean(p - shift) + fresh noise``; the expected displacement is
    ``+shift`` wherever it lies inside the search window.
    """
    r_c, r_s, r_a, r_nr, r_nf = _streams(seed, 5)
    centres = r_c.uniform(0.0, n, size=(n_blobs, 3))
    sigmas = r_s.uniform(3.0, 8.0, size=n_blobs)
    amps = r_a.uniform(0.2, 1.0, size=n_blobs)
    shape = (n, n, n)
    ref = _blob_field(shape, centres, sigmas, amps) + r_nr.normal(0.0, noise, size=shape)
    flt = _blob_field(shape, centres, sigmas, amps, offset=tuple(float(v) for v in shift)) \
        + r_nf.normal(0.0, noise, size=shape)
    return VolumePair(ref.astype(np.float32), flt.astype(np.float32), (n, n, n),
                      {"workload": "translation_f32", "seed": seed, "shift": tuple(shift)})


def _sag_field(shape_zyx, n_sags, centre_lo, centre_hi, sigma_lo, sigma_hi, amp_lo, amp_hi, rng):
    """Smooth brain-shift field u(p) = sum_k A_k exp(-|p-c_k|^2 / 2 s_k^2) n_k.

    Returns (ux, uy, uz) as float64 arrays of ``shape_zyx`` and the sag list.
    Draw order: centres (x, y, z), sigmas, peaks, directions (normalised
    Gaussian vectors).
    """
    nz, ny, nx = shape_zyx
    dims = np.array([nx, ny, nz], dtype=np.float64)
    centres = rng.uniform(centre_lo * dims, centre_hi * dims, size=(n_sags, 3))
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=n_sags)
    peaks = rng.uniform(amp_lo, amp_hi, size=n_sags)
    dirs = rng.normal(size=(n_sags, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    import torch

    ux = torch.zeros(shape_zyx, dtype=torch.float64)
    uy = torch.zeros(shape_zyx, dtype=torch.float64)
    uz = torch.zeros(shape_zyx, dtype=torch.float64)
    for (cx, cy, cz), s, a, d in zip(centres, sigmas, peaks, dirs):
        inv = 1.0 / (2.0 * s * s)
        ez = torch.from_numpy(a * np.exp(-((np.arange(nz) - cz) ** 2) * inv))
        ey = torch.from_numpy(np.exp(-((np.arange(ny) - cy) ** 2) * inv))
        ex = torch.from_numpy(np.exp(-((np.arange(nx) - cx) ** 2) * inv))
        g = ez[:, None, None] * (ey[None, :, None] * ex[None, None, :])
        ux.add_(g, alpha=float(d[0]))
        uy.add_(g, alpha=float(d[1]))
        uz.add_(g, alpha=float(d[2]))
        del g
    ux, uy, uz = ux.numpy(), uy.numpy(), uz.numpy()
    sags = [{"centre": c.tolist(), "sigma": float(s), "peak": float(a), "dir": d.tolist()}
            for c, s, a, d in zip(centres, sigmas, peaks, dirs)]
    return (ux, uy, uz), sags


def _warp_trilinear(vol, u, chunk_z: int = 16):
    """flt_clean(p) = trilinear(vol, p - u(p)) with clamp-to-edge sampling."""
    from scipy.ndimage import map_coordinates

    ux, uy, uz = u
    nz, ny, nx = vol.shape
    out = np.empty_like(vol, dtype=np.float64)
    yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                         indexing="ij")
    for z0 in range(0, nz, chunk_z):
        z1 = min(nz, z0 + chunk_z)
        zz = np.arange(z0, z1, dtype=np.float64)[:, None, None]
        cz = np.broadcast_to(zz, (z1 - z0, ny, nx)) - uz[z0:z1]
        cy = yy[None] - uy[z0:z1]
        cx = xx[None] - ux[z0:z1]
        out[z0:z1] = map_coordinates(vol, np.stack([cz, cy, cx]), order=1, mode="nearest")
    return out


def _rician_u16(clean, sigma, rng):
    n1 = rng.normal(0.0, sigma, size=clean.shape)
    n2 = rng.normal(0.0, sigma, size=clean.shape)
    v = np.sqrt((clean + n1) ** 2 + n2 ** 2)
    return np.clip(np.rint(v), 0, U16_MAX12).astype(np.uint16)


def gen_mri_u16(seed: int = 0, dims=(256, 256, 124), class_means=(600.0, 1400.0, 2600.0),
                noise_sigma: float = 40.0, n_sags=None, peak=(4.0, 10.0)) -> VolumePair:
    """MRI-shaped workload: 12-bit uint16 tissue-class volumes and a sag warp.

    Draw order (child streams): label noise N(0, 1); sag count (1-3, unless
    given) then the sag field; ref Rician noise; flt Rician noise.
    Labels: white noise -> Gaussian filter sigma 10 -> thresholds at the 1/3
    and 2/3 quantiles -> class means -> Gaussian sigma 1 (partial volume).
    """
    from scipy.ndimage import gaussian_filter

    nx, ny, nz = dims
    shape = (nz, ny, nx)
    r_lab, r_sag, r_nr, r_nf = _streams(seed, 4)
    smooth = gaussian_filter(r_lab.normal(size=shape), sigma=10.0)
    t1, t2 = np.quantile(smooth, [1.0 / 3.0, 2.0 / 3.0])
    labels = np.where(smooth < t1, 0, np.where(smooth < t2, 1, 2))
    clean = gaussian_filter(np.asarray(class_means)[labels], sigma=1.0)
    k = int(r_sag.integers(1, 4)) if n_sags is None else int(n_sags)
    u, sags = _sag_field(shape, k, 0.25, 0.75, 15.0, 30.0, peak[0], peak[1], r_sag)
    flt_clean = _warp_trilinear(clean, u)
    ref = _rician_u16(clean, noise_sigma, r_nr)
    flt = _rician_u16(flt_clean, noise_sigma, r_nf)
    return VolumePair(ref, flt, tuple(dims),
                      {"workload": "mri_u16", "seed": seed, "sags": sags, "u": u})


def gen_blobs_u16(seed: int = 0, dims=(512, 512, 256), blob_density: float = 40.0 / 64 ** 3,
                  n_sags: int = 3, peak=(4.0, 14.0), noise_frac: float = 0.02) -> VolumePair:
    """Large dense workload: 12-bit uint16 blob volumes warped by sags.

    Blob model as in ``gen_translation_f32`` (sigma U(3, 8), amplitude
    U(0.2, 1)), blob count scaled to the same density per voxel, each blob
    evaluated on its +-4 sigma box.  Clean field normalised by its maximum and
    mapped to 4095 * v; flt is the trilinear sag warp of the clean field; each
    volume gets fresh N(0, (noise_frac * 4095)^2) noise, then round-half-even,
    clip to [0, 4095], uint16.
    Draw order (child streams): centres, sigmas, amplitudes, sag field, ref
    noise, flt noise.
    """
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    n_blobs = int(round(blob_density * nx * ny * nz))
    r_c, r_s, r_a, r_sag, r_nr, r_nf = _streams(seed, 6)
    centres = r_c.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    sigmas = r_s.uniform(3.0, 8.0, size=n_blobs)
    amps = r_a.uniform(0.2, 1.0, size=n_blobs)
    clean = _blob_field(shape, centres, sigmas, amps, support=4.0)
    clean *= U16_MAX12 / clean.max()
    u, sags = _sag_field(shape, n_sags, 0.25, 0.75, 15.0, 30.0, peak[0], peak[1], r_sag)
    flt_clean = _warp_trilinear(clean, u)
    sd = noise_frac * U16_MAX12

    def q(c, rng):
        return np.clip(np.rint(c + rng.normal(0.0, sd, size=c.shape)), 0, U16_MAX12).astype(np.uint16)

    return VolumePair(q(clean, r_nr), q(flt_clean, r_nf), tuple(dims),
                      {"workload": "blobs_u16", "seed": seed, "n_blobs": n_blobs, "sags": sags,
                       "u": u})


def gen_random(seed: int, dims, dtype: str = "u16", smooth: float = 0.0) -> VolumePair:
    """Tiny random pair for brute-force parity (non-cubic dims welcome).

    u16: independent uniform integers in [0, 4095]; f32: N(0, 1).  With
    ``smooth`` > 0 both volumes are Gaussian-filtered first (u16 re-quantised),
    which gives NCC surfaces with a clear peak.  ``flt`` is an independent
    draw, so every shift is a generic (non-tied) candidate.
    """
    from scipy.ndimage import gaussian_filter

    nx, ny, nz = dims
    shape = (nz, ny, nx)
    r1, r2 = _streams(seed, 2)
    if dtype == "u16":
        a = r1.integers(0, U16_MAX12 + 1, size=shape).astype(np.float64)
        b = r2.integers(0, U16_MAX12 + 1, size=shape).astype(np.float64)
        if smooth > 0:
            a = gaussian_filter(a, smooth)
            b = gaussian_filter(b, smooth)
        return VolumePair(np.clip(np.rint(a), 0, U16_MAX12).astype(np.uint16),
                          np.clip(np.rint(b), 0, U16_MAX12).astype(np.uint16), tuple(dims),
                          {"workload": "random_u16", "seed": seed})
    a = r1.normal(size=shape)
    b = r2.normal(size=shape)
    if smooth > 0:
        a = gaussian_filter(a, smooth)
        b = gaussian_filter(b, smooth)
    return VolumePair(a.astype(np.float32), b.astype(np.float32), tuple(dims),
                      {"workload": "random_f32", "seed": seed})


def gen_param_sets(n: int = 32, seed: int = 1, blocks=(5, 7, 9), windows=(5, 8, 12),
                   fractions=(0.05, 0.1, 0.25, 0.5)):
    """Parameter sets of the batched parametric search: (block, window,
    stride, fraction) with block, window and fraction drawn uniformly from
    the given choices and the grid stride equal to the block size."""
    (r,) = _streams(seed, 1)
    b = r.choice(np.asarray(blocks), size=n)
    w = r.choice(np.asarray(windows), size=n)
    f = r.choice(np.asarray(fractions, dtype=np.float64), size=n)
    return [(int(b[i]), int(w[i]), int(b[i]), float(f[i])) for i in range(n)]


SERVING_SIZES = ((128, 128, 128), (192, 192, 96), (256, 256, 124), (384, 384, 160))


def gen_serving_requests(n: int, seed: int = 4, rate_hz: float = 4.0, pool_seeds: int = 2):
    """Registration requests for the serving workload: Poisson arrivals at
    `rate_hz` (exponential gaps), volume size uniform over SERVING_SIZES,
    window uniform in 5..15, block uniform in {5, 7, 9} (grid stride = block),
    fraction uniform in [0.1, 0.3].  Each request names the volume pair it
    registers by (size, volume seed), the seed drawn from `pool_seeds` values
    so a benchmark can generate the pairs once (gen_blobs_u16 at that size)."""
    (r,) = _streams(seed, 1)
    gaps = r.exponential(1.0 / rate_hz, size=n)
    out = []
    t = 0.0
    for i in range(n):
        t += float(gaps[i])
        b = int(r.choice([5, 7, 9]))
        out.append({"arrival_s": t, "size": SERVING_SIZES[int(r.integers(0, len(SERVING_SIZES)))],
                    "block": b, "stride": b, "window": int(r.integers(5, 16)),
                    "fraction": float(r.uniform(0.1, 0.3)),
                    "volume_seed": int(r.integers(0, pool_seeds))})
    return out
