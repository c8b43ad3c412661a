"""Seeded input generators: determinism, value ranges, deformation sanity."""

import numpy as np
import pytest

from paper_2308_10868_amd import synth


def test_translation_deterministic_and_shaped():
    a = synth.gen_translation_f32(seed=0)
    b = synth.gen_translation_f32(seed=0)
    c = synth.gen_translation_f32(seed=1)
    assert a.ref.shape == (64, 64, 64) and a.ref.dtype == np.float32
    assert synth.sha256(a.ref) == synth.sha256(b.ref) and synth.sha256(a.flt) == synth.sha256(b.flt)
    assert synth.sha256(a.ref) != synth.sha256(c.ref)
    assert -0.2 < a.ref.min() and a.ref.max() < 3.0


def test_translation_is_a_shift_without_noise():
    p = synth.gen_translation_f32(seed=3, n=32, n_blobs=10, shift=(3, -2, 1), noise=0.0)
    # flt(p) = ref(p - s): compare the overlapping region
    a = p.ref[0:31, 2:32, 0:29]    # z 0..30, y 2..31, x 0..28
    b = p.flt[1:32, 0:30, 3:32]    # z+1, y-2, x+3
    assert np.max(np.abs(a - b)) < 1e-6


@pytest.mark.slow
def test_mri_u16_ranges_and_fold_free():
    p = synth.gen_mri_u16(seed=0, dims=(96, 80, 48))
    assert p.ref.dtype == np.uint16 and p.ref.shape == (48, 80, 96)
    assert p.ref.max() <= 4095 and p.flt.max() <= 4095
    ux, uy, uz = p.meta["u"]
    # Jacobian of the displacement stays well below 1 (no folding)
    g = max(np.abs(np.gradient(c, axis=ax)).max() for c in (ux, uy, uz) for ax in range(3))
    assert g < 1.0
    q = synth.gen_mri_u16(seed=0, dims=(96, 80, 48))
    assert synth.sha256(p.flt) == synth.sha256(q.flt)


def test_blobs_u16_small():
    p = synth.gen_blobs_u16(seed=0, dims=(48, 40, 32))
    assert p.ref.dtype == np.uint16 and p.ref.shape == (32, 40, 48)
    assert p.ref.max() <= 4095 and p.flt.max() <= 4095 and p.ref.max() > 3000
    assert p.meta["n_blobs"] == round(40 * 48 * 40 * 32 / 64 ** 3)


def test_random_pairs():
    p = synth.gen_random(1, (10, 9, 8), "u16")
    assert p.ref.shape == (8, 9, 10) and p.ref.max() <= 4095
    f = synth.gen_random(1, (10, 9, 8), "f32", smooth=1.0)
    assert f.ref.dtype == np.float32
