"""Pins of the oracle's transforms and spectral helpers: a direct DFT sum
written out on a tiny grid, Parseval, and the derivative convention."""

import numpy as np

from oracle import spectral as sp


def test_forward_matches_direct_dft():
    rng = np.random.default_rng(12)
    shape = (4, 3, 6)
    f = rng.standard_normal(shape)
    got = sp.forward(f)
    x = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), axis=-1)
    for m in np.ndindex(*shape):
        phase = sum(2 * np.pi * m[a] * x[..., a] / shape[a] for a in range(3))
        ref = np.sum(f * np.exp(-1j * phase))
        assert abs(got[m] - ref) <= 1e-12


def test_inverse_and_parseval():
    rng = np.random.default_rng(13)
    f = rng.standard_normal((8, 4, 16))
    F = sp.forward(f)
    assert np.max(np.abs(sp.inverse(F) - f)) <= 1e-14
    assert abs(np.sum(np.abs(F) ** 2) / f.size - np.sum(f * f)) <= 1e-10


def test_derivative_is_plus_ik():
    """d/dx of sin(k0 x) is k0 cos(k0 x): multiplying the spectrum by +i k
    and transforming back gives it (the Fourier convention of the update)."""
    shape, spacing = (32, 4, 4), (0.5, 1.0, 1.0)
    k = sp.wavevectors(shape, spacing)
    x = np.arange(shape[0]) * spacing[0]
    k0 = 2 * np.pi * 3 / (shape[0] * spacing[0])
    f = np.broadcast_to(np.sin(k0 * x)[:, None, None], shape)
    d = sp.inverse(1j * k[0] * sp.forward(f))
    assert np.max(np.abs(d - np.broadcast_to((k0 * np.cos(k0 * x))[:, None, None], shape))) <= 1e-12


def test_held_zero_mask_counts():
    m = sp.held_zero_mask((4, 6, 8))
    # k = 0 plus the three Nyquist planes (inclusion-exclusion)
    n = 1 + (6 * 8 + 4 * 8 + 4 * 6) - (8 + 6 + 4) + 1
    assert int(m.sum()) == n
