"""Seeded random test vectors."""

from __future__ import annotations

import numpy as np


def complex_gaussian(shape, seed: int = 12345, rng: np.random.Generator | None = None):
    """complex128 array with independent N(0,1) real and imaginary parts."""
    if rng is None:
        rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im
