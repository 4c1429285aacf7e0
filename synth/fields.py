"""Seeded density fields on an element grid.

Arrays are shaped ``(nz, ny, nx)`` so that a C-order flatten gives the
element index ``e = i + nx * (j + ny * k)`` (x fastest).  All generators use
``numpy.random.default_rng(seed)`` (PCG64).
"""

from __future__ import annotations

import numpy as np


def uniform_iid(nx: int, ny: int, nz: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nz, ny, nx))


def smoothed_field(nx: int, ny: int, nz: int, sigma: float, lo: float, hi: float,
                   seed: int) -> np.ndarray:
    """Standard normal noise per element, Gaussian-smoothed with standard
    deviation ``sigma`` voxels (periodic wrap), min-max mapped to [lo, hi]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    z = rng.standard_normal(size=(nz, ny, nx))
    s = gaussian_filter(z, sigma=sigma, mode="wrap")
    s = (s - s.min()) / max(s.max() - s.min(), 1e-300)
    return lo + (hi - lo) * s


def thresholded_field(nx: int, ny: int, nz: int, sigma: float, lo: float, hi: float,
                      seed: int, frac: float = 0.5) -> np.ndarray:
    """Near-binary variant: the smoothed field thresholded at its ``frac``
    quantile into {lo, hi}.  Mimics late-iteration density contrast."""
    s = smoothed_field(nx, ny, nz, sigma, 0.0, 1.0, seed)
    t = np.quantile(s, 1.0 - frac)
    return np.where(s >= t, hi, lo)


def perturb(field: np.ndarray, amount: float, seed: int, lo: float = 1e-3,
            hi: float = 1.0) -> np.ndarray:
    """Add a seeded uniform perturbation of mean absolute size ``amount``
    (in density units) and clip to [lo, hi]."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-2.0 * amount, 2.0 * amount, size=field.shape)
    return np.clip(field + d, lo, hi)


def smooth_perturb(field: np.ndarray, amount: float, seed: int, sigma: float = 2.0,
                   lo: float = 1e-3, hi: float = 1.0) -> np.ndarray:
    """Add a seeded smoothed perturbation (standard normal noise, Gaussian-
    smoothed with ``sigma`` voxels, periodic wrap) scaled to mean absolute
    size ``amount`` (in density units) and clip to [lo, hi]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    d = gaussian_filter(rng.standard_normal(field.shape), sigma, mode="wrap")
    d *= amount / max(float(np.mean(np.abs(d))), 1e-300)
    return np.clip(field + d, lo, hi)
