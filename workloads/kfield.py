"""Seeded lognormal hydraulic-conductivity fields.

The heterogeneous aquifer of the paper's first test case (section "Synthetic
test cases", Table 1) is built from one standard Gaussian field Y with an
isotropic exponential covariance of unit variance, and K = exp(sigma_Y * Y).
Here Y is drawn by circulant embedding on a padded periodic grid (negative
eigenvalues of the embedding are clipped to zero), cropped to the model grid,
and standardised to sample mean 0 and sample variance 1. K = K_g * exp(sigma*Y)
with K_g the geometric mean.

Correlation lengths are given in cell units on every axis.  Only input
generation lives here: nothing in this module touches particle tracking.
"""
from __future__ import annotations

import numpy as np


def _embed_size(n: int, lam: float) -> int:
    m = max(2 * n, n + int(np.ceil(4.0 * lam)))
    return m + (m % 2)


def gaussian_field(shape, corr_len: float, rng: np.random.Generator) -> np.ndarray:
    """Standardised Gaussian field Y[nz, ny, nx] with covariance exp(-|h|/corr_len)."""
    nz, ny, nx = (int(s) for s in shape)
    mz, my, mx = (_embed_size(n, corr_len) for n in (nz, ny, nx))
    if nz == 1:
        mz = 1      # a two-dimensional field: no embedding along the unused axis

    def lag(m):
        a = np.arange(m, dtype=np.float64)
        return np.minimum(a, m - a)

    hz, hy, hx = lag(mz), lag(my), lag(mx)
    h = np.sqrt(hz[:, None, None] ** 2 + hy[None, :, None] ** 2 + hx[None, None, :] ** 2)
    cov = np.exp(-h / float(corr_len))
    eig = np.fft.rfftn(cov).real
    np.maximum(eig, 0.0, out=eig)
    z = rng.standard_normal((mz, my, mx))
    y = np.fft.irfftn(np.sqrt(eig) * np.fft.rfftn(z), s=(mz, my, mx), axes=(0, 1, 2))
    y = np.ascontiguousarray(y[:nz, :ny, :nx])
    y -= y.mean()
    sd = y.std()
    if sd > 0:
        y /= sd
    return y


def lognormal_k(shape, k_geo: float, sigma2: float, corr_len: float, seed: int) -> np.ndarray:
    """K[nz, ny, nx] = k_geo * exp(sqrt(sigma2) * Y), Y standardised (seeded PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y = gaussian_field(shape, corr_len, rng)
    return k_geo * np.exp(np.sqrt(sigma2) * y)
