"""Seeded permeability generators (log K on a Cartesian grid, x fastest).

Arrays are returned with numpy shape ``ncell[::-1]`` (``(ny, nx)`` or
``(nz, ny, nx)``) so that ``arr.ravel()`` is the x-fastest cell order used by
every consumer.

* ``gaussian_logk``: stationary Gaussian field with squared-exponential
  covariance ``sigma2 * exp(-sum_a (r_a / ell_a)^2)``, sampled by circulant
  embedding on a torus twice the domain size (negative spectral weights are
  clipped to zero).  Stands in for the heterogeneous benchmark field of the
  paper (Section 5), which is not available.
* ``channel_logk``: binary channelised field (background 1, channels
  ``contrast``), sinusoidal channel centrelines along x.
* ``layered_logk``: anisotropic Gaussian field clipped to a contrast bound.
"""
import numpy as np


def gaussian_logk(ncell, h, sigma2, corr, seed):
    ncell = tuple(int(n) for n in ncell)
    d = len(ncell)
    corr = np.broadcast_to(np.asarray(corr, dtype=np.float64), (d,))
    hs = np.broadcast_to(np.asarray(h, dtype=np.float64), (d,))
    rng = np.random.Generator(np.random.PCG64(seed))
    # torus twice the size of the domain along every axis (numpy order: last axis = x)
    tshape = tuple(2 * n for n in ncell[::-1])
    grids = []
    for ax_np, m in enumerate(tshape):
        a = d - 1 - ax_np  # physical axis
        k = np.arange(m)
        r = np.minimum(k, m - k) * hs[a] / corr[a]
        shp = [1] * d
        shp[ax_np] = m
        grids.append((r ** 2).reshape(shp))
    r2 = sum(grids)
    cov = sigma2 * np.exp(-r2)
    lam = np.real(np.fft.fftn(cov))
    lam = np.clip(lam, 0.0, None)
    white = rng.standard_normal(tshape) + 1j * rng.standard_normal(tshape)
    field = np.fft.ifftn(np.sqrt(lam) * white) * np.sqrt(np.prod(tshape))
    y = np.real(field)[tuple(slice(0, n) for n in ncell[::-1])]
    return np.ascontiguousarray(y, dtype=np.float64)


def channel_logk(nx, ny, seed, n_channels=30, contrast=1e4,
                 width_cells=(4, 12), amp=(0.02, 0.08), wavelength=(0.25, 1.0)):
    rng = np.random.Generator(np.random.PCG64(seed))
    hx = 1.0 / nx
    hy = 1.0 / ny
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    mask = np.zeros((ny, nx), dtype=bool)
    for _ in range(n_channels):
        y0 = rng.uniform(0.0, 1.0)
        a = rng.uniform(*amp)
        lam = rng.uniform(*wavelength)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        w = rng.integers(width_cells[0], width_cells[1] + 1)
        centre = y0 + a * np.sin(2.0 * np.pi * xc / lam + ph)
        mask |= np.abs(yc[:, None] - centre[None, :]) <= 0.5 * w * hy
    return np.where(mask, np.log(contrast), 0.0).astype(np.float64)


def layered_logk(ncell, h, sigma2, corr, seed, contrast):
    y = gaussian_logk(ncell, h, sigma2, corr, seed)
    bound = 0.5 * np.log(contrast)
    return np.clip(y, -bound, bound)
