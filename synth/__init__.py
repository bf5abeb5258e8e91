"""Seeded synthetic inputs, shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method itself (no sphere test, no
transform): callers pass the sphere's Miller indices in, and the generator
only draws random numbers and shapes them.

Recipe (all in grid-index units):

* coefficients: ``x = default_rng(1000 + ik).standard_normal((nb, npw, 2))``,
  ``c = (x[...,0] + 1j x[...,1]) / (1 + |g + kappa|^2)`` where
  ``|g + kappa|^2 = sum_i (g_i + kappa_i)^2``;
* potential: ``default_rng(2000)``; ``V(j) = 0.5 + sum_m A_m exp(-d^2/(2 sigma^2))``
  with sigma = 2, ``A_m ~ U[0.5, 1.5]``, centres ``U[0, N_i)`` per axis and d the
  minimum-image periodic distance; stored [N3][N2][N1], x fastest;
* band weights: ``default_rng(3000).uniform(0, 2, nb)``.
"""
from __future__ import annotations

import numpy as np


def coefficients(hkl, nbands: int, kpt=(0.0, 0.0, 0.0), ik: int = 0) -> np.ndarray:
    hkl = np.asarray(hkl, dtype=np.float64)
    rng = np.random.default_rng(1000 + ik)
    x = rng.standard_normal((nbands, hkl.shape[0], 2))
    f = hkl + np.asarray(kpt, dtype=np.float64)
    w = 1.0 / (1.0 + np.einsum("ij,ij->i", f, f))
    return (x[..., 0] + 1j * x[..., 1]) * w[None, :]


def potential(grid, ngauss: int, sigma: float = 2.0, seed: int = 2000) -> np.ndarray:
    N1, N2, N3 = (int(g) for g in grid)
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.5, ngauss)
    centres = np.stack([rng.uniform(0, N1, ngauss), rng.uniform(0, N2, ngauss),
                        rng.uniform(0, N3, ngauss)], axis=1)
    V = np.full((N3, N2, N1), 0.5, dtype=np.float64)
    jx = np.arange(N1, dtype=np.float64)
    jy = np.arange(N2, dtype=np.float64)
    jz = np.arange(N3, dtype=np.float64)

    def mind2(j, c, n):
        d = np.abs(j - c)
        d = np.minimum(d, n - d)
        return d * d

    for m in range(ngauss):
        ex = np.exp(-mind2(jx, centres[m, 0], N1) / (2 * sigma * sigma))
        ey = np.exp(-mind2(jy, centres[m, 1], N2) / (2 * sigma * sigma))
        ez = np.exp(-mind2(jz, centres[m, 2], N3) / (2 * sigma * sigma))
        V += amp[m] * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    return V


def band_weights(nbands: int, seed: int = 3000) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 2.0, nbands)


def cubic_cell(scale: float = 2.0 * np.pi) -> np.ndarray:
    """Cell rows a1, a2, a3 = scale * I; 2 pi I gives b_i = e_i (grid units)."""
    return np.eye(3) * scale


def ecut_for_radius(R: float) -> float:
    """E_cut such that sqrt(2 E_cut) = R for the 2 pi I cell."""
    return 0.5 * R * R


# Named workloads (grid, radius in grid units, bands, Gaussians in V).
WORKLOADS = {
    "c1_24": dict(grid=(24, 24, 24), R=6.0, nbands=8, ngauss=4),
    "c2_96": dict(grid=(96, 96, 96), R=24.0, nbands=256, ngauss=32),
    "c5_128": dict(grid=(128, 128, 128), R=32.0, nbands=512, ngauss=32),
    "m0_80": dict(grid=(80, 80, 80), R=float(np.sqrt(413.0)), nbands=1001, ngauss=32),
}

# Several k-points on one orthorhombic grid: spheres of radius 0.25 min(grid)
# shifted by k (uneven plane-wave counts) with uneven band counts.
BATCH_WORKLOADS = {
    "c4_kpts": dict(grid=(72, 96, 128), R=18.0,
                    kpts=((0.0, 0.0, 0.0), (0.25, 0.0, 0.0), (0.25, 0.25, 0.0),
                          (0.25, 0.25, 0.25)),
                    nbands=(64, 128, 256, 512), ngauss=32),
    # many k-points with few bands each: the case where one launch over all of
    # them fills the device and separate per-k launches do not
    "small_kpts": dict(grid=(72, 96, 128), R=18.0,
                       kpts=((0.0, 0.0, 0.0), (0.25, 0.0, 0.0), (0.25, 0.25, 0.0),
                             (0.25, 0.25, 0.25), (0.5, 0.0, 0.0), (0.5, 0.5, 0.0),
                             (0.5, 0.5, 0.5), (0.25, 0.5, 0.0)),
                       nbands=(2, 4, 6, 8, 2, 4, 6, 8), ngauss=32),
}
