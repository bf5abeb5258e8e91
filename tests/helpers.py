"""Independent test-side helpers: literal dense DFTs and norms.

Nothing here calls the oracle or the product; these are the brute-force
definitions the oracle is pinned against."""
from __future__ import annotations

import numpy as np


def relerr(x, y) -> float:
    x = np.asarray(x)
    y = np.asarray(y)
    d = np.linalg.norm((x - y).ravel())
    n = np.linalg.norm(y.ravel())
    return float(d / n) if n > 0 else float(d)


def relerr_per_band(x, y) -> np.ndarray:
    x = np.asarray(x)
    y = np.asarray(y)
    nb = x.shape[0]
    d = np.linalg.norm((x - y).reshape(nb, -1), axis=1)
    n = np.linalg.norm(y.reshape(nb, -1), axis=1)
    return d / np.where(n > 0, n, 1.0)


def grid_points(grid):
    """All grid indices j = (j1, j2, j3) in [N3][N2][N1] storage order."""
    N1, N2, N3 = grid
    j3, j2, j1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    return np.stack([j1.ravel(), j2.ravel(), j3.ravel()], axis=1)


def phase_matrix(grid, gvecs, sign=-1):
    """E[j, g] = exp(sign 2 pi i sum_i g_i j_i / N_i), dense."""
    N = np.asarray(grid, dtype=np.float64)
    J = grid_points(grid).astype(np.float64)
    G = np.asarray(gvecs, dtype=np.float64)
    theta = 2.0 * np.pi * (J / N) @ G.T
    return np.exp(sign * 1j * theta)


def dense_dft_matrix(grid, sign=-1):
    """The literal (N^3)^2 3-D DFT matrix over every grid frequency m."""
    return phase_matrix(grid, grid_points(grid), sign)


def scatter(grid, hkl, c):
    N1, N2, N3 = grid
    cube = np.zeros((c.shape[0], N3, N2, N1), dtype=np.complex128)
    h = np.mod(hkl[:, 0], N1)
    k = np.mod(hkl[:, 1], N2)
    l = np.mod(hkl[:, 2], N3)
    cube[:, l, k, h] = c
    return cube


def gather(grid, hkl, cube):
    N1, N2, N3 = grid
    return cube[:, np.mod(hkl[:, 2], N3), np.mod(hkl[:, 1], N2), np.mod(hkl[:, 0], N1)]


def brute_apply_dense(grid, hkl, c, V, sign=-1):
    """out = gather((1/N) D^H (V . (D scatter(c)))) with the literal dense matrix."""
    D = dense_dft_matrix(grid, sign)
    N = D.shape[0]
    cube = scatter(grid, hkl, c).reshape(c.shape[0], N)
    psi = cube @ D.T
    prod = psi * np.asarray(V).reshape(1, N)
    back = (prod @ np.conj(D)) / N
    return gather(grid, hkl, back.reshape((c.shape[0],) + tuple(reversed(grid))))


def direct_sphere_g2r(grid, hkl, c, sign=-1, chunk=4096):
    """psi(j) = sum_{g in S} c(g) exp(sign 2 pi i g.j/N), O(npw N) by direct sums."""
    J = grid_points(grid)
    out = np.empty((c.shape[0], J.shape[0]), dtype=np.complex128)
    for s in range(0, J.shape[0], chunk):
        E = phase_matrix_rows(grid, J[s:s + chunk], hkl, sign)
        out[:, s:s + chunk] = c @ E.T
    return out


def direct_sphere_r2g(grid, hkl, psi_flat, sign=-1, chunk=4096):
    """c(g) = (1/N) sum_j exp(-sign 2 pi i g.j/N) psi(j)."""
    J = grid_points(grid)
    N = J.shape[0]
    acc = np.zeros((psi_flat.shape[0], hkl.shape[0]), dtype=np.complex128)
    for s in range(0, N, chunk):
        E = phase_matrix_rows(grid, J[s:s + chunk], hkl, -sign)
        acc += psi_flat[:, s:s + chunk] @ E
    return acc / N


def phase_matrix_rows(grid, J, gvecs, sign):
    N = np.asarray(grid, dtype=np.float64)
    theta = 2.0 * np.pi * (np.asarray(J, dtype=np.float64) / N) @ np.asarray(gvecs, dtype=np.float64).T
    return np.exp(sign * 1j * theta)


def isqrt_count(R2: int):
    """Closed-form integer recount of a centred sphere h^2+k^2+l^2 <= R2:
    (npw, nsticks, count range) with npw = sum_{h^2+k^2<=R2} (2 isqrt(R2-h^2-k^2) + 1)."""
    import math
    R = math.isqrt(R2)
    npw = 0
    nst = 0
    cmin, cmax = 10 ** 9, 0
    for h in range(-R, R + 1):
        for k in range(-R, R + 1):
            r = R2 - h * h - k * k
            if r >= 0:
                cnt = 2 * math.isqrt(r) + 1
                npw += cnt
                nst += 1
                cmin = min(cmin, cnt)
                cmax = max(cmax, cnt)
    return npw, nst, (cmin, cmax)
