"""CPU oracle for the local-potential action on plane-wave wave functions.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product library never does.  It
shares no code with the GPU path.

Two parts:

* ``liboracle_vloc.so`` (``vloc_oracle.c``): FP64 plain mixed-radix FFTs on the
  full cube; sphere enumeration; G->r, r->G and the full V_loc application
  (paper Sec. 2, eqs. 2-3 and the operator paragraph after eq. 3).
* pure-Python/numpy helpers written independently of the C code: sphere
  enumeration, the z-stick table of the sphere (the compact FFT's first-pass
  columns, Sec. 4.3), and the greedy "sort by plane-wave count, deal round
  robin" column distribution (Sec. 3.2).

Conventions (the readings are listed with their reasons in the design notes):
sign -1 on G->r (eq. 2), no normalisation G->r, 1/N on r->G, cutoff
``|k+G|^2 <= 2 Ecut (1 + 1e-12)``, canonical G order lexicographic on signed
(h, k, l), real-space arrays [N3][N2][N1] with x fastest, k in reduced
coordinates of the reciprocal basis.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle_vloc.so")
_lib = None


def lib():
    """Load (building with gcc if absent) the C oracle."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    L.oracle_fft1d.argtypes = [dp, dp, ctypes.c_long, ctypes.c_int]
    L.oracle_fft1d.restype = ctypes.c_int
    L.oracle_sphere.argtypes = [dp, ctypes.c_double, dp, ctypes.POINTER(ctypes.c_int32), ctypes.c_long]
    L.oracle_sphere.restype = ctypes.c_long
    for name in ("oracle_g2r", "oracle_r2g"):
        f = getattr(L, name)
        f.argtypes = [ip, dp, ctypes.c_double, dp, ctypes.c_int, dp, ctypes.c_long, dp, ctypes.c_int]
        f.restype = ctypes.c_int
    L.oracle_apply.argtypes = [ip, dp, ctypes.c_double, dp, ctypes.c_int, dp, ctypes.c_long,
                               dp, dp, ctypes.c_int]
    L.oracle_apply.restype = ctypes.c_int
    L.oracle_max_threads.argtypes = []
    L.oracle_max_threads.restype = ctypes.c_int
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cell(cell):
    return np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))


def _k(k):
    return np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(3))


def _grid(grid):
    return (ctypes.c_int * 3)(*[int(g) for g in grid])


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# ----------------------------------------------------------------- C oracle

def fft1d(x, sign: int) -> np.ndarray:
    """X[k] = sum_n x[n] exp(sign 2 pi i n k / L), FP64, by the C oracle."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    out = np.empty_like(x)
    rc = lib().oracle_fft1d(_dp(x.view(np.float64)), _dp(out.view(np.float64)), x.size, int(sign))
    if rc != 0:
        raise ValueError("oracle_fft1d failed")
    return out


def sphere_c(cell, ecut: float, k=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Sphere points (npw, 3) int32 from the C oracle, canonical order."""
    c, kk = _cell(cell), _k(k)
    n = lib().oracle_sphere(_dp(c), float(ecut), _dp(kk), None, 0)
    if n < 0:
        raise ValueError("bad cell or cutoff")
    hkl = np.zeros((max(n, 1), 3), dtype=np.int32)
    lib().oracle_sphere(_dp(c), float(ecut), _dp(kk),
                        hkl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n)
    return hkl[:n]


def g2r(grid, cell, ecut, k, c, sign: int = -1, nthreads: int = 0) -> np.ndarray:
    """psi[b] on the full grid, shape (nb, N3, N2, N1) complex128."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
    nb = c.shape[0]
    N1, N2, N3 = (int(g) for g in grid)
    psi = np.empty((nb, N3, N2, N1), dtype=np.complex128)
    rc = lib().oracle_g2r(_grid(grid), _dp(_cell(cell)), float(ecut), _dp(_k(k)), int(sign),
                          _dp(c.view(np.float64)), nb, _dp(psi.view(np.float64)), nthreads)
    if rc != 0:
        raise ValueError(f"oracle_g2r failed ({rc})")
    return psi


def r2g(grid, cell, ecut, k, psi, sign: int = -1, nthreads: int = 0) -> np.ndarray:
    psi = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    nb = psi.shape[0]
    npw = sphere_c(cell, ecut, k).shape[0]
    out = np.empty((nb, npw), dtype=np.complex128)
    rc = lib().oracle_r2g(_grid(grid), _dp(_cell(cell)), float(ecut), _dp(_k(k)), int(sign),
                          _dp(psi.view(np.float64)), nb, _dp(out.view(np.float64)), nthreads)
    if rc != 0:
        raise ValueError(f"oracle_r2g failed ({rc})")
    return out


def apply(grid, cell, ecut, k, c, V, sign: int = -1, nthreads: int = 0) -> np.ndarray:
    """out[b] = V_loc applied to band b, shape (nb, npw) complex128."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float64))
    N1, N2, N3 = (int(g) for g in grid)
    if V.size != N1 * N2 * N3:
        raise ValueError("V must hold N3*N2*N1 values")
    nb = c.shape[0]
    out = np.empty_like(c)
    rc = lib().oracle_apply(_grid(grid), _dp(_cell(cell)), float(ecut), _dp(_k(k)), int(sign),
                            _dp(c.view(np.float64)), nb, _dp(V), _dp(out.view(np.float64)),
                            nthreads)
    if rc != 0:
        raise ValueError(f"oracle_apply failed ({rc})")
    return out


# ------------------------------------------------- independent Python helpers

def reciprocal(cell) -> np.ndarray:
    """Rows b_j with a_i . b_j = 2 pi delta_ij."""
    A = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    return 2.0 * math.pi * np.linalg.inv(A).T


def sphere_py(cell, ecut: float, k=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Sphere |k+G|^2 <= 2 Ecut (1+1e-12) (eq. 3, non-strict reading), canonical
    lexicographic (h, k, l) order, written with numpy independently of the C code."""
    A = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    B = reciprocal(A)
    kk = np.asarray(k, dtype=np.float64)
    gcut = math.sqrt(2.0 * ecut)
    ranges = []
    for i in range(3):
        ext = gcut * np.linalg.norm(A[i]) / (2.0 * math.pi)
        ranges.append(np.arange(math.floor(-ext - kk[i]) - 1, math.ceil(ext - kk[i]) + 2))
    H, K, L = np.meshgrid(*ranges, indexing="ij")
    f = np.stack([H.ravel(), K.ravel(), L.ravel()], axis=1).astype(np.float64) + kk
    G = f @ B
    keep = np.einsum("ij,ij->i", G, G) <= 2.0 * ecut * (1.0 + 1e-12)
    pts = np.stack([H.ravel(), K.ravel(), L.ravel()], axis=1)[keep]
    order = np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0]))
    return pts[order].astype(np.int32)


def sticks(hkl) -> np.ndarray:
    """z-stick table of a canonically ordered sphere: rows (h, k, offset, count, lmin).

    A stick is the set of sphere points sharing (h, k); in canonical order each
    stick is one contiguous run with l ascending (the sphere is convex, so the
    run has no holes).  These are the columns that meet the sphere, i.e. the
    first-pass columns of the compact 3-D FFT (Sec. 4.3)."""
    hkl = np.asarray(hkl)
    rows = []
    i = 0
    n = hkl.shape[0]
    while i < n:
        j = i
        while j < n and hkl[j, 0] == hkl[i, 0] and hkl[j, 1] == hkl[i, 1]:
            j += 1
        ls = hkl[i:j, 2]
        if not np.array_equal(ls, np.arange(ls[0], ls[0] + (j - i))):
            raise AssertionError("stick is not a contiguous l-ascending run")
        rows.append((int(hkl[i, 0]), int(hkl[i, 1]), i, j - i, int(ls[0])))
        i = j
    return np.array(rows, dtype=np.int64).reshape(-1, 5)


def greedy_deal(counts, ngroups: int, mode: str = "cyclic"):
    """Greedy column distribution (Sec. 3.2): sort columns by descending
    plane-wave count and deal them to `ngroups` groups in turn.

    Reading of the unstated details: ties keep canonical order (stable sort),
    and "round robin" is a plain cyclic deal g = rank mod ngroups.  ``snake``
    reverses every other pass; ``unsorted`` deals in canonical order (the
    no-balancing baseline).  Returns (group_of_column, order) where ``order``
    lists columns by rank."""
    counts = np.asarray(counts, dtype=np.int64)
    n = counts.size
    if mode == "unsorted":
        order = np.arange(n)
    else:
        order = sorted(range(n), key=lambda i: (-int(counts[i]), i))
        order = np.asarray(order, dtype=np.int64)
    group = np.empty(n, dtype=np.int64)
    for r, col in enumerate(order):
        g = r % ngroups
        if mode == "snake" and (r // ngroups) % 2 == 1:
            g = ngroups - 1 - g
        group[col] = g
    return group, order


def group_loads(counts, group, ngroups: int) -> np.ndarray:
    loads = np.zeros(ngroups, dtype=np.int64)
    np.add.at(loads, np.asarray(group), np.asarray(counts, dtype=np.int64))
    return loads


# ------------------------------------------------------------ real (gamma) mode
# Sec. 4.3, last paragraph: at the Gamma point psi_n is real in space, so
# c_n(-G) = conj(c_n(G)) and half of reciprocal space suffices.  The half
# sphere kept is H = {h > 0} u {h = 0, k > 0} u {h = k = 0, l >= 0}, in the
# canonical order restricted to H; Im c(0) is taken as zero.


def half_mask(hkl) -> np.ndarray:
    """True for the points of the full sphere that belong to H."""
    h, k, l = (np.asarray(hkl)[:, i] for i in range(3))
    return (h > 0) | ((h == 0) & (k > 0)) | ((h == 0) & (k == 0) & (l >= 0))


def expand_half(hkl_full, c_half) -> np.ndarray:
    """Full-sphere coefficients from half-sphere ones: c(g) on H, conj c(-g)
    off H, real c(0)."""
    hkl_full = np.asarray(hkl_full)
    m = half_mask(hkl_full)
    c_half = np.atleast_2d(np.asarray(c_half, dtype=np.complex128))
    full = np.zeros((c_half.shape[0], hkl_full.shape[0]), dtype=np.complex128)
    full[:, m] = c_half
    index = {tuple(g): i for i, g in enumerate(hkl_full.tolist())}
    for i in np.nonzero(~m)[0]:
        j = index[tuple((-hkl_full[i]).tolist())]
        full[:, i] = np.conj(full[:, j])
    z = np.nonzero((hkl_full == 0).all(axis=1))[0]
    full[:, z] = full[:, z].real
    return full


def apply_gamma(grid, cell, ecut, c_half, V, nthreads: int = 0) -> np.ndarray:
    """V_loc on half-sphere coefficients: expand, apply the full operator,
    keep H."""
    hkl = sphere_py(cell, ecut)
    full = expand_half(hkl, c_half)
    out = apply(grid, cell, ecut, (0.0, 0.0, 0.0), full, V, nthreads=nthreads)
    return out[:, half_mask(hkl)]
