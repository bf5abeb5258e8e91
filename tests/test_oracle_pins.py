"""Pins of the CPU oracle against things other than itself (CPU only).

Each test names what fixes the expected value: the literal DFT definition,
numpy's FFT (a library routine the oracle does not call), closed forms of the
operator for special potentials, the paper's band-limit argument, integer
recounts of the sphere, and algebraic identities."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import (brute_apply_dense, dense_dft_matrix, direct_sphere_g2r, direct_sphere_r2g,
                     gather, isqrt_count, relerr, relerr_per_band, scatter)

SKEW = np.array([[6.0, 0.3, -0.2], [0.5, 7.0, 0.4], [-0.3, 0.6, 6.5]])


# ------------------------------------------------------------ 1-D transforms

@pytest.mark.parametrize("L", list(range(1, 33)) + [36, 45, 48, 49, 60, 64, 72, 80, 96, 125, 128])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_matches_definition(L, sign):
    rng = np.random.default_rng(L * 7 + (sign > 0))
    x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    n = np.arange(L)
    M = np.exp(sign * 2j * np.pi * np.outer(n, n) / L)  # literal definition
    ref = M @ x
    got = oracle.fft1d(x, sign)
    assert relerr(got, ref) < 1e-13
    # numpy's FFT: sign -1 is fft, sign +1 is L*ifft
    lib = np.fft.fft(x) if sign < 0 else np.fft.ifft(x) * L
    assert relerr(got, lib) < 1e-13


# ------------------------------------------------------------------- sphere

@pytest.mark.parametrize("R2,grid", [(36, 24), (576, 96), (1024, 128), (413, 80), (9, 12)])
def test_sphere_counts_closed_form(R2, grid):
    """npw = sum over (h,k) of 2 isqrt(R^2-h^2-k^2)+1 (integer recount)."""
    npw, nst, crange = isqrt_count(R2)
    cell = synth.cubic_cell()
    ecut = 0.5 * R2
    hkl = oracle.sphere_c(cell, ecut)
    assert hkl.shape[0] == npw
    st = oracle.sticks(hkl)
    assert st.shape[0] == nst
    assert (st[:, 3].min(), st[:, 3].max()) == crange
    assert int(st[:, 0].max() - st[:, 0].min() + 1) == 2 * math.isqrt(R2) + 1
    assert np.array_equal(oracle.sphere_py(cell, ecut), hkl)


def test_sphere_counts_known_values():
    # integer recounts of the two main workloads (checked against the closed form above)
    assert isqrt_count(36) == (925, 113, (1, 13))
    assert isqrt_count(576) == (57777, 1793, (1, 49))
    assert isqrt_count(1024)[:2] == (137065, 3209)


def test_sphere_boundary_inclusive():
    """|k+G| = G_cut exactly is kept (non-strict reading of eq. 3)."""
    hkl = oracle.sphere_c(synth.cubic_cell(), 0.5 * 36)
    assert any((h, k, l) == (6, 0, 0) for h, k, l in hkl)
    assert not any((h, k, l) == (6, 1, 0) for h, k, l in hkl)


@pytest.mark.parametrize("seed", range(6))
def test_sphere_c_vs_python_random_cells(seed):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        cell = np.eye(3) * rng.uniform(5, 9) + rng.uniform(-0.8, 0.8, (3, 3))
        k = rng.uniform(-0.5, 0.5, 3)
        ecut = rng.uniform(2, 12)
        a = oracle.sphere_c(cell, ecut, k)
        b = oracle.sphere_py(cell, ecut, k)
        # reject samples with a lattice point within 1e-10 of the boundary
        B = oracle.reciprocal(cell)
        if a.shape[0] != b.shape[0]:
            pts = np.unique(np.concatenate([a, b]), axis=0)
            g = (pts + k) @ B
            margin = np.abs(np.einsum("ij,ij->i", g, g) / (2 * ecut) - 1).min()
            assert margin < 1e-10
            continue
        assert np.array_equal(a, b)
        # brute force over a generous box
        box = np.arange(-12, 13)
        H, K, L = np.meshgrid(box, box, box, indexing="ij")
        P = np.stack([H.ravel(), K.ravel(), L.ravel()], 1)
        g = (P + k) @ B
        inside = P[np.einsum("ij,ij->i", g, g) <= 2 * ecut * (1 + 1e-12)]
        assert inside.shape[0] == a.shape[0]


def test_sticks_are_contiguous_runs():
    hkl = oracle.sphere_py(SKEW, 6.0, (0.25, 1 / 3, 0.0))
    st = oracle.sticks(hkl)
    assert st[:, 3].sum() == hkl.shape[0]
    assert np.array_equal(np.cumsum(np.r_[0, st[:-1, 3]]), st[:, 2])


# -------------------------------------------------------------- greedy deal

def test_greedy_deal_hand_example():
    # Sec. 3.2: sort descending, deal round robin.  counts by column index:
    counts = [3, 9, 1, 7, 7, 2]
    g, order = oracle.greedy_deal(counts, 2)
    # ranks: col1(9) col3(7) col4(7) col0(3) col5(2) col2(1) -> groups 0 1 0 1 0 1
    assert list(order) == [1, 3, 4, 0, 5, 2]
    assert list(g) == [1, 0, 1, 1, 0, 0]
    assert list(oracle.group_loads(counts, g, 2)) == [18, 11]
    gs, _ = oracle.greedy_deal(counts, 2, "snake")
    # snake by rank: 0 1 | 1 0 | 0 1 -> col1:0 col3:1 col4:1 col0:0 col5:0 col2:1
    assert list(gs) == [0, 0, 1, 1, 1, 0]


@pytest.mark.parametrize("ngroups", [1, 7, 64, 113, 256])
def test_greedy_deal_invariants(ngroups):
    st = oracle.sticks(oracle.sphere_py(synth.cubic_cell(), 288.0))
    counts = st[:, 3]
    for mode in ("cyclic", "snake", "unsorted"):
        g, order = oracle.greedy_deal(counts, ngroups, mode)
        assert sorted(order.tolist()) == list(range(counts.size))
        loads = oracle.group_loads(counts, g, ngroups)
        assert loads.sum() == counts.sum()
        sizes = np.bincount(g, minlength=ngroups)
        assert sizes.max() - sizes.min() <= 1
        if mode != "unsorted":
            # a sorted round-robin deal keeps any two groups within the largest column
            assert loads.max() - loads.min() <= counts.max()
            assert np.all(np.diff(counts[order]) <= 0)


# Balance of the 96^3 / R = 24 sphere's 1,793 sticks dealt to 64 and 256 groups,
# (max, min) plane waves per group: integers counted independently (by brute
# force over the sphere, then the deal rules of Sec. 3.2 read as stable sort by
# descending count, cyclic / snake / canonical-order deal).
BALANCE_PINS = {
    (64, "cyclic"): (929, 880), (64, "snake"): (910, 894), (64, "unsorted"): (965, 852),
    (256, "cyclic"): (250, 201), (256, "snake"): (231, 217), (256, "unsorted"): (257, 191),
}


@pytest.mark.parametrize("ngroups,mode", sorted(BALANCE_PINS))
def test_greedy_deal_balance_pins_96(ngroups, mode):
    st = oracle.sticks(oracle.sphere_py(synth.cubic_cell(), 288.0))
    g, _ = oracle.greedy_deal(st[:, 3], ngroups, mode)
    loads = oracle.group_loads(st[:, 3], g, ngroups)
    assert (int(loads.max()), int(loads.min())) == BALANCE_PINS[(ngroups, mode)]
    assert loads.sum() == 57777


@pytest.mark.parametrize("cell", [SKEW, SKEW * np.array([[1.0], [0.6], [0.7]]),
                                  np.array([[4.38, 1.0686, -2.8831], [2.3836, 8.7056, -0.1596],
                                            [-2.339, 2.8047, 3.0992]])])
def test_reciprocal_basis_duality(cell):
    """a_i . b_j = 2 pi delta_ij (eq. 3's G = h b1 + k b2 + l b3), checked as dot
    products of the rows, not by inverting again."""
    B = oracle.reciprocal(cell)
    for i in range(3):
        for j in range(3):
            d = float(np.dot(cell[i], B[j]))
            assert abs(d - (2 * math.pi if i == j else 0.0)) < 1e-13, (i, j, d)
    # the volume relation det(B) = (2 pi)^3 / det(A)
    assert abs(np.linalg.det(B) * np.linalg.det(cell) - (2 * math.pi) ** 3) < 1e-9


# --------------------------------------------------------- dense brute force

TINY = [((4, 4, 4), 1.0), ((6, 6, 6), 1.0), ((8, 8, 8), 2.0), ((10, 10, 10), 2.0),
        ((12, 12, 12), 3.0), ((6, 8, 10), 1.0), ((5, 6, 12), 1.0)]


@pytest.mark.parametrize("grid,R", TINY)
@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.25, 1 / 3, 0.0)])
@pytest.mark.parametrize("skew", [False, True])
def test_apply_vs_dense_dft(grid, R, kpt, skew):
    """T1: oracle vs the literal (N^3)^2 DFT matrix."""
    if skew:
        cell = SKEW  # |b_i| close to 1, so R*0.9 keeps a similar sphere
        ecut = 0.5 * (R * 0.9) ** 2
    else:
        cell = synth.cubic_cell()
        ecut = 0.5 * R * R
    hkl = oracle.sphere_c(cell, ecut, kpt)
    if hkl.shape[0] == 0:
        pytest.skip("empty sphere")
    ext = hkl.max(0) - hkl.min(0)
    if np.any(ext >= np.asarray(grid)):
        pytest.skip("sphere aliases on this grid")
    rng = np.random.default_rng(hash((grid, R, kpt, skew)) % 2 ** 32)
    c = rng.standard_normal((3, hkl.shape[0])) + 1j * rng.standard_normal((3, hkl.shape[0]))
    V = rng.uniform(0.2, 2.0, grid[0] * grid[1] * grid[2])
    ref = brute_apply_dense(grid, hkl, c, V)
    got = oracle.apply(grid, cell, ecut, kpt, c, V)
    assert relerr_per_band(got, ref).max() < 1e-13
    # G->r alone
    D = dense_dft_matrix(grid, -1)
    psi_ref = scatter(grid, hkl, c).reshape(3, -1) @ D.T
    psi = oracle.g2r(grid, cell, ecut, kpt, c).reshape(3, -1)
    assert relerr(psi, psi_ref) < 1e-13


def test_g2r_vs_numpy_fftn():
    """G->r with sign -1 is numpy's unnormalised fftn of the scattered cube."""
    grid = (12, 10, 16)
    cell = synth.cubic_cell()
    hkl = oracle.sphere_c(cell, 0.5 * 9)
    rng = np.random.default_rng(5)
    c = rng.standard_normal((2, hkl.shape[0])) + 1j * rng.standard_normal((2, hkl.shape[0]))
    psi = oracle.g2r(grid, cell, 4.5, (0, 0, 0), c)
    ref = np.fft.fftn(scatter(grid, hkl, c), axes=(1, 2, 3))
    assert relerr(psi, ref) < 1e-13
    back = oracle.r2g(grid, cell, 4.5, (0, 0, 0), psi)
    ref_back = gather(grid, hkl, np.fft.ifftn(psi, axes=(1, 2, 3)))
    assert relerr(back, ref_back) < 1e-13
    assert relerr(back, c) < 1e-13


def test_c1_vs_sphere_direct_dft():
    """T2: the 24^3 / R=6 / 8-band workload against direct sphere-restricted sums."""
    w = synth.WORKLOADS["c1_24"]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    hkl = oracle.sphere_c(cell, ecut)
    assert hkl.shape[0] == 925
    c = synth.coefficients(hkl, w["nbands"])
    V = synth.potential(grid, w["ngauss"])
    psi_ref = direct_sphere_g2r(grid, hkl, c)
    out_ref = direct_sphere_r2g(grid, hkl, psi_ref * V.reshape(1, -1))
    out = oracle.apply(grid, cell, ecut, (0, 0, 0), c, V)
    assert relerr_per_band(out, out_ref).max() < 1e-13


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("Q", [(1, 0, 0), (0, 2, -1), (3, -2, 5), (-4, 1, 2)])
def test_cos_sin_potential_closed_form(Q):
    """T3: V = v0 + 2a cos(theta) + 2b sin(theta), theta = 2 pi Q.j/N gives
    out(g) = v0 c(g) + (a - ib) c(g+Q) + (a + ib) c(g-Q) (c = 0 off the sphere).
    b != 0 distinguishes the two sign conventions; the 1/N and index wrap enter too."""
    grid = (16, 18, 20)
    R = 4
    cell = synth.cubic_cell()
    ecut = 0.5 * R * R
    hkl = oracle.sphere_c(cell, ecut)
    assert all(abs(Q[i]) <= grid[i] - 2 * R - 1 for i in range(3))
    rng = np.random.default_rng(11)
    c = rng.standard_normal((2, hkl.shape[0])) + 1j * rng.standard_normal((2, hkl.shape[0]))
    v0, a, b = 0.7, 0.31, -0.45
    N1, N2, N3 = grid
    j3, j2, j1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    theta = 2 * np.pi * (Q[0] * j1 / N1 + Q[1] * j2 / N2 + Q[2] * j3 / N3)
    V = v0 + 2 * a * np.cos(theta) + 2 * b * np.sin(theta)
    index = {tuple(p): i for i, p in enumerate(hkl.tolist())}

    def cat(g):
        i = index.get(tuple(g))
        return c[:, i] if i is not None else np.zeros(c.shape[0], complex)

    ref = np.empty_like(c)
    for i, g in enumerate(hkl.tolist()):
        gp = [g[0] + Q[0], g[1] + Q[1], g[2] + Q[2]]
        gm = [g[0] - Q[0], g[1] - Q[1], g[2] - Q[2]]
        ref[:, i] = v0 * c[:, i] + (a - 1j * b) * cat(gp) + (a + 1j * b) * cat(gm)
    out = oracle.apply(grid, cell, ecut, (0, 0, 0), c, V)
    assert relerr(out, ref) < 1e-13
    # the opposite convention swaps +Q and -Q, so it must not match when b != 0
    out_flip = oracle.apply(grid, cell, ecut, (0, 0, 0), c, V, sign=+1)
    assert relerr(out_flip, ref) > 1e-2


def _bandlimited_V(grid, R, seed):
    """Real V from a random Hermitian spectrum on |Q_i| <= 2R-1, by direct sum."""
    rng = np.random.default_rng(seed)
    q = np.arange(-(2 * R - 1), 2 * R)
    Qs = np.stack(np.meshgrid(q, q, q, indexing="ij"), -1).reshape(-1, 3)
    Vh = {}
    for Qv in Qs.tolist():
        t = tuple(Qv)
        if t in Vh:
            continue
        m = tuple(-x for x in t)
        if t == m:
            Vh[t] = complex(rng.standard_normal())
        else:
            z = complex(rng.standard_normal(), rng.standard_normal()) * 0.3
            Vh[t] = z
            Vh[m] = np.conj(z)
    N1, N2, N3 = grid
    j3, j2, j1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    V = np.zeros((N3, N2, N1), complex)
    for (a, b, cc), val in Vh.items():
        V += val * np.exp(-2j * np.pi * (a * j1 / N1 + b * j2 / N2 + cc * j3 / N3))
    assert np.abs(V.imag).max() < 1e-10
    return V.real.copy(), Vh


def test_bandlimited_convolution_on_4R_grid():
    """T4 (Sec. 3.1, Fig. 1): with V band-limited to 2 G_cut a grid of 4R per axis
    gives out(g) = sum_{g' in S} Vhat(g-g') c(g') exactly: no wrap-around inside G_cut."""
    R = 3
    grid = (4 * R, 4 * R, 4 * R)
    cell = synth.cubic_cell()
    ecut = 0.5 * R * R
    hkl = oracle.sphere_c(cell, ecut)
    V, Vh = _bandlimited_V(grid, R, 21)
    rng = np.random.default_rng(22)
    c = rng.standard_normal((2, hkl.shape[0])) + 1j * rng.standard_normal((2, hkl.shape[0]))
    pts = hkl.tolist()
    M = np.zeros((len(pts), len(pts)), complex)
    for i, g in enumerate(pts):
        for j, gp in enumerate(pts):
            M[i, j] = Vh.get((g[0] - gp[0], g[1] - gp[1], g[2] - gp[2]), 0.0)
    ref = c @ M.T
    out = oracle.apply(grid, cell, ecut, (0, 0, 0), c, V)
    assert relerr(out, ref) < 1e-12
    # too small a grid (< 4R) folds the 2G_cut..3G_cut shell back: must differ
    small = (4 * R - 2,) * 3
    Vs, Vhs = _bandlimited_V(small, R, 21)
    assert Vhs == Vh
    outs = oracle.apply(small, cell, ecut, (0, 0, 0), c, Vs)
    assert relerr(outs, ref) > 1e-3


# ----------------------------------------------------------- identities

def _setup(grid=(12, 12, 15), R=3.0, nb=4, seed=3, kpt=(0, 0, 0)):
    cell = synth.cubic_cell()
    ecut = 0.5 * R * R
    hkl = oracle.sphere_c(cell, ecut, kpt)
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((nb, hkl.shape[0])) + 1j * rng.standard_normal((nb, hkl.shape[0]))
    V = rng.uniform(0.3, 2.5, grid[0] * grid[1] * grid[2])
    return grid, cell, ecut, hkl, c, V


def test_parseval_roundtrip_constant_V():
    grid, cell, ecut, hkl, c, V = _setup()
    N = np.prod(grid)
    psi = oracle.g2r(grid, cell, ecut, (0, 0, 0), c)
    assert abs(np.sum(np.abs(psi) ** 2) / (N * np.sum(np.abs(c) ** 2)) - 1) < 1e-13
    assert relerr(oracle.r2g(grid, cell, ecut, (0, 0, 0), psi), c) < 1e-14
    assert relerr(oracle.apply(grid, cell, ecut, (0, 0, 0), c, np.ones(N)), c) < 1e-14
    assert relerr(oracle.apply(grid, cell, ecut, (0, 0, 0), c, np.full(N, 2.75)), 2.75 * c) < 1e-14


def test_single_plane_wave():
    grid, cell, ecut, hkl, c, V = _setup()
    i0 = 17
    c = np.zeros((1, hkl.shape[0]), complex)
    c[0, i0] = 1.0
    psi = oracle.g2r(grid, cell, ecut, (0, 0, 0), c)[0]
    assert np.abs(np.abs(psi) - 1).max() < 1e-13
    h, k, l = hkl[i0]
    N1, N2, N3 = grid
    assert abs(psi[1, 0, 0] - np.exp(-2j * np.pi * l / N3)) < 1e-13
    assert abs(psi[0, 0, 1] - np.exp(-2j * np.pi * h / N1)) < 1e-13
    back = oracle.r2g(grid, cell, ecut, (0, 0, 0), psi[None])
    assert relerr(back, c) < 1e-14


def test_hermiticity_energy_bounds():
    """T6: H = C^H (V C) is Hermitian; Re H_nn = (1/N) sum_j V |psi_n|^2;
    min V <= H_nn/|c_n|^2 <= max V."""
    grid, cell, ecut, hkl, c, V = _setup(nb=6, kpt=(0.25, 1 / 3, 0))
    N = np.prod(grid)
    out = oracle.apply(grid, cell, ecut, (0.25, 1 / 3, 0), c, V)
    H = np.conj(c) @ out.T
    assert np.linalg.norm(H - H.conj().T) / np.linalg.norm(H) < 1e-13
    psi = oracle.g2r(grid, cell, ecut, (0.25, 1 / 3, 0), c).reshape(c.shape[0], -1)
    e = (V[None, :] * np.abs(psi) ** 2).sum(1) / N
    assert relerr(np.real(np.diag(H)), e) < 1e-13
    ray = np.real(np.diag(H)) / np.sum(np.abs(c) ** 2, 1)
    assert np.all(ray >= V.min() - 1e-12) and np.all(ray <= V.max() + 1e-12)


def test_linearity():
    grid, cell, ecut, hkl, c, V = _setup(nb=2)
    rng = np.random.default_rng(9)
    c2 = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
    V2 = rng.uniform(-1, 1, V.size)
    f = lambda cc, vv: oracle.apply(grid, cell, ecut, (0, 0, 0), cc, vv)
    a, b = 0.3 - 1.1j, 2.2
    assert relerr(f(a * c + b * c2, V), a * f(c, V) + b * f(c2, V)) < 1e-13
    assert relerr(f(c, 0.5 * V + 3 * V2), 0.5 * f(c, V) + 3 * f(c, V2)) < 1e-13


def test_sign_reflection_identity():
    """T8: the opposite convention equals the paper's with g -> -g and k -> -k."""
    kpt = (0.25, 1 / 3, 0.0)
    grid, cell, ecut, hkl, c, V = _setup(kpt=kpt)
    out_flip = oracle.apply(grid, cell, ecut, kpt, c, V, sign=+1)
    mk = tuple(-x for x in kpt)
    hkl_m = oracle.sphere_c(cell, ecut, mk)
    idx = {tuple(p): i for i, p in enumerate(hkl_m.tolist())}
    perm = np.array([idx[(-h, -k, -l)] for h, k, l in hkl.tolist()])
    c_ref = np.empty_like(c)
    c_ref[:, perm] = c
    out_ref = oracle.apply(grid, cell, ecut, mk, c_ref, V)
    assert relerr(out_flip, out_ref[:, perm]) < 1e-13


# ------------------------------------------------- real (gamma) mode oracle

def test_gamma_half_sphere_counts():
    for ecut, npw in ((18.0, 925), (288.0, 57777)):
        hkl = oracle.sphere_py(synth.cubic_cell(), ecut)
        assert hkl.shape[0] == npw
        m = oracle.half_mask(hkl)
        assert m.sum() == (npw + 1) // 2
        # H and -H partition the sphere minus the origin
        neg = {tuple((-g).tolist()) for g in hkl[m]}
        assert len(neg & {tuple(g.tolist()) for g in hkl[m]}) == 1  # only g = 0


def test_gamma_expansion_gives_real_psi():
    grid, cell, ecut = (24, 24, 24), synth.cubic_cell(), 18.0
    hkl = oracle.sphere_py(cell, ecut)
    ch = synth.coefficients(hkl[oracle.half_mask(hkl)], 3)
    psi = oracle.g2r(grid, cell, ecut, (0, 0, 0), oracle.expand_half(hkl, ch))
    assert np.abs(psi.imag).max() <= 1e-13 * np.abs(psi.real).max()
    assert np.abs(psi.real).max() > 1e-3


def test_gamma_apply_brute_force_tiny():
    """Closed form of the real mode on a 6^3 grid: psi(j) = Re c(0) +
    2 Re sum_{g in H, g != 0} c(g) e^{-2 pi i g.j/N}, out(g) = (1/N) sum_j
    e^{+2 pi i g.j/N} V(j) psi(j) for g in H."""
    grid, cell, ecut = (6, 6, 6), synth.cubic_cell(), 2.0
    hkl = oracle.sphere_py(cell, ecut)
    m = oracle.half_mask(hkl)
    H = hkl[m]
    rng = np.random.default_rng(11)
    ch = rng.standard_normal((2, H.shape[0])) + 1j * rng.standard_normal((2, H.shape[0]))
    V = rng.uniform(0.5, 1.5, 216)
    N = 216
    j3, j2, j1 = np.meshgrid(np.arange(6), np.arange(6), np.arange(6), indexing="ij")
    J = np.stack([j1.ravel(), j2.ravel(), j3.ravel()], axis=1)  # x fastest
    ph = np.exp(-2j * np.pi * (H @ J.T) / 6.0)                  # [g in H][j]
    zero = (H == 0).all(axis=1)
    ref = []
    for b in range(2):
        c = ch[b].copy()
        psi = np.real(c[zero]).sum() + 2 * np.real(c[~zero] @ ph[~zero])
        ref.append((np.conj(ph) @ (V * psi)) / N)
    got = oracle.apply_gamma(grid, cell, ecut, ch, V)
    assert np.abs(got - np.array(ref)).max() <= 1e-13 * np.abs(ref).max()


def test_gamma_output_symmetry_and_real_origin():
    grid, cell, ecut = (24, 24, 24), synth.cubic_cell(), 18.0
    hkl = oracle.sphere_py(cell, ecut)
    m = oracle.half_mask(hkl)
    ch = synth.coefficients(hkl[m], 2)
    V = synth.potential(grid, 4)
    full = oracle.apply(grid, cell, ecut, (0, 0, 0), oracle.expand_half(hkl, ch), V)
    index = {tuple(g): i for i, g in enumerate(hkl.tolist())}
    mirror = np.array([index[tuple((-g).tolist())] for g in hkl])
    assert np.abs(full[:, mirror] - np.conj(full)).max() <= 1e-14 * np.abs(full).max()
    # Im c(0) is ignored
    ch2 = ch.copy()
    z = np.nonzero((hkl[m] == 0).all(axis=1))[0]
    ch2[:, z] += 0.7j
    a = oracle.apply_gamma(grid, cell, ecut, ch, V)
    b = oracle.apply_gamma(grid, cell, ecut, ch2, V)
    assert np.array_equal(a, b)
    assert np.abs(a[:, z].imag).max() <= 1e-15 * np.abs(a).max()
