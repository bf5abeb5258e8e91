"""Host-side checks of libvloc (CPU only, no kernel launches).

* every function declared in include/vloc.h is exported;
* the plan's sphere, canonical G order, stick table and greedy deal equal the
  oracle's independent Python enumeration, bit for bit;
* argument validation returns the documented status before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from conftest import ROOT, gpu_available

vloc = pytest.importorskip("paper_1601_07378_amd.vloc")

SKEW = np.array([[6.0, 0.3, -0.2], [0.5, 7.0, 0.4], [-0.3, 0.6, 6.5]])
# Strongly skewed cells with a k-shift (cell, Ecut, k): on some x-planes the
# sphere's sticks skip a k value (the section at fixed (h, k) holds no integer l)
HOLE_A = (np.array([[4.38, 1.0686, -2.8831], [2.3836, 8.7056, -0.1596], [-2.339, 2.8047, 3.0992]]),
          39.588, (-0.3216, -0.2485, -0.2091))
HOLE_B = (np.array([[3.7123, -1.7955, 2.7501], [-0.9051, 5.5968, 2.7584],
                    [2.9182, 1.8833, 5.3089]]), 37.086, (-0.229, 0.1557, -0.141))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "vloc.h")).read()
    names = set(re.findall(r"\b(vloc_[a-z0-9_]+)\s*\(", hdr))
    assert names, "no declarations found"
    assert names == set(vloc.EXPORTS)
    L = vloc.lib()
    for n in names:
        assert hasattr(L, n), n


CASES = [
    ((24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0)),
    ((96, 96, 96), synth.cubic_cell(), 288.0, (0, 0, 0)),
    ((128, 128, 128), synth.cubic_cell(), 512.0, (0, 0, 0)),
    ((80, 80, 80), synth.cubic_cell(), 206.5, (0, 0, 0)),
    ((72, 96, 128), synth.cubic_cell(), 162.0, (0.25, 0, 0)),
    ((72, 96, 128), synth.cubic_cell(), 162.0, (0.25, 0.25, 0)),
    ((72, 96, 128), synth.cubic_cell(), 162.0, (0.25, 0.25, 0.25)),
    ((16, 18, 20), SKEW, 12.0, (0.25, 1 / 3, 0.0)),
    ((15, 9, 10), SKEW * np.array([[1.0], [0.6], [0.7]]), 5.0, (0.1, -0.2, 0.3)),
    # skewed cells with a k-shift whose x-planes have holes in their k span
    ((16, 30, 15), HOLE_A[0], HOLE_A[1], HOLE_A[2]),
    ((15, 18, 18), HOLE_B[0], HOLE_B[1], HOLE_B[2]),
    # lengths that need codelets above 16 points, and a z axis above 256
    ((125, 24, 24), np.diag([5.0, 1.0, 1.0]) * 2 * np.pi, 18.0, (0, 0, 0)),
    ((250, 27, 25), np.diag([10.0, 1.0, 1.0]) * 2 * np.pi, 18.0, (0.1, 0, 0)),
    ((24, 24, 288), np.diag([1.0, 1.0, 12.0]) * 2 * np.pi, 18.0, (0, 0, 0)),
]


@pytest.mark.parametrize("grid,cell,ecut,k", CASES)
def test_stick_map_matches_oracle(grid, cell, ecut, k):
    """T9: G list, stick table, occupied range, deal and balance, bit-exact."""
    p = vloc.Plan(grid, cell, ecut, k)
    ref = oracle.sphere_py(cell, ecut, k)
    assert np.array_equal(p.gvectors(), ref)
    st_ref = oracle.sticks(ref)
    assert np.array_equal(p.sticks().astype(np.int64), st_ref)
    lay = p.layout()
    assert lay["nxo"] == st_ref[:, 0].max() - st_ref[:, 0].min() + 1
    ng = p.balance().size
    g_ref, _ = oracle.greedy_deal(st_ref[:, 3], ng, "cyclic")
    assert np.array_equal(p.stick_groups(), g_ref)
    assert np.array_equal(p.balance(), oracle.group_loads(st_ref[:, 3], g_ref, ng))
    ps = vloc.Plan(grid, cell, ecut, k, deal="snake")
    gs_ref, _ = oracle.greedy_deal(st_ref[:, 3], ng, "snake")
    assert np.array_equal(ps.stick_groups(), gs_ref)
    pu = vloc.Plan(grid, cell, ecut, k, deal="unsorted")
    gu_ref, _ = oracle.greedy_deal(st_ref[:, 3], ng, "unsorted")
    assert np.array_equal(pu.stick_groups(), gu_ref)


@pytest.mark.parametrize("cell,ecut,k,grid,nholes", [(*HOLE_A, (16, 30, 15), 1),
                                                     (*HOLE_B, (15, 18, 18), 7)])
def test_planes_with_k_holes_are_accepted(cell, ecut, k, grid, nholes):
    """An x-plane's sticks need not be contiguous in k on a skewed cell; the
    plan accepts such spheres (the oracle's enumeration shows the holes)."""
    st = oracle.sticks(oracle.sphere_py(cell, ecut, k))
    holes = 0
    for h in np.unique(st[:, 0]):
        ks = st[st[:, 0] == h, 1]
        holes += (ks.max() - ks.min() + 1) - ks.size
    assert holes == nholes
    p = vloc.Plan(grid, cell, ecut, k)
    assert np.array_equal(p.sticks().astype(np.int64), st)


def test_known_counts():
    p = vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0)
    assert (p.npw, p.sticks().shape[0]) == (925, 113)
    p = vloc.Plan((96, 96, 96), synth.cubic_cell(), 288.0)
    assert (p.npw, p.sticks().shape[0], p.layout()["nxo"]) == (57777, 1793, 49)


def test_greedy_balance_beats_unsorted():
    """Tab. 2's statistic per workgroup: the sorted deal narrows max-min."""
    p = vloc.Plan((96, 96, 96), synth.cubic_cell(), 288.0, sticks_per_group=28)
    loads = p.balance()
    st = p.sticks()
    g_u, _ = oracle.greedy_deal(st[:, 3], loads.size, "unsorted")
    lu = oracle.group_loads(st[:, 3], g_u, loads.size)
    assert loads.max() - loads.min() < lu.max() - lu.min()
    assert loads.max() - loads.min() <= st[:, 3].max()


def _create(grid, cell=None, ecut=18.0, k=(0, 0, 0), opt=None):
    L = vloc.lib()
    h = ctypes.c_void_p()
    g = np.asarray(grid, dtype=np.int32)
    c = np.ascontiguousarray(np.asarray(synth.cubic_cell() if cell is None else cell,
                                        dtype=np.float64).reshape(9))
    kk = np.asarray(k, dtype=np.float64)
    o = ctypes.byref(opt) if opt is not None else None
    s = L.vloc_plan_create_ex(ctypes.byref(h), vloc._i32(g), vloc._f64(c), ecut, vloc._f64(kk), o)
    return s, h


def _smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.parametrize("grid,status", [((7, 24, 24), vloc.VLOC_E_GRID),
                                         ((14, 24, 24), vloc.VLOC_E_GRID),
                                         ((24, 21, 24), vloc.VLOC_E_GRID),
                                         ((24, 24, 22), vloc.VLOC_E_GRID),
                                         ((961, 24, 24), vloc.VLOC_E_GRID),
                                         ((972, 24, 24), vloc.VLOC_E_GRID),
                                         ((0, 24, 24), vloc.VLOC_E_GRID),
                                         ((125, 24, 24), vloc.VLOC_OK),
                                         ((243, 24, 24), vloc.VLOC_OK),
                                         ((250, 24, 24), vloc.VLOC_OK),
                                         ((24, 24, 960), vloc.VLOC_OK),
                                         ((24, 24, 24), vloc.VLOC_OK)])
def test_grid_validation(grid, status):
    s, h = _create(grid)
    assert s == status
    assert (h.value is None) == (status != vloc.VLOC_OK)
    vloc.lib().vloc_plan_destroy(h)


def test_every_smooth_length_accepted():
    """Every 2,3,5-smooth length up to 960 is accepted on each axis, every other
    length is refused with VLOC_E_GRID (the sphere is kept small)."""
    for n in range(1, 961):
        for axis in range(3):
            grid = [24, 24, 24]
            grid[axis] = n
            s, h = _create(tuple(grid), ecut=0.3)
            vloc.lib().vloc_plan_destroy(h)
            assert s == (vloc.VLOC_OK if _smooth(n) else vloc.VLOC_E_GRID), (grid, s)


def test_big_codelets_need_512_threads():
    s, h = _create((125, 24, 24), opt=vloc.make_options(plane_threads=1024))
    assert s == vloc.VLOC_E_INVALID
    p = vloc.Plan((125, 24, 24), synth.cubic_cell(), 18.0)
    assert p.layout()["plane_threads"] <= 512
    assert max(p.layout()["L1x"], p.layout()["L2x"]) == 25


def test_sphere_and_cell_validation():
    assert _create((24, 24, 24), ecut=0.5 * 12 ** 2)[0] == vloc.VLOC_E_SPHERE  # extent 25 > 24
    assert _create((24, 24, 24), ecut=0.0)[0] == vloc.VLOC_E_SPHERE
    assert _create((24, 24, 24), ecut=float("nan"))[0] == vloc.VLOC_E_SPHERE
    assert _create((24, 24, 24), cell=-np.eye(3))[0] == vloc.VLOC_E_CELL
    assert _create((24, 24, 24), cell=np.zeros((3, 3)))[0] == vloc.VLOC_E_CELL
    bad = np.eye(3)
    bad[0, 0] = float("inf")
    assert _create((24, 24, 24), cell=bad)[0] == vloc.VLOC_E_CELL
    assert _create((24, 24, 24), k=(float("nan"), 0, 0))[0] == vloc.VLOC_E_SPHERE
    o = vloc.Options(7, 0, 0, 0, 0, 0)
    assert _create((24, 24, 24), opt=o)[0] == vloc.VLOC_E_INVALID
    o = vloc.Options(0, 0, 0, 0, 0, 100)
    assert _create((24, 24, 24), opt=o)[0] == vloc.VLOC_E_INVALID
    L = vloc.lib()
    assert L.vloc_plan_create(None, None, None, 1.0, None) == vloc.VLOC_E_INVALID
    assert L.vloc_plan_destroy(None) == vloc.VLOC_OK
    assert b"NULL" in L.vloc_last_error() or L.vloc_last_error()


def test_apply_argument_validation_before_device():
    """Checks that return before any HIP call; the pointers are never dereferenced."""
    L = vloc.lib()
    p = vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0)
    h = p._h
    fake_c, fake_v = ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x40000000)
    assert L.vloc_apply(h, fake_c, 0, fake_v, fake_c) == vloc.VLOC_OK  # no-op
    assert L.vloc_apply(h, fake_c, -1, fake_v, ctypes.c_void_p(0x20000000)) == vloc.VLOC_E_INVALID
    assert L.vloc_apply(h, None, 3, fake_v, ctypes.c_void_p(0x20000000)) == vloc.VLOC_E_INVALID
    assert L.vloc_apply(h, fake_c, 3, fake_v, fake_c) == vloc.VLOC_E_ALIAS
    # out starts inside c's 3 bands
    assert L.vloc_apply(h, fake_c, 3, fake_v, ctypes.c_void_p(0x10000000 + 16 * 925)) == \
        vloc.VLOC_E_ALIAS
    assert L.vloc_apply(h, fake_c, 3, fake_v, ctypes.c_void_p(0x40000000 - 16)) == \
        vloc.VLOC_E_ALIAS
    assert L.vloc_apply(h, ctypes.c_void_p(0x10000008), 3, fake_v,
                        ctypes.c_void_p(0x20000000)) == vloc.VLOC_E_INVALID  # misaligned
    assert L.vloc_apply(None, fake_c, 1, fake_v, fake_c) == vloc.VLOC_E_INVALID
    assert L.vloc_g2r(h, fake_c, 2, fake_c) == vloc.VLOC_E_ALIAS
    assert L.vloc_r2g(h, fake_c, 0, fake_c) == vloc.VLOC_OK
    assert L.vloc_status_string(vloc.VLOC_E_ALIAS) == b"output overlaps an input"


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_apply_without_device_reports_device_error():
    L = vloc.lib()
    p = vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0)
    s = L.vloc_apply(p._h, ctypes.c_void_p(0x10000000), 1, ctypes.c_void_p(0x40000000),
                     ctypes.c_void_p(0x20000000))
    assert s == vloc.VLOC_E_DEVICE
    assert L.vloc_last_error()


def test_parted_plane_rules():
    # forced on a grid whose plane fits whole: parts of N2 / P rows with P
    # dividing L1y, chosen by plane_rows
    p = vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0, plane_xmode=6)
    lay = p.layout()
    assert lay["plane_xmode"] == 6 and (lay["L1y"], lay["L2y"]) == (6, 4)
    assert lay["plane_rows"] == 12 and lay["plane_threads"] == 768  # fewest parts: P = 2
    for rows in (12, 8, 4):
        lay = vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0, plane_xmode=6,
                        plane_rows=rows).layout()
        assert lay["plane_rows"] == rows and lay["plane_xmode"] == 6
    with pytest.raises(vloc.VlocError):  # 24 / 5 rows: 5 does not divide L1y
        vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0, plane_xmode=6, plane_rows=5)
    # an explicit split is kept
    lay = vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0, plane_xmode=6,
                    split=(4, 4, 0)).layout()
    assert (lay["L1x"], lay["L2x"], lay["L1y"], lay["L2y"]) == (4, 6, 4, 6)
    # nxo L1y / P lines of y stage B must fit the workgroup in one round
    with pytest.raises(vloc.VlocError):
        vloc.Plan((24, 24, 24), synth.cubic_cell(), 18.0, plane_xmode=6, plane_threads=64,
                  split=(0, 12, 0), plane_rows=12)


def test_layout_defaults():
    p = vloc.Plan((96, 96, 96), synth.cubic_cell(), 288.0)
    lay = p.layout()
    assert (lay["L1x"], lay["L2x"]) == (8, 12)
    assert lay["plane_lds_bytes"] <= 160 * 1024
    assert lay["sticks_per_group"] * max(lay["L1z"], lay["L2z"]) <= 256
    # the whole plane fits (96 x 97 complex): x pass in place, 16 waves in FP64
    # plane, then twiddles of both axes and the 49 columns' k ranges
    assert lay["plane_xmode"] == 3
    assert lay["plane_lds_bytes"] == 96 * 97 * 16 + (96 + 96) * 16 + 49 * 8
    assert lay["plane_threads"] == 1024
    pf = vloc.Plan((96, 96, 96), synth.cubic_cell(), 288.0, precision="f32")
    assert pf.layout()["plane_lds_bytes"] == 96 * 97 * 8 + (96 + 96) * 8 + 49 * 8
    p1 = vloc.Plan((96, 96, 96), synth.cubic_cell(), 288.0, plane_xmode=1)
    assert p1.layout()["plane_xmode"] == 1 and p1.layout()["plane_lds_bytes"] <= 160 * 1024
    # 128^3 FP64: the whole plane (128 x 129 x 16 B) does not fit; the parted
    # plane: 65 columns (stride 129) or a row buffer of 128 x (64 + 1), two
    # parts, the longer y codelet first (y 16 x 8, x 8 x 16), 768 threads
    p128 = vloc.Plan((128, 128, 128), synth.cubic_cell(), 512.0)
    lay = p128.layout()
    assert lay["plane_xmode"] == 6 and lay["plane_rows"] == 64 and lay["plane_threads"] == 768
    assert (lay["L1x"], lay["L2x"], lay["L1y"], lay["L2y"]) == (8, 16, 16, 8)
    assert lay["plane_lds_bytes"] == max(65 * 129, 128 * 65) * 16 + (128 + 128) * 16 + 65 * 8
    for opts in (dict(plane_xmode=6), dict(plane_xmode=6, plane_threads=768, split=(8, 0, 0)),
                 dict(plane_xmode=6, plane_rows=32)):
        lay = vloc.Plan((128, 128, 128), synth.cubic_cell(), 512.0, **opts).layout()
        assert lay["plane_xmode"] == 6
    # FP32 at 144^3 (the whole plane 144 x 145 x 8 B does not fit): parted, 1024 threads
    lay = vloc.Plan((144, 144, 144), synth.cubic_cell(), 648.0, precision="f32").layout()
    assert lay["plane_xmode"] == 6 and lay["plane_threads"] == 1024
    rows = vloc.Plan((128, 128, 128), synth.cubic_cell(), 512.0, plane_xmode=1).layout()
    assert rows["plane_xmode"] == 1 and (rows["L1x"], rows["L2x"]) == (8, 16)
    with pytest.raises(vloc.VlocError):
        vloc.Plan((128, 128, 128), synth.cubic_cell(), 512.0, plane_xmode=3)
    l32 = vloc.Plan((128, 128, 128), synth.cubic_cell(), 512.0, precision="f32").layout()
    # the whole plane; y split 16 x 8 so that the 65 x 8 y stage-A tasks fit the
    # direct y form (65 x 16 would not)
    assert l32["plane_xmode"] == 3 and (l32["L1y"], l32["L2y"]) == (16, 8)
    l32s = vloc.Plan((128, 128, 128), synth.cubic_cell(), 512.0, precision="f32",
                     split=(0, 8, 0)).layout()
    assert (l32s["L1y"], l32s["L2y"]) == (8, 16)  # an explicit split is kept
    pq = vloc.Plan((96, 96, 96), synth.cubic_cell(), 288.0, plane_xmode=2)
    assert pq.layout()["plane_xmode"] == 2 and pq.layout()["plane_lds_bytes"] == 49 * 97 * 16
    with pytest.raises(vloc.VlocError):
        vloc.Plan((16, 18, 20), SKEW, 12.0, plane_xmode=2)


# ------------------------------------------------------------ real mode

@pytest.mark.parametrize("grid,ecut", [((24, 24, 24), 18.0), ((96, 96, 96), 288.0),
                                       ((15, 9, 10), 5.0)])
def test_gamma_plan_half_sphere_and_paired_deal(grid, ecut):
    cell = synth.cubic_cell() if grid[0] != 15 else SKEW * np.array([[1.0], [0.6], [0.7]])
    p = vloc.Plan(grid, cell, ecut, gamma=True)
    full = oracle.sphere_py(cell, ecut)
    half = full[oracle.half_mask(full)]
    assert np.array_equal(p.gvectors(), half) and p.npw == half.shape[0]
    st = p.sticks()
    assert np.array_equal(st.astype(np.int64), oracle.sticks(full))
    grp = p.stick_groups()
    index = {(h, k): i for i, (h, k) in enumerate(st[:, :2].tolist())}
    for i, (h, k) in enumerate(st[:, :2].tolist()):
        assert grp[i] == grp[index[(-h, -k)]]      # a stick and its mirror share a group
    # the deal of pairs: greedy order of the half-sphere sticks' counts
    loads = p.balance()
    assert loads.sum() == full.shape[0]
    assert loads.max() - loads.min() <= 2 * st[:, 3].max()


def test_gamma_validation():
    cell = synth.cubic_cell()
    with pytest.raises(vloc.VlocError) as e:
        vloc.Plan((24, 24, 24), cell, 18.0, (0.25, 0, 0), gamma=True)
    assert e.value.status == vloc.VLOC_E_INVALID
    with pytest.raises(vloc.VlocError):
        vloc.Batch((24, 24, 24), cell, 18.0, [(0, 0, 0)], gamma=True)
    L = vloc.lib()
    p = vloc.Plan((24, 24, 24), cell, 18.0, gamma=True)
    fake = ctypes.c_void_p(0x10000000)
    other = ctypes.c_void_p(0x20000000)
    assert L.vloc_g2r(p._h, fake, 1, other) == vloc.VLOC_E_INVALID
    assert L.vloc_r2g(p._h, fake, 1, other) == vloc.VLOC_E_INVALID
    assert L.vloc_band_dot(p._h, fake, other, 1, other) == vloc.VLOC_E_INVALID
    assert L.vloc_density(p._h, fake, 1, other, None, other) == vloc.VLOC_E_INVALID
    assert L.vloc_scale_bands(p._h, fake, 1, None, None, 1.0, other) == vloc.VLOC_E_INVALID
    # apply's alias check covers the two half-sphere bands (2 x 463 coefficients)
    assert L.vloc_apply(p._h, fake, 2, ctypes.c_void_p(0x40000000),
                        ctypes.c_void_p(0x10000000 + 16 * 925)) == vloc.VLOC_E_ALIAS


def test_stick_group_fits_lds():
    """A stick workgroup keeps its group's z lines (N3 + 1 each) and the N3 stage
    twiddles in the 160 KiB of LDS: at N3 = 256 that is at most 38 FP64 sticks or
    77 FP32 ones.  An explicit larger group is rejected; the automatic choice stays
    below the bound."""
    grid, cell, ecut = (16, 16, 256), synth.cubic_cell(), 0.5 * 4.0 ** 2
    p = vloc.Plan(grid, cell, ecut)
    assert p.sticks().shape[0] >= 39
    cap64 = (160 * 1024 // 16 - 256) // 257
    assert cap64 == 38
    assert p.layout()["sticks_per_group"] <= cap64
    vloc.Plan(grid, cell, ecut, sticks_per_group=38)
    with pytest.raises(vloc.VlocError) as e:
        vloc.Plan(grid, cell, ecut, sticks_per_group=39)
    assert e.value.status == vloc.VLOC_E_INVALID
    assert "LDS" in str(e.value)
    vloc.Plan(grid, cell, ecut, precision="f32", sticks_per_group=39)
