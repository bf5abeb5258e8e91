"""GPU parity: libvloc's HIP path against the CPU oracle, through the C ABI.

FP64 gate: norm-wise relative error per band <= 1e-12.  FP32 error is
measured against the oracle on the FP32-rounded inputs and reported; its gate
(<= 2e-6) follows from about log2(N) rounding steps of unit roundoff 6e-8.
Stick-map equality is checked bit for bit on the CPU (test_plan_abi)."""
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import relerr, relerr_per_band

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vloc = pytest.importorskip("paper_1601_07378_amd.vloc")

TOL64 = 1e-12
TOL32 = 2e-6
SKEW = np.array([[6.0, 0.3, -0.2], [0.5, 7.0, 0.4], [-0.3, 0.6, 6.5]])


@pytest.fixture(scope="module", autouse=True)
def _gpu(require_gpu):
    yield


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def run(plan, c, V):
    ct, rt = (torch.complex128, torch.float64) if plan.precision == "f64" else \
        (torch.complex64, torch.float32)
    out = plan.apply(dev(c, ct), dev(V, rt))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


def case(grid, cell, ecut, k, nb, ngauss=4, seed=0):
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, nb, k, ik=seed)
    V = synth.potential(grid, ngauss, seed=2000 + seed)
    return hkl, c, V


def label(**kw):
    print("CASE", kw, flush=True)


# ------------------------------------------------------------------ FP64

PARITY = [
    ("c1", (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0), 8),
    ("ragged_skew_k", (16, 18, 20), SKEW, 12.0, (0.25, 1 / 3, 0.0), 5),
    ("odd_radices", (15, 9, 10), SKEW * np.array([[1.0], [0.6], [0.7]]), 5.0, (0.1, -0.2, 0.3), 3),
    ("radix5_80", (40, 30, 50), synth.cubic_cell(), 0.5 * 9.5 ** 2, (0, 0, 0), 4),
    ("ortho_72_96_128_k", (72, 96, 128), synth.cubic_cell(), 162.0, (0.25, 0.25, 0.25), 3),
    ("sizes_16", (64, 48, 32), synth.cubic_cell(), 0.5 * 7.5 ** 2, (0.5, 0, 0), 5),
]


@pytest.mark.parametrize("name,grid,cell,ecut,k,nb", PARITY)
def test_apply_f64_vs_oracle(name, grid, cell, ecut, k, nb):
    label(test="apply_f64", name=name, grid=grid, nb=nb)
    hkl, c, V = case(grid, cell, ecut, k, nb)
    p = vloc.Plan(grid, cell, ecut, k)
    assert np.array_equal(p.gvectors(), hkl)
    got = run(p, c, V)
    ref = oracle.apply(grid, cell, ecut, k, c, V)
    err = relerr_per_band(got, ref)
    print(name, "max per-band rel err", err.max())
    assert err.max() <= TOL64


def test_c2_full_size_sampled_bands():
    """96^3, R = 24, 256 bands in the benchmark's launch configuration; bands
    sampled across chunks are checked against the oracle one by one."""
    w = synth.WORKLOADS["c2_96"]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    label(test="c2_full", grid=grid, nb=w["nbands"])
    hkl = oracle.sphere_py(cell, ecut)
    c = synth.coefficients(hkl, w["nbands"])
    V = synth.potential(grid, w["ngauss"])
    p = vloc.Plan(grid, cell, ecut)
    got = run(p, c, V)
    sample = [0, 1, 77, 131, 200, 255]
    ref = oracle.apply(grid, cell, ecut, (0, 0, 0), c[sample], V)
    err = relerr_per_band(got[sample], ref)
    print("c2 sampled per-band rel err", err)
    assert err.max() <= TOL64
    # property at every band: Re <c_n|V c_n> / |c_n|^2 lies in [min V, max V]
    ray = np.real(np.sum(np.conj(c) * got, axis=1)) / np.sum(np.abs(c) ** 2, axis=1)
    assert ray.min() >= V.min() - 1e-12 and ray.max() <= V.max() + 1e-12


def test_g2r_r2g_vs_oracle():
    grid, cell, ecut, k = (16, 18, 20), SKEW, 12.0, (0.25, 1 / 3, 0.0)
    label(test="g2r_r2g", grid=grid)
    hkl, c, V = case(grid, cell, ecut, k, 3)
    p = vloc.Plan(grid, cell, ecut, k)
    psi = p.g2r(dev(c, torch.complex128))
    torch.cuda.synchronize()
    psi_ref = oracle.g2r(grid, cell, ecut, k, c)
    assert relerr(psi.cpu().numpy(), psi_ref) <= TOL64
    back = p.r2g(dev(psi_ref, torch.complex128))
    torch.cuda.synchronize()
    ref = oracle.r2g(grid, cell, ecut, k, psi_ref)
    assert relerr(back.cpu().numpy(), ref) <= TOL64
    assert relerr(back.cpu().numpy(), c) <= TOL64
    # Parseval on the device result
    N = np.prod(grid)
    pn = np.sum(np.abs(psi.cpu().numpy()) ** 2)
    assert abs(pn / (N * np.sum(np.abs(c) ** 2)) - 1) < 1e-13


def test_identities_on_gpu():
    grid, cell, ecut, k = (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0)
    label(test="identities", grid=grid)
    hkl, c, V = case(grid, cell, ecut, k, 6)
    p = vloc.Plan(grid, cell, ecut, k)
    N = np.prod(grid)
    assert relerr(run(p, c, np.ones(N)), c) < 1e-14
    assert relerr(run(p, c, np.full(N, 2.5)), 2.5 * c) < 1e-14
    # single plane wave through a constant potential and g2r: |psi| = 1
    d = np.zeros((1, p.npw), complex)
    d[0, 100] = 1.0
    psi = p.g2r(dev(d, torch.complex128)).cpu().numpy()
    assert np.abs(np.abs(psi) - 1).max() < 1e-13
    out = run(p, c, V)
    H = np.conj(c) @ out.T
    assert np.linalg.norm(H - H.conj().T) / np.linalg.norm(H) < 1e-13


def test_determinism_and_chunk_invariance():
    grid, cell, ecut, k = (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0)
    label(test="determinism", grid=grid)
    hkl, c, V = case(grid, cell, ecut, k, 23)
    base = run(vloc.Plan(grid, cell, ecut, k), c, V)
    assert np.array_equal(base, run(vloc.Plan(grid, cell, ecut, k), c, V))
    for kw in (dict(band_chunk=7), dict(band_chunk=1), dict(deal="contiguous"),
               dict(deal="snake", sticks_per_group=5), dict(plane_rows=5, plane_threads=128),
               dict(plane_threads=64), dict(sticks_per_group=64), dict(plane_threads=1024),
               dict(plane_threads=1024, plane_xwaves=16, plane_rows=2),
               dict(plane_threads=768, plane_xwaves=12), dict(plane_xmode=4),
               dict(plane_xmode=4, plane_threads=256)):
        got = run(vloc.Plan(grid, cell, ecut, k, **kw), c, V)
        assert np.array_equal(got, base), kw


def test_edge_cases():
    label(test="edges")
    # single plane wave sphere (only g = 0), odd grid
    p = vloc.Plan((5, 6, 4), synth.cubic_cell(), 0.3)
    assert p.npw == 1
    c = np.array([[1.5 - 0.5j], [2.0 + 0j]])
    V = np.random.default_rng(1).uniform(0, 1, 120)
    got = run(p, c, V)
    assert relerr(got, c * V.mean()) < 1e-14
    # one band, and nbands = 0 is a no-op
    grid, cell, ecut, k = (16, 18, 20), SKEW, 12.0, (0.25, 1 / 3, 0.0)
    hkl, c, V = case(grid, cell, ecut, k, 1)
    p = vloc.Plan(grid, cell, ecut, k)
    assert relerr_per_band(run(p, c, V), oracle.apply(grid, cell, ecut, k, c, V)).max() <= TOL64
    empty = torch.empty((0, p.npw), dtype=torch.complex128, device="cuda")
    out = p.apply(empty, dev(V, torch.float64))
    assert out.shape == (0, p.npw)
    # flat grid dimension of 1 (sphere confined to h = 0)
    cell1 = np.diag([0.5, 6.0, 6.0])
    p1 = vloc.Plan((1, 12, 10), cell1, 0.5 * 2.2 ** 2)
    hkl1 = p1.gvectors()
    assert np.all(hkl1[:, 0] == 0)
    c1 = synth.coefficients(hkl1, 2)
    V1 = synth.potential((1, 12, 10), 2)
    got = run(p1, c1, V1)
    ref = oracle.apply((1, 12, 10), cell1, 0.5 * 2.2 ** 2, (0, 0, 0), c1, V1)
    assert relerr_per_band(got, ref).max() <= TOL64


# ------------------------------------------------------------------ FP32

@pytest.mark.parametrize("name,grid,cell,ecut,k,nb", PARITY[:3])
def test_apply_f32_error(name, grid, cell, ecut, k, nb):
    label(test="apply_f32", name=name, grid=grid)
    hkl, c, V = case(grid, cell, ecut, k, nb)
    c32 = c.astype(np.complex64).astype(np.complex128)
    V32 = V.astype(np.float32).astype(np.float64)
    p = vloc.Plan(grid, cell, ecut, k, precision="f32")
    got = run(p, c, V)
    arith = relerr_per_band(got, oracle.apply(grid, cell, ecut, k, c32, V32))
    total = relerr_per_band(got, oracle.apply(grid, cell, ecut, k, c, V))
    print(name, "f32 arithmetic err", arith.max(), "total err", total.max())
    assert arith.max() <= TOL32 and total.max() <= TOL32


# ------------------------------------------- plane-kernel x-pass variants

XMODE_CASES = [
    ("c1", (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0), 3),
    ("ortho_k", (72, 96, 128), synth.cubic_cell(), 162.0, (0.25, 0.25, 0.0), 2),
    ("m0_80", (80, 80, 80), synth.cubic_cell(), 206.5, (0, 0, 0), 2),
]


@pytest.mark.parametrize("xmode", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,cell,ecut,k,nb", XMODE_CASES)
def test_plane_xmodes_vs_oracle(xmode, precision, name, grid, cell, ecut, k, nb):
    """Row-buffer (1), lane-quad (2) and whole-plane (3, 4) layouts of the plane kernel."""
    label(test="xmode", xmode=xmode, precision=precision, name=name, grid=grid)
    hkl, c, V = case(grid, cell, ecut, k, nb)
    p = vloc.Plan(grid, cell, ecut, k, precision=precision, plane_xmode=xmode)
    assert p.layout()["plane_xmode"] == xmode
    got = run(p, c, V)
    if precision == "f64":
        ref = oracle.apply(grid, cell, ecut, k, c, V)
        tol = TOL64
    else:
        ref = oracle.apply(grid, cell, ecut, k, c.astype(np.complex64).astype(np.complex128),
                           V.astype(np.float32).astype(np.float64))
        tol = TOL32
    err = relerr_per_band(got, ref)
    print(name, precision, "xmode", xmode, "err", err.max())
    assert err.max() <= tol


# ------------------------------------------- radix splits chosen by option

@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("split", [(12, 6, 16), (16, 16, 6), (6, 12, 8)])
def test_radix_splits_vs_oracle(split, precision):
    """Non-default L = L1 * L2 splits (run-time sized kernels) on 96^3."""
    grid, cell, ecut, k, nb = (96, 96, 96), synth.cubic_cell(), 288.0, (0, 0, 0), 2
    label(test="split", split=split, precision=precision)
    hkl, c, V = case(grid, cell, ecut, k, nb)
    p = vloc.Plan(grid, cell, ecut, k, precision=precision, split=split)
    got = run(p, c, V)
    if precision == "f64":
        ref, tol = oracle.apply(grid, cell, ecut, k, c, V), TOL64
    else:
        ref = oracle.apply(grid, cell, ecut, k, c.astype(np.complex64).astype(np.complex128),
                           V.astype(np.float32).astype(np.float64))
        tol = TOL32
    err = relerr_per_band(got, ref)
    print("split", split, precision, "err", err.max())
    assert err.max() <= tol


# ------------------------------------------- direct and scatter forms of the y pass

@pytest.mark.parametrize("precision,direct,scatter", [("f64", 1024, 512), ("f32", 512, 256)])
def test_direct_y_form_equals_scatter_form(precision, direct, scatter):
    """The plane kernel takes the y stage-A inputs straight from the prefetched
    stick values (and stores stage A' straight to S) when every thread has at
    most one y task (1024/768-thread FP64 workgroups) or two (512-thread FP32
    ones): at 96^3 that is 49 columns x 12 = 588 tasks.  With `scatter` threads
    the same plan runs the scatter/gather form.  The arithmetic is the same, so
    outputs and densities agree bit for bit; both match the oracle."""
    grid, cell, ecut, k, nb = (96, 96, 96), synth.cubic_cell(), 288.0, (0, 0, 0), 3
    label(test="direct_y", precision=precision)
    hkl, c, V = case(grid, cell, ecut, k, nb)
    # the y split given explicitly (8 x 12): otherwise the planner would swap it
    # for the smaller workgroup, so that its y tasks fit the direct form too
    pd = vloc.Plan(grid, cell, ecut, k, precision=precision, plane_threads=direct,
                   split=(0, 8, 0))
    ps = vloc.Plan(grid, cell, ecut, k, precision=precision, plane_threads=scatter,
                   split=(0, 8, 0))
    assert pd.layout()["plane_xmode"] == ps.layout()["plane_xmode"] == 3
    assert pd.layout()["L2y"] == ps.layout()["L2y"] == 12
    got_d, got_s = run(pd, c, V), run(ps, c, V)
    assert np.array_equal(got_d, got_s)
    if precision == "f64":
        ref, tol = oracle.apply(grid, cell, ecut, k, c, V), TOL64
    else:
        ref = oracle.apply(grid, cell, ecut, k, c.astype(np.complex64).astype(np.complex128),
                           V.astype(np.float32).astype(np.float64))
        tol = TOL32
    assert relerr_per_band(got_d, ref).max() <= tol
    # the density pass (direct form in FP32 only) against the scatter form
    ct = torch.complex128 if precision == "f64" else torch.complex64
    tc = torch.from_numpy(c).to("cuda", ct)
    w = torch.from_numpy(synth.band_weights(nb)).cuda()
    rd, rs = pd.density(tc, w), ps.density(tc, w)
    torch.cuda.synchronize()
    assert torch.equal(rd, rs)


# ------------------------------------------- row-block layout of the plane kernel

@pytest.mark.parametrize("R,k", [(24.0, (0, 0, 0)), (47.0, (0, 0, 0)), (24.0, (0.25, 0.25, 0.0))])
def test_rowblock_layout_vs_oracle(R, k):
    """plane_xmode 5 (FP64, 96^3): each wavefront runs one block of eight rows
    from y stage B to y stage B'; the 47-radius sphere fills 95 of 96 x-planes
    (760 y tasks on 768 threads).  The diagnostic transforms and the density
    of such a plan run the whole-plane kernel with its splits."""
    grid, cell = (96, 96, 96), synth.cubic_cell()
    ecut = synth.ecut_for_radius(R)
    label(test="rowblock", R=R, k=k)
    hkl, c, V = case(grid, cell, ecut, k, 3)
    p = vloc.Plan(grid, cell, ecut, k, plane_xmode=5)
    lay = p.layout()
    assert lay["plane_xmode"] == 5 and (lay["L1x"], lay["L2x"], lay["L1y"], lay["L2y"]) == (12, 8, 12, 8)
    got = run(p, c, V)
    err = relerr_per_band(got, oracle.apply(grid, cell, ecut, k, c, V))
    print("rowblock R", R, "k", k, "err", err.max())
    assert err.max() <= TOL64
    if R == 24.0 and k == (0, 0, 0):
        psi = p.g2r(dev(c, torch.complex128))
        w = synth.band_weights(3)
        rho = p.density(dev(c, torch.complex128), dev(w, torch.float64))
        torch.cuda.synchronize()
        psi_ref = oracle.g2r(grid, cell, ecut, k, c)
        assert relerr(psi.cpu().numpy(), psi_ref) <= TOL64
        ref = (w[:, None] * np.abs(psi_ref.reshape(3, -1)) ** 2).sum(0) / np.prod(grid)
        assert relerr(rho.cpu().numpy().ravel(), ref) <= TOL64


# ------------------------------------------- the tuner's compiled splits

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tuner_split_kernels_vs_oracle(precision):
    """Every x / y split the schedule tuner tries at 96^3 (compiled with the
    workload's zero masks) and a few at 72 x 96 x 128, against the oracle."""
    at = pytest.importorskip("paper_1601_07378_amd.autotune")
    label(test="tuner_splits", precision=precision)
    cases = [((96, 96, 96), 288.0, (0, 0, 0), sx, sy) for sx in at.plane_splits(96)
             for sy in at.plane_splits(96)]
    cases += [((72, 96, 128), 162.0, (0.25, 0, 0), sx, sy) for sx, sy in ((6, 6), (9, 12), (12, 16))]
    cell = synth.cubic_cell()
    for grid, ecut, k, sx, sy in cases:
        hkl, c, V = case(grid, cell, ecut, k, 2)
        p = vloc.Plan(grid, cell, ecut, k, precision=precision, split=(sx, sy, 0))
        got = run(p, c, V)
        if precision == "f64":
            ref, tol = oracle.apply(grid, cell, ecut, k, c, V), TOL64
        else:
            ref = oracle.apply(grid, cell, ecut, k, c.astype(np.complex64).astype(np.complex128),
                               V.astype(np.float32).astype(np.float64))
            tol = TOL32
        err = relerr_per_band(got, ref)
        print(grid, sx, sy, precision, "err", err.max(), flush=True)
        assert err.max() <= tol, (grid, sx, sy)


# --------------------------- runtime-sized kernels, by codelet class

@pytest.mark.parametrize("grid,radius,split,cls", [
    ((100, 100, 100), 25.0, (0, 0, 0), 10),   # 10 x 10 lines
    ((108, 108, 108), 27.0, (0, 0, 0), 12),   # 9 x 12
    ((120, 120, 120), 30.0, (0, 0, 0), 12),   # 10 x 12
    ((128, 128, 128), 32.0, (16, 0, 0), 16),  # x 16 x 8, not compiled for the whole plane
])
def test_runtime_sized_f32_one_workgroup_per_cu_vs_oracle(grid, radius, split, cls):
    """FP32 planes of more than 80 KB (one workgroup per CU) with no compiled
    specialisation: the application runs the runtime-sized kernel on 1024
    threads; against the oracle on FP32-rounded inputs."""
    cell, k = synth.cubic_cell(), (0.0, 0.0, 0.0)
    ecut = synth.ecut_for_radius(radius)
    label(test="runtime_sized_1024", grid=grid, split=split)
    hkl, c, V = case(grid, cell, ecut, k, 2)
    p = vloc.Plan(grid, cell, ecut, k, precision="f32", split=split)
    lay = p.layout()
    assert lay["plane_xmode"] == 3 and lay["plane_lds_bytes"] > 80 * 1024
    assert max(lay["L1x"], lay["L2x"], lay["L1y"], lay["L2y"]) <= cls
    got = run(p, c, V)
    ref = oracle.apply(grid, cell, ecut, k, c.astype(np.complex64).astype(np.complex128),
                       V.astype(np.float32).astype(np.float64))
    err = relerr_per_band(got, ref)
    print(grid, split, "f32 runtime-sized 1024 err", err.max())
    assert err.max() <= TOL32


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("grid,ecut,split,cls", [
    ((20, 24, 18), 12.0, (2, 0, 0), 10),     # x = 2 x 10, y = 4 x 6: the <= 10 class
    ((24, 24, 20), 18.0, (2, 0, 0), 12),     # x = 2 x 12: the <= 12 class
    ((32, 30, 24), 18.0, (2, 2, 0), 16),     # x = 2 x 16, y = 2 x 15: every size
])
def test_runtime_sized_classes_vs_oracle(precision, grid, ecut, split, cls):
    """Plans with no compiled specialisation run the runtime-sized plane kernel
    of the smallest codelet class that covers their largest line codelet (at
    most 10, 12 or 16 points); each class against the oracle."""
    cell, k = SKEW, (0.1, -0.2, 0.3)
    label(test="runtime_sized", grid=grid, split=split, precision=precision)
    hkl, c, V = case(grid, cell, ecut, k, 3)
    p = vloc.Plan(grid, cell, ecut, k, precision=precision, split=split)
    lay = p.layout()
    biggest = max(lay["L1x"], lay["L2x"], lay["L1y"], lay["L2y"])
    assert {10: 0, 12: 10, 16: 12}[cls] < biggest <= cls
    got = run(p, c, V)
    if precision == "f64":
        ref, tol = oracle.apply(grid, cell, ecut, k, c, V), TOL64
    else:
        ref = oracle.apply(grid, cell, ecut, k, c.astype(np.complex64).astype(np.complex128),
                           V.astype(np.float32).astype(np.float64))
        tol = TOL32
    err = relerr_per_band(got, ref)
    print(grid, split, precision, "class", cls, "err", err.max())
    assert err.max() <= tol
