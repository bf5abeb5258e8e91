"""GPU parity at the edges of the method's domain, through the C ABI.

* spheres whose extent is N_i - 1 on every axis (the largest sphere a grid
  holds without aliasing, eq. 3 on the grid): every x position of a row is
  occupied, stick runs span almost all of N3, and at 96^3 the y pass runs in
  its scatter form (95 occupied x-planes x 12 > 1024 threads);
* skewed cells with a k-shift whose x-planes have holes in their k span;
* grid lengths that need codelets above 16 points (125, 250, 27, 25) and a z
  axis of 288;
* the 96^3 / 256-band workload in full, FP64 and FP32, every band against the
  oracle;
* a change of stream between two calls on one plan;
* an allocation failure (forced by the VLOC_TEST_FAIL_ALLOC hook) and recovery.

FP64 gate: 1e-12 norm-wise per band.  FP32: against the oracle on the
FP32-rounded inputs, 2e-6 (about log2 N roundings of 6e-8)."""
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
HOLE_A = (np.array([[4.38, 1.0686, -2.8831], [2.3836, 8.7056, -0.1596], [-2.339, 2.8047, 3.0992]]),
          39.588, (-0.3216, -0.2485, -0.2091))
HOLE_B = (np.array([[3.7123, -1.7955, 2.7501], [-0.9051, 5.5968, 2.7584],
                    [2.9182, 1.8833, 5.3089]]), 37.086, (-0.229, 0.1557, -0.141))


@pytest.fixture(scope="module", autouse=True)
def _gpu(require_gpu):
    yield


def label(**kw):
    print("CASE", kw, flush=True)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def run(plan, c, V):
    ct, rt = (torch.complex128, torch.float64) if plan.precision == "f64" else \
        (torch.complex64, torch.float32)
    out = plan.apply(dev(c, ct), dev(V, rt))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


def check(plan, grid, cell, ecut, k, c, V, precision):
    got = run(plan, c, V)
    if precision == "f64":
        ref, tol = oracle.apply(grid, cell, ecut, k, c, V), TOL64
    else:
        ref = oracle.apply(grid, cell, ecut, k, c.astype(np.complex64).astype(np.complex128),
                           V.astype(np.float32).astype(np.float64))
        tol = TOL32
    err = relerr_per_band(got, ref)
    print("max per-band rel err", err.max(), flush=True)
    assert err.max() <= tol
    return got


def extent(hkl):
    return tuple(int(x) for x in hkl.max(0) - hkl.min(0) + 1)


# ------------------------------------------------------- near-maximal spheres

MAXIMAL = [
    ("24_R11", (24, 24, 24), 11.0, 3),
    ("96_R47", (96, 96, 96), 47.0, 2),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,R,nb", MAXIMAL)
def test_maximal_sphere_apply(name, grid, R, nb, precision):
    cell, ecut, k = synth.cubic_cell(), synth.ecut_for_radius(R), (0, 0, 0)
    label(test="maximal_apply", name=name, precision=precision)
    hkl = oracle.sphere_py(cell, ecut, k)
    assert extent(hkl) == tuple(n - 1 for n in grid)
    c = synth.coefficients(hkl, nb)
    V = synth.potential(grid, 8)
    p = vloc.Plan(grid, cell, ecut, k, precision=precision)
    assert p.layout()["nxo"] == grid[0] - 1
    check(p, grid, cell, ecut, k, c, V, precision)


@pytest.mark.parametrize("xmode", [1, 3])
def test_maximal_sphere_shifted_k_layouts(xmode):
    """A k-shifted sphere of extent N - 1 (it reaches one side further), in the
    row-buffer (1) and whole-plane (3) layouts."""
    grid, cell, k = (24, 24, 24), synth.cubic_cell(), (0.25, 0.25, 0.0)
    ecut = synth.ecut_for_radius(11.3)
    label(test="maximal_k", xmode=xmode)
    hkl = oracle.sphere_py(cell, ecut, k)
    assert extent(hkl) == (23, 23, 23)
    c = synth.coefficients(hkl, 3, k)
    V = synth.potential(grid, 8)
    p = vloc.Plan(grid, cell, ecut, k, plane_xmode=xmode)
    check(p, grid, cell, ecut, k, c, V, "f64")


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,R,nb", MAXIMAL)
def test_maximal_sphere_gamma(name, grid, R, nb, precision):
    cell, ecut = synth.cubic_cell(), synth.ecut_for_radius(R)
    label(test="maximal_gamma", name=name, precision=precision)
    full = oracle.sphere_py(cell, ecut)
    half = full[oracle.half_mask(full)]
    c = synth.coefficients(half, 2 * nb + 1)
    c[:, 0] = c[:, 0].real  # g = 0 is the first point of the half sphere
    V = synth.potential(grid, 8)
    p = vloc.Plan(grid, cell, ecut, precision=precision, gamma=True)
    assert np.array_equal(p.gvectors(), half)
    got = run(p, c, V)
    if precision == "f64":
        ref, tol = oracle.apply_gamma(grid, cell, ecut, c, V), TOL64
    else:
        ref = oracle.apply_gamma(grid, cell, ecut, c.astype(np.complex64).astype(np.complex128),
                                 V.astype(np.float32).astype(np.float64))
        tol = TOL32
    err = relerr_per_band(got, ref)
    print(name, precision, "gamma err", err.max())
    assert err.max() <= tol


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,R,nb", MAXIMAL)
def test_maximal_sphere_density(name, grid, R, nb, precision):
    cell, ecut = synth.cubic_cell(), synth.ecut_for_radius(R)
    label(test="maximal_density", name=name, precision=precision)
    hkl = oracle.sphere_py(cell, ecut)
    c = synth.coefficients(hkl, nb)
    w = synth.band_weights(nb)
    if precision == "f32":
        c = c.astype(np.complex64).astype(np.complex128)
    p = vloc.Plan(grid, cell, ecut, precision=precision)
    ct = torch.complex128 if precision == "f64" else torch.complex64
    rho = p.density(dev(c, ct), dev(w, torch.float64))
    torch.cuda.synchronize()
    psi = oracle.g2r(grid, cell, ecut, (0, 0, 0), c).reshape(nb, -1)
    ref = (w[:, None] * np.abs(psi) ** 2).sum(0) / np.prod(grid)
    err = relerr(rho.cpu().numpy().ravel(), ref)
    print(name, precision, "density err", err)
    assert err <= (TOL64 if precision == "f64" else 3e-6)


# ------------------------------------------------ x-planes with holes in k

HOLES = [("hole_a", (16, 30, 15), HOLE_A), ("hole_b", (15, 18, 18), HOLE_B)]


@pytest.mark.parametrize("opts", [dict(), dict(plane_threads=128), dict(plane_xmode=1),
                                  dict(precision="f32")])
@pytest.mark.parametrize("name,grid,case", HOLES)
def test_k_holes_apply(name, grid, case, opts):
    cell, ecut, k = case
    label(test="holes", name=name, opts=opts)
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, 4, k)
    V = synth.potential(grid, 4)
    p = vloc.Plan(grid, cell, ecut, k, **opts)
    check(p, grid, cell, ecut, k, c, V, opts.get("precision", "f64"))


@pytest.mark.parametrize("name,grid,case", HOLES)
def test_k_holes_g2r_density_batch(name, grid, case):
    cell, ecut, k = case
    label(test="holes_aux", name=name)
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, 3, k)
    p = vloc.Plan(grid, cell, ecut, k)
    psi = p.g2r(dev(c, torch.complex128))
    torch.cuda.synchronize()
    psi_ref = oracle.g2r(grid, cell, ecut, k, c)
    assert relerr(psi.cpu().numpy(), psi_ref) <= TOL64
    w = synth.band_weights(3)
    rho = p.density(dev(c, torch.complex128), dev(w, torch.float64))
    ref = (w[:, None] * np.abs(psi_ref.reshape(3, -1)) ** 2).sum(0) / np.prod(grid)
    assert relerr(rho.cpu().numpy().ravel(), ref) <= TOL64
    # a batch of this k-point with the opposite one (a different hole pattern)
    kpts = [k, tuple(-x for x in k)]
    b = vloc.Batch(grid, cell, ecut, kpts)
    cs, refs = [], []
    V = synth.potential(grid, 4)
    for i, kk in enumerate(kpts):
        h = oracle.sphere_py(cell, ecut, kk)
        ci = synth.coefficients(h, 2 + i, kk, ik=i)
        cs.append(dev(ci, torch.complex128))
        refs.append(oracle.apply(grid, cell, ecut, kk, ci, V))
    outs = b.apply(cs, dev(V, torch.float64))
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert relerr_per_band(o.cpu().numpy(), r).max() <= TOL64


# ----------------------------------------- lengths needing large codelets

BIG = [
    ("x125", (125, 24, 24), np.diag([5.0, 1.0, 1.0]) * 2 * np.pi, 18.0, (0, 0, 0)),
    ("x250_y27_z25", (250, 27, 25), np.diag([10.0, 1.0, 1.0]) * 2 * np.pi, 18.0, (0.1, 0, 0)),
    ("z288", (24, 24, 288), np.diag([1.0, 1.0, 12.0]) * 2 * np.pi, 18.0, (0, 0, 0.25)),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,cell,ecut,k", BIG)
def test_large_codelet_grids(name, grid, cell, ecut, k, precision):
    label(test="big_codelets", name=name, precision=precision)
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, 3, k)
    V = synth.potential(grid, 4)
    p = vloc.Plan(grid, cell, ecut, k, precision=precision)
    print(name, p.layout())
    check(p, grid, cell, ecut, k, c, V, precision)


# ------------------------------------------- the 96^3 workload in full

@pytest.fixture(scope="module")
def c2_full():
    w = synth.WORKLOADS["c2_96"]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    hkl = oracle.sphere_py(cell, ecut)
    c = synth.coefficients(hkl, w["nbands"])
    V = synth.potential(grid, w["ngauss"])
    return grid, cell, ecut, c, V


def test_c2_all_bands_f64(c2_full):
    """Every band of the 96^3 / 256-band workload in the benchmark's launch
    configuration (three chunks of 86/86/84 bands) against the oracle."""
    grid, cell, ecut, c, V = c2_full
    label(test="c2_all_f64")
    p = vloc.Plan(grid, cell, ecut)
    got = run(p, c, V)
    err = relerr_per_band(got, oracle.apply(grid, cell, ecut, (0, 0, 0), c, V))
    print("c2 f64 all bands: max", err.max(), "mean", err.mean())
    assert err.max() <= TOL64


def test_c2_all_bands_f32(c2_full):
    """The metric's FP32 column: 256 bands in two 128-band chunks, every band
    against the oracle on the FP32-rounded inputs (arithmetic error) and on the
    FP64 inputs (total error)."""
    grid, cell, ecut, c, V = c2_full
    label(test="c2_all_f32")
    p = vloc.Plan(grid, cell, ecut, precision="f32")
    assert p.layout()["band_chunk"] >= 128
    got = run(p, c, V)
    c32 = c.astype(np.complex64).astype(np.complex128)
    V32 = V.astype(np.float32).astype(np.float64)
    arith = relerr_per_band(got, oracle.apply(grid, cell, ecut, (0, 0, 0), c32, V32))
    total = relerr_per_band(got, oracle.apply(grid, cell, ecut, (0, 0, 0), c, V))
    print("c2 f32 all bands: arithmetic max", arith.max(), "total max", total.max())
    assert arith.max() <= TOL32 and total.max() <= TOL32
    # both chunks are represented
    assert arith[:128].max() > 0 and arith[128:].max() > 0


# ------------------------------------------------------- change of stream

def test_stream_change_orders_work():
    """apply on stream A, then on stream B with other inputs: the second call
    reuses the stick buffer, so B must wait for A's kernels."""
    grid, cell, ecut = (96, 96, 96), synth.cubic_cell(), 288.0
    label(test="stream_change")
    hkl = oracle.sphere_py(cell, ecut)
    c1 = synth.coefficients(hkl, 96)
    c2 = synth.coefficients(hkl, 96, ik=1)
    V = synth.potential(grid, 8)
    p = vloc.Plan(grid, cell, ecut)
    tV = dev(V, torch.float64)
    t1, t2 = dev(c1, torch.complex128), dev(c2, torch.complex128)
    ref1 = p.apply(t1, tV)
    ref2 = p.apply(t2, tV)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    o1, o2 = torch.empty_like(t1), torch.empty_like(t2)
    for _ in range(3):
        p.apply(t1, tV, out=o1, stream=sa)
        p.apply(t2, tV, out=o2, stream=sb)
        torch.cuda.synchronize()
        assert torch.equal(o1, ref1) and torch.equal(o2, ref2)


# ----------------------------------------------- allocation failure path

def test_allocation_failure_and_recovery(monkeypatch):
    """VLOC_TEST_FAIL_ALLOC=1 makes the stick-buffer allocation fail: the call
    returns VLOC_E_NOMEM, nothing leaks (device free memory is back to its
    value once the plan is destroyed), and with the variable unset the same
    plan succeeds."""
    grid, cell, ecut = (24, 24, 24), synth.cubic_cell(), 18.0
    label(test="fail_alloc")
    hkl = oracle.sphere_py(cell, ecut)
    c = synth.coefficients(hkl, 4)
    V = synth.potential(grid, 4)
    tc, tV = dev(c, torch.complex128), dev(V, torch.float64)
    out = torch.empty_like(tc)
    warm = vloc.Plan(grid, cell, ecut)
    warm.apply(tc, tV, out=out)  # loads the code objects
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    p = vloc.Plan(grid, cell, ecut)
    monkeypatch.setenv("VLOC_TEST_FAIL_ALLOC", "1")
    with pytest.raises(vloc.VlocError) as e:
        p.apply(tc, tV, out=out)
    assert e.value.status == vloc.VLOC_E_NOMEM
    torch.cuda.synchronize()
    p.close()
    free1 = torch.cuda.mem_get_info()[0]
    print("free before", free0, "after failure and destroy", free1)
    assert free1 == free0
    p = vloc.Plan(grid, cell, ecut)
    with pytest.raises(vloc.VlocError):
        p.apply(tc, tV, out=out)
    monkeypatch.delenv("VLOC_TEST_FAIL_ALLOC")
    got = p.apply(tc, tV, out=out)
    torch.cuda.synchronize()
    assert relerr_per_band(got.cpu().numpy(), oracle.apply(grid, cell, ecut, (0, 0, 0), c, V)).max() <= TOL64
