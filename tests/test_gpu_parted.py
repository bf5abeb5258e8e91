"""GPU parity of the parted-plane layout of the plane kernel (plane_xmode 6):
the occupied columns for the y pass, the x pass in parts of N2 / P rows
through one row buffer, the other parts in a per-workgroup device scratch.

Forced on small grids (every part count the planner allows, FP64 and FP32,
skewed cells and k-shifts, the diagnostic transforms, the density, the real
mode, batches and the allocation-free entry point), and the default layout of
the 128^3 FP64 plans, all against the CPU oracle.  FP64 gate
1e-12 per band; FP32 2e-6 against the oracle on FP32-rounded inputs."""
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


def types(precision):
    return (torch.complex128, torch.float64) if precision == "f64" else \
        (torch.complex64, torch.float32)


def label(**kw):
    print("CASE", kw, flush=True)


def reference(grid, cell, ecut, k, c, V, precision):
    if precision == "f32":
        c = c.astype(np.complex64).astype(np.complex128)
        V = V.astype(np.float32).astype(np.float64)
    return oracle.apply(grid, cell, ecut, k, c, V)


# (name, grid, cell, ecut, k, bands, rows per part): every part count of the
# 24^3 plan (y split 6 x 4: 12, 8, 4 rows), a skewed k-shifted ragged grid
# (y split 6 x 3), radix 5 (y split 6 x 5), a sphere that fills 23 of 24
# x-planes, and the orthorhombic k-point grid (y split 12 x 8)
CASES = [
    ("c1_p2", (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0), 5, 12),
    ("c1_p3", (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0), 5, 8),
    ("c1_p6", (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0), 5, 4),
    ("skew_k", (16, 18, 20), SKEW, 12.0, (0.25, 1 / 3, 0.0), 4, 6),
    ("radix5", (40, 30, 50), synth.cubic_cell(), 0.5 * 9.5 ** 2, (0, 0, 0), 3, 10),
    ("near_max", (24, 24, 24), synth.cubic_cell(), 0.5 * 11.5 ** 2, (0, 0, 0), 3, 12),
    ("ortho_k", (72, 96, 128), synth.cubic_cell(), 162.0, (0.25, 0.25, 0.0), 2, 24),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,cell,ecut,k,nb,rows", CASES)
def test_parted_apply_vs_oracle(precision, name, grid, cell, ecut, k, nb, rows):
    label(test="parted_apply", name=name, precision=precision, rows=rows)
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, nb, k)
    V = synth.potential(grid, 4)
    p = vloc.Plan(grid, cell, ecut, k, precision=precision, plane_xmode=6, plane_rows=rows)
    lay = p.layout()
    assert lay["plane_xmode"] == 6 and lay["plane_rows"] == rows
    ct, rt = types(precision)
    got = p.apply(dev(c, ct), dev(V, rt))
    torch.cuda.synchronize()
    err = relerr_per_band(got.cpu().numpy().astype(np.complex128),
                          reference(grid, cell, ecut, k, c, V, precision))
    print(name, precision, "rows", rows, "err", err.max())
    assert err.max() <= (TOL64 if precision == "f64" else TOL32)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_parted_transforms_and_density(precision):
    """g2r (x pass forward only, real-space rows out), r2g (rows in, reverse
    passes), the density and the fused application + density of a parted plan."""
    grid, cell, ecut, k = (16, 18, 20), SKEW, 12.0, (0.25, 1 / 3, 0.0)
    label(test="parted_transforms", precision=precision)
    nb = 3
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, nb, k)
    V = synth.potential(grid, 4)
    w = synth.band_weights(nb)
    p = vloc.Plan(grid, cell, ecut, k, precision=precision, plane_xmode=6, plane_rows=6)
    assert p.layout()["plane_xmode"] == 6
    ct, rt = types(precision)
    tol = TOL64 if precision == "f64" else TOL32
    cr = c if precision == "f64" else c.astype(np.complex64).astype(np.complex128)
    psi = p.g2r(dev(c, ct))
    torch.cuda.synchronize()
    psi_ref = oracle.g2r(grid, cell, ecut, k, cr)
    assert relerr(psi.cpu().numpy().astype(np.complex128), psi_ref) <= tol
    back = p.r2g(dev(psi_ref, ct))
    torch.cuda.synchronize()
    assert relerr(back.cpu().numpy().astype(np.complex128),
                  oracle.r2g(grid, cell, ecut, k, psi_ref)) <= tol
    rho = p.density(dev(c, ct), dev(w, torch.float64))
    torch.cuda.synchronize()
    rho_ref = (w[:, None] * np.abs(psi_ref.reshape(nb, -1)) ** 2).sum(0) / np.prod(grid)
    assert relerr(rho.cpu().numpy().ravel(), rho_ref) <= tol
    out, rho2 = p.apply_density(dev(c, ct), dev(V, rt), dev(w, torch.float64))
    torch.cuda.synchronize()
    assert relerr_per_band(out.cpu().numpy().astype(np.complex128),
                           reference(grid, cell, ecut, k, c, V, precision)).max() <= tol
    assert relerr(rho2.cpu().numpy().ravel(), rho_ref) <= tol


def test_parted_128_default_layout_vs_oracle():
    """The default FP64 layout at 128^3 with the |G| <= 32 sphere (two parts of
    64 rows, the compiled x 8 x 16 / y 16 x 8 splits), over two band chunks."""
    grid, cell, ecut, k = (128, 128, 128), synth.cubic_cell(), 512.0, (0, 0, 0)
    label(test="parted_128")
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, 3, k)
    V = synth.potential(grid, 32)
    p = vloc.Plan(grid, cell, ecut, k, band_chunk=2)
    lay = p.layout()
    assert lay["plane_xmode"] == 6 and lay["plane_rows"] == 64
    got = p.apply(dev(c, torch.complex128), dev(V, torch.float64))
    torch.cuda.synchronize()
    err = relerr_per_band(got.cpu().numpy(), oracle.apply(grid, cell, ecut, k, c, V))
    print("128^3 parted err", err.max())
    assert err.max() <= TOL64


def test_parted_144_f32_default_layout_vs_oracle():
    """The default FP32 layout at 144^3 with the |G| <= 36 sphere: the parted
    plane on 1024 threads, runtime-sized 12 x 12 lines."""
    grid, cell, ecut, k = (144, 144, 144), synth.cubic_cell(), 648.0, (0, 0, 0)
    label(test="parted_144_f32")
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, 2, k)
    V = synth.potential(grid, 8)
    p = vloc.Plan(grid, cell, ecut, k, precision="f32")
    lay = p.layout()
    assert lay["plane_xmode"] == 6 and lay["plane_threads"] == 1024
    got = p.apply(dev(c, torch.complex64), dev(V, torch.float32))
    torch.cuda.synchronize()
    err = relerr_per_band(got.cpu().numpy().astype(np.complex128),
                          reference(grid, cell, ecut, k, c, V, "f32"))
    print("144^3 f32 parted err", err.max())
    assert err.max() <= TOL32


def test_parted_batch_and_noalloc():
    """A batch of two k-points (two segments in one launch) and the
    allocation-free entry point on a parted plan equal the plain calls."""
    grid, cell, ecut = (24, 24, 24), synth.cubic_cell(), 18.0
    kpts = [(0.0, 0.0, 0.0), (0.25, 0.0, 0.25)]
    label(test="parted_batch")
    V = synth.potential(grid, 4)
    Vd = dev(V, torch.float64)
    b = vloc.Batch(grid, cell, ecut, kpts, plane_xmode=6, plane_rows=8)
    cs, refs = [], []
    for i, k in enumerate(kpts):
        hkl = oracle.sphere_py(cell, ecut, k)
        c = synth.coefficients(hkl, 3 + i, k, ik=i)
        cs.append(dev(c, torch.complex128))
        refs.append(oracle.apply(grid, cell, ecut, k, c, V))
    outs = b.apply(cs, Vd)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert relerr_per_band(o.cpu().numpy(), r).max() <= TOL64
    p = vloc.Plan(grid, cell, ecut, kpts[1], plane_xmode=6, plane_rows=8)
    first = p.apply(cs[1], Vd)
    out = torch.empty_like(cs[1])
    p.apply_noalloc(cs[1], Vd, out)
    torch.cuda.synchronize()
    assert torch.equal(out, first)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_parted_real_mode_vs_oracle(precision):
    """The real (Gamma) mode on a parted plan: two real bands per complex
    transform through the parted plane kernel (odd band count)."""
    grid, cell, ecut = (24, 24, 24), synth.cubic_cell(), 18.0
    label(test="parted_gamma", precision=precision)
    p = vloc.Plan(grid, cell, ecut, precision=precision, gamma=True, plane_xmode=6,
                  plane_rows=8)
    assert p.layout()["plane_xmode"] == 6
    c = synth.coefficients(p.gvectors(), 5)
    V = synth.potential(grid, 4)
    ct, rt = types(precision)
    got = p.apply(dev(c, ct), dev(V, rt))
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.complex128)
    if precision == "f64":
        ref, tol = oracle.apply_gamma(grid, cell, ecut, c, V), TOL64
    else:
        ref = oracle.apply_gamma(grid, cell, ecut, c.astype(np.complex64).astype(np.complex128),
                                 V.astype(np.float32).astype(np.float64))
        tol = TOL32
    err = relerr_per_band(got, ref)
    print("parted gamma", precision, "err", err.max())
    assert err.max() <= tol
