"""GPU checks of the differentiable local-potential energy
E = sum_n w_n Re <c_n | V c_n> and its gradients (torch.autograd.Function over
libvloc's kernels).

References: the CPU oracle (E from oracle.apply; dE/dc = 2 w_n V c_n; dE/dV =
(1/N) sum_n w_n |psi_n|^2 from oracle.g2r; dE/dw = e_n) and central finite
differences of the GPU energy itself.  E is quadratic in c and linear in V, so
central differences have no truncation error; with h = 1e-4 the round-off is
about eps |E| / h, far below the 1e-7 relative gate."""
import numpy as np
import pytest

import oracle
import synth
from helpers import relerr, relerr_per_band

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vloc = pytest.importorskip("paper_1601_07378_amd.vloc")
ag = pytest.importorskip("paper_1601_07378_amd.autograd")

SKEW = np.array([[6.0, 0.3, -0.2], [0.5, 7.0, 0.4], [-0.3, 0.6, 6.5]])


@pytest.fixture(scope="module", autouse=True)
def _gpu(require_gpu):
    yield


def label(**kw):
    print("CASE", kw, flush=True)


def tensors(c, V, w, precision):
    ct, rt = (torch.complex128, torch.float64) if precision == "f64" else \
        (torch.complex64, torch.float32)
    tc = torch.from_numpy(np.ascontiguousarray(c)).to("cuda", ct).requires_grad_(True)
    tV = torch.from_numpy(np.ascontiguousarray(V)).to("cuda", rt).requires_grad_(True)
    tw = torch.from_numpy(np.ascontiguousarray(w)).to("cuda", torch.float64).requires_grad_(True)
    return tc, tV, tw


def oracle_refs(grid, cell, ecut, k, c, V, w):
    out = oracle.apply(grid, cell, ecut, k, c, V)
    e = np.real(np.sum(np.conj(c) * out, axis=1))
    psi = oracle.g2r(grid, cell, ecut, k, c).reshape(c.shape[0], -1)
    N = np.prod(grid)
    rho = (w[:, None] * np.abs(psi) ** 2).sum(0) / N
    return float(np.dot(w, e)), 2 * w[:, None] * out, rho, e


GRAD_CASES = [
    ("c1", (24, 24, 24), synth.cubic_cell(), 18.0, (0, 0, 0), 8),
    ("skew_k_generic", (16, 18, 20), SKEW, 12.0, (0.25, 1 / 3, 0.0), 5),
    ("ortho_k", (72, 96, 128), synth.cubic_cell(), 162.0, (0.25, 0.25, 0.0), 3),
    ("c2_96", (96, 96, 96), synth.cubic_cell(), 288.0, (0, 0, 0), 6),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,cell,ecut,k,nb", GRAD_CASES)
def test_energy_gradients_vs_oracle(precision, name, grid, cell, ecut, k, nb):
    label(test="grad_vs_oracle", name=name, precision=precision)
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, nb, k)
    V = synth.potential(grid, 4)
    w = synth.band_weights(nb)
    if precision == "f32":  # compare against the oracle on the rounded inputs
        c = c.astype(np.complex64).astype(np.complex128)
        V = V.astype(np.float32).astype(np.float64)
    plan = vloc.Plan(grid, cell, ecut, k, precision=precision)
    tc, tV, tw = tensors(c, V, w, precision)
    E = ag.local_energy(plan, tc, tV, tw)
    E.backward()
    torch.cuda.synchronize()
    E_ref, gc_ref, rho_ref, e_ref = oracle_refs(grid, cell, ecut, k, c, V, w)
    tol = 1e-12 if precision == "f64" else 3e-6
    print(name, precision, "E", E.item(), E_ref)
    assert abs(E.item() - E_ref) <= tol * abs(E_ref)
    assert relerr(tc.grad.cpu().numpy(), gc_ref) <= tol
    assert relerr(tV.grad.cpu().numpy().ravel(), rho_ref) <= tol
    assert relerr(tw.grad.cpu().numpy(), e_ref) <= tol


def test_density_is_deterministic_and_chunk_invariant():
    grid, cell, ecut = (24, 24, 24), synth.cubic_cell(), 18.0
    label(test="density_determinism")
    hkl = oracle.sphere_py(cell, ecut)
    c = torch.from_numpy(synth.coefficients(hkl, 13)).cuda()
    w = torch.from_numpy(synth.band_weights(13)).cuda()
    r1 = vloc.Plan(grid, cell, ecut).density(c, w)
    r2 = vloc.Plan(grid, cell, ecut).density(c, w)
    r3 = vloc.Plan(grid, cell, ecut, band_chunk=4).density(c, w)
    r4 = vloc.Plan(grid, cell, ecut, plane_threads=1024).density(c, w)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
    assert torch.equal(r1, r4)  # wide workgroups: same per-point order
    # chunking changes the grouping of the FP64 sums, not the value beyond rounding
    assert relerr(r3.cpu().numpy(), r1.cpu().numpy()) < 1e-14
    # density accumulates into rho and scales
    rho = torch.ones_like(r1)
    s = torch.tensor([2.5], dtype=torch.float64, device="cuda")
    vloc.Plan(grid, cell, ecut).density(c, w, scale=s, rho=rho)
    assert relerr((rho - 1).cpu().numpy(), 2.5 * r1.cpu().numpy()) < 1e-14


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,cell,ecut,k,nb", GRAD_CASES)
def test_apply_density_one_pass(precision, name, grid, cell, ecut, k, nb):
    """vloc_apply_density gives vloc_apply's output bit for bit and the density
    of vloc_density (same per-point band order), both against the oracle."""
    label(test="apply_density", name=name, precision=precision)
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, nb, k)
    V = synth.potential(grid, 4)
    w = synth.band_weights(nb)
    if precision == "f32":
        c = c.astype(np.complex64).astype(np.complex128)
        V = V.astype(np.float32).astype(np.float64)
    ct, rt = (torch.complex128, torch.float64) if precision == "f64" else \
        (torch.complex64, torch.float32)
    plan = vloc.Plan(grid, cell, ecut, k, precision=precision)
    tc = torch.from_numpy(c).to("cuda", ct)
    tV = torch.from_numpy(V).to("cuda", rt)
    tw = torch.from_numpy(w).cuda()
    out, rho = plan.apply_density(tc, tV, tw)
    ref_out = plan.apply(tc, tV)
    ref_rho = plan.density(tc, tw)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out)
    assert relerr(rho.cpu().numpy(), ref_rho.cpu().numpy()) <= 1e-15
    _, _, rho_or, _ = oracle_refs(grid, cell, ecut, k, c, V, w)
    tol = 1e-12 if precision == "f64" else 3e-6
    assert relerr(rho.cpu().numpy().ravel(), rho_or) <= tol
    # accumulates into rho (rho + rho = 2 rho exactly); the scaling call
    rho2 = rho.clone()
    plan.apply_density(tc, tV, tw, rho=rho2)
    s = torch.tensor([0.5], dtype=torch.float64, device="cuda")
    scaled = plan.scale_real(rho2, s, factor=4.0)
    torch.cuda.synchronize()
    assert torch.equal(rho2, 2.0 * rho)
    assert torch.equal(scaled, 4.0 * rho)


@pytest.mark.parametrize("ysplit", [0, 8])
def test_density_register_sums_128_f32(ysplit):
    """FP32 density at 128^3 (|G| <= 32), where the whole plane fills a CU's LDS
    and the density kernels run 1024 threads, each keeping the density sums of
    its x stage-B task over a work item (one z-plane, one band subset) in
    registers: 7 bands in launches of 5 and 2 (subsets of 3 + 2 bands, then
    1 + 1) against the oracle; the
    fused application + density equals the separate calls, and 256-thread
    workgroups (per-band sums into the partial plane, another y layout, so
    psi differs by FP32 rounding) agree to the FP32 level.  Both compiled y
    splits, 16 x 8 and 8 x 16."""
    grid, cell, ecut = (128, 128, 128), synth.cubic_cell(), 512.0
    label(test="density_registers_128_f32", ysplit=ysplit)
    hkl = oracle.sphere_py(cell, ecut)
    nb = 7
    c = synth.coefficients(hkl, nb).astype(np.complex64).astype(np.complex128)
    V = synth.potential(grid, 8).astype(np.float32).astype(np.float64)
    w = synth.band_weights(nb)
    plan = vloc.Plan(grid, cell, ecut, precision="f32", band_chunk=5, split=(0, ysplit, 0))
    lay = plan.layout()
    assert lay["plane_xmode"] == 3 and lay["plane_threads"] == 512
    assert (lay["L1x"], lay["L2x"]) == (8, 16) and lay["plane_lds_bytes"] > 80 * 1024
    assert lay["L1y"] == (ysplit or 16)
    tc = torch.from_numpy(c).to("cuda", torch.complex64)
    tV = torch.from_numpy(V).to("cuda", torch.float32)
    tw = torch.from_numpy(w).cuda()
    rho = plan.density(tc, tw)
    out, rho2 = plan.apply_density(tc, tV, tw)
    ref_out = plan.apply(tc, tV)
    p256 = vloc.Plan(grid, cell, ecut, precision="f32", band_chunk=5, plane_threads=256)
    assert p256.layout()["plane_threads"] == 256
    rho3 = p256.density(tc, tw)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out)
    assert relerr(rho2.cpu().numpy(), rho.cpu().numpy()) <= 1e-15
    psi = oracle.g2r(grid, cell, ecut, (0, 0, 0), c).reshape(nb, -1)
    rho_or = (w[:, None] * np.abs(psi) ** 2).sum(0) / np.prod(grid)
    err = relerr(rho.cpu().numpy().ravel(), rho_or)
    err3 = relerr(rho3.cpu().numpy().ravel(), rho_or)
    print("128^3 f32 density err: register sums", err, "per-band sums", err3)
    assert err <= 3e-6 and err3 <= 3e-6
    assert relerr(rho3.cpu().numpy(), rho.cpu().numpy()) <= 1e-6
    # the application itself (1024-thread whole-plane kernel) against the oracle
    err_out = relerr_per_band(ref_out.cpu().numpy().astype(np.complex128),
                              oracle.apply(grid, cell, ecut, (0, 0, 0), c, V)).max()
    print("128^3 f32 apply err", err_out)
    assert err_out <= 2e-6


def test_f32_128_k_shifted_1024_thread_kernels_vs_oracle():
    """A k-shifted 128^3 FP32 plan (64 occupied x-planes, y split 8 x 16): the
    1024-thread application kernel (direct y form, 64 x 16 y tasks) and the
    1024-thread density kernels with register sums, against the oracle."""
    grid, cell, ecut, k = (128, 128, 128), synth.cubic_cell(), 512.0, (0.25, 0.25, 0.25)
    label(test="f32_128_k_1024", k=k)
    hkl = oracle.sphere_py(cell, ecut, k)
    nb = 3
    c = synth.coefficients(hkl, nb, k).astype(np.complex64).astype(np.complex128)
    V = synth.potential(grid, 8).astype(np.float32).astype(np.float64)
    w = synth.band_weights(nb)
    plan = vloc.Plan(grid, cell, ecut, k, precision="f32")
    lay = plan.layout()
    assert lay["plane_xmode"] == 3 and lay["nxo"] == 64 and (lay["L1y"], lay["L2y"]) == (8, 16)
    tc = torch.from_numpy(c).to("cuda", torch.complex64)
    tV = torch.from_numpy(V).to("cuda", torch.float32)
    tw = torch.from_numpy(w).cuda()
    out = plan.apply(tc, tV)
    out2, rho = plan.apply_density(tc, tV, tw)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    err = relerr_per_band(out.cpu().numpy().astype(np.complex128),
                          oracle.apply(grid, cell, ecut, k, c, V)).max()
    psi = oracle.g2r(grid, cell, ecut, k, c).reshape(nb, -1)
    rho_or = (w[:, None] * np.abs(psi) ** 2).sum(0) / np.prod(grid)
    err_rho = relerr(rho.cpu().numpy().ravel(), rho_or)
    print("128^3 f32 k-shifted: apply err", err, "density err", err_rho)
    assert err <= 2e-6 and err_rho <= 3e-6


def test_density_register_sums_128_f64_parted():
    """FP64 density at 128^3 (|G| <= 32) on the parted plane (two parts of 64
    rows): the density kernels run 512 threads and keep the sums of a work
    item in registers, one x stage-B task per thread and part.  7 bands in
    launches of 5 and 2 against the oracle (1e-12); the fused application +
    density equals the separate calls; a 256-thread plan (the row-buffer
    layout, per-band sums into the partial plane) agrees to rounding."""
    grid, cell, ecut = (128, 128, 128), synth.cubic_cell(), 512.0
    label(test="density_registers_128_f64")
    hkl = oracle.sphere_py(cell, ecut)
    nb = 7
    c = synth.coefficients(hkl, nb)
    V = synth.potential(grid, 8)
    w = synth.band_weights(nb)
    plan = vloc.Plan(grid, cell, ecut, band_chunk=5)
    lay = plan.layout()
    assert lay["plane_xmode"] == 6 and lay["plane_rows"] == 64
    assert (lay["L1x"], lay["L2x"], lay["L1y"], lay["L2y"]) == (8, 16, 16, 8)
    tc = torch.from_numpy(c).cuda()
    tV = torch.from_numpy(V).cuda()
    tw = torch.from_numpy(w).cuda()
    rho = plan.density(tc, tw)
    out, rho2 = plan.apply_density(tc, tV, tw)
    ref_out = plan.apply(tc, tV)
    p256 = vloc.Plan(grid, cell, ecut, band_chunk=5, plane_threads=256)
    assert p256.layout()["plane_threads"] == 256 and p256.layout()["plane_xmode"] == 1
    rho3 = p256.density(tc, tw)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out)
    assert relerr(rho2.cpu().numpy(), rho.cpu().numpy()) <= 1e-15
    psi = oracle.g2r(grid, cell, ecut, (0, 0, 0), c).reshape(nb, -1)
    rho_or = (w[:, None] * np.abs(psi) ** 2).sum(0) / np.prod(grid)
    err = relerr(rho.cpu().numpy().ravel(), rho_or)
    err3 = relerr(rho3.cpu().numpy().ravel(), rho_or)
    print("128^3 f64 density err: register sums", err, "per-band sums", err3)
    assert err <= 1e-12 and err3 <= 1e-12
    assert relerr(rho3.cpu().numpy(), rho.cpu().numpy()) <= 1e-13


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("grid,ecut,nb", [((24, 24, 24), 0.4, 3), ((24, 24, 24), 3.0, 5),
                                          ((24, 24, 24), 18.0, 4), ((48, 48, 48), 40.0, 3),
                                          ((128, 128, 128), 512.0, 2)])
def test_band_dot_and_scale_bands_vs_numpy(precision, grid, ecut, nb):
    """The band energies and the band scaling on spheres of 1, 81, 925, 2969 and
    137,065 plane waves (every remainder of the 1024-wide steps and several
    blocks per band): Re <a_n|b_n> in FP64 against numpy on the same (rounded)
    values to 1e-13; factor * scale * w_n * x_n bit-exact, since the factor is
    rounded to the plan's precision once and each element takes one multiply."""
    label(test="band_kernels", grid=grid, npw_ecut=ecut, precision=precision)
    cell = synth.cubic_cell()
    plan = vloc.Plan(grid, cell, ecut, precision=precision)
    hkl = oracle.sphere_py(cell, ecut)
    ct, cnp, rnp = (torch.complex128, np.complex128, np.float64) if precision == "f64" else \
        (torch.complex64, np.complex64, np.float32)
    rng = np.random.default_rng(11)
    a = (rng.standard_normal((nb, hkl.shape[0])) + 1j * rng.standard_normal((nb, hkl.shape[0]))).astype(cnp)
    b = (rng.standard_normal((nb, hkl.shape[0])) + 1j * rng.standard_normal((nb, hkl.shape[0]))).astype(cnp)
    w = synth.band_weights(nb)
    ta, tb = torch.from_numpy(a).to("cuda", ct), torch.from_numpy(b).to("cuda", ct)
    e = plan.band_dot(ta, tb)
    sc = torch.tensor([0.75], dtype=torch.float64, device="cuda")
    y = plan.scale_bands(ta, w=torch.from_numpy(w).cuda(), scale=sc, factor=2.0)
    torch.cuda.synchronize()
    ref = np.real(np.sum(np.conj(a.astype(np.complex128)) * b.astype(np.complex128), axis=1))
    assert np.max(np.abs(e.cpu().numpy() - ref) / np.abs(ref).max()) <= 1e-13
    f = (2.0 * 0.75 * w).astype(rnp)
    want = (a.real * f[:, None]) + 1j * (a.imag * f[:, None])
    assert np.array_equal(y.cpu().numpy(), want.astype(cnp))


def _energy(plan, c, V, w):
    with torch.no_grad():
        return ag.local_energy(plan, c, V, w).item()


@pytest.mark.parametrize("name,grid,cell,ecut,k,nb", [GRAD_CASES[0], GRAD_CASES[2]])
def test_finite_differences_16_directions(name, grid, cell, ecut, k, nb):
    """Central differences, h = 1e-4, FP64, 16 random directions in c and in V."""
    label(test="fd", name=name)
    hkl = oracle.sphere_py(cell, ecut, k)
    c = synth.coefficients(hkl, nb, k)
    V = synth.potential(grid, 4)
    w = synth.band_weights(nb)
    plan = vloc.Plan(grid, cell, ecut, k)
    tc, tV, tw = tensors(c, V, w, "f64")
    E = ag.local_energy(plan, tc, tV, tw)
    E.backward()
    gc, gV = tc.grad.detach(), tV.grad.detach()
    rng = np.random.default_rng(77)
    h = 1e-4
    for i in range(16):
        d = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
        td = torch.from_numpy(d).cuda()
        fd = (_energy(plan, tc.detach() + h * td, tV.detach(), tw.detach()) -
              _energy(plan, tc.detach() - h * td, tV.detach(), tw.detach())) / (2 * h)
        an = torch.sum(torch.real(torch.conj(gc) * td)).item()
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (i, fd, an)
        u = torch.from_numpy(rng.standard_normal(V.shape)).cuda()
        fdv = (_energy(plan, tc.detach(), tV.detach() + h * u, tw.detach()) -
               _energy(plan, tc.detach(), tV.detach() - h * u, tw.detach())) / (2 * h)
        anv = torch.sum(gV * u).item()
        assert abs(fdv - anv) <= 1e-7 * max(1.0, abs(anv)), (i, fdv, anv)


def test_grad_128_r32_512_bands_f32_with_f64_check():
    """128^3, |G| <= 32 (137,065 PW), 512 bands: FP32 energy and gradients (FP64
    reductions) against the FP64 path on the GPU; the FP64 path against the
    oracle on sampled bands; central differences (h = 1e-4, FP64) on 16 random
    directions in c and 16 in V, drawn on the device."""
    w_ = synth.WORKLOADS["c5_128"]
    grid, cell, ecut = w_["grid"], synth.cubic_cell(), synth.ecut_for_radius(w_["R"])
    nb = w_["nbands"]
    label(test="grad128", grid=grid, nb=nb)
    hkl = oracle.sphere_py(cell, ecut)
    assert hkl.shape[0] == 137065
    c = synth.coefficients(hkl, nb)
    V = synth.potential(grid, w_["ngauss"])
    w = synth.band_weights(nb)
    res = {}
    for prec in ("f64", "f32"):
        plan = vloc.Plan(grid, cell, ecut, precision=prec)
        tc, tV, tw = tensors(c, V, w, prec)
        E = ag.local_energy(plan, tc, tV, tw)
        E.backward()
        torch.cuda.synchronize()
        res[prec] = (E.item(), tc.grad.cpu().numpy().astype(np.complex128),
                     tV.grad.cpu().numpy().astype(np.float64).ravel(), plan, tc, tV, tw)
        del E
    E64, gc64, gV64 = res["f64"][:3]
    E32, gc32, gV32 = res["f32"][:3]
    errE, errc, errV = abs(E32 - E64) / abs(E64), relerr(gc32, gc64), relerr(gV32, gV64)
    print("128^3 f32 vs f64: E", errE, "grad_c", errc, "grad_V", errV)
    assert errE < 1e-5 and errc < 5e-6 and errV < 5e-6
    sample = [0, 255, 511]
    out = oracle.apply(grid, cell, ecut, (0, 0, 0), c[sample], V)
    assert relerr(gc64[sample], 2 * w[sample, None] * out) < 1e-12
    # FD (FP64) on 16 random directions in c and 16 in V, drawn on the device
    plan, tc, tV, tw = res["f64"][3:]
    gc_d = tc.grad.detach()
    gV_d = tV.grad.detach()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    h = 1e-4
    for i in range(16):
        d = torch.complex(torch.randn(c.shape, generator=gen, device="cuda", dtype=torch.float64),
                          torch.randn(c.shape, generator=gen, device="cuda", dtype=torch.float64))
        fd = (_energy(plan, tc.detach() + h * d, tV.detach(), tw.detach()) -
              _energy(plan, tc.detach() - h * d, tV.detach(), tw.detach())) / (2 * h)
        an = torch.sum(torch.real(torch.conj(gc_d) * d)).item()
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (i, fd, an)
        u = torch.randn(V.shape, generator=gen, device="cuda", dtype=torch.float64)
        fdv = (_energy(plan, tc.detach(), tV.detach() + h * u, tw.detach()) -
               _energy(plan, tc.detach(), tV.detach() - h * u, tw.detach())) / (2 * h)
        anv = torch.sum(gV_d * u).item()
        assert abs(fdv - anv) <= 1e-7 * max(1.0, abs(anv)), (i, fdv, anv)
