"""GPU parity of the real (gamma) mode: half-sphere coefficients, two bands
per complex transform, against the oracle's real-mode definition (expand by
c(-g) = conj c(g), apply, keep the half sphere).  FP64 <= 1e-12 per band;
FP32 <= 2e-6 against the oracle on the FP32-rounded inputs."""
import numpy as np
import pytest

import oracle
import synth
from helpers import relerr_per_band

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vloc = pytest.importorskip("paper_1601_07378_amd.vloc")

SKEW = np.array([[6.0, 0.3, -0.2], [0.5, 7.0, 0.4], [-0.3, 0.6, 6.5]])


@pytest.fixture(scope="module", autouse=True)
def _gpu(require_gpu):
    yield


def label(**kw):
    print("CASE", kw, flush=True)


def run(p, c, V):
    ct, rt = (torch.complex128, torch.float64) if p.precision == "f64" else \
        (torch.complex64, torch.float32)
    out = p.apply(torch.from_numpy(np.ascontiguousarray(c)).to("cuda", ct),
                  torch.from_numpy(V).to("cuda", rt))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


CASES = [
    ("c1", (24, 24, 24), synth.cubic_cell(), 18.0, 8, 4),
    ("c1_odd", (24, 24, 24), synth.cubic_cell(), 18.0, 7, 4),
    ("one_band", (24, 24, 24), synth.cubic_cell(), 18.0, 1, 4),
    ("skew_odd_radices", (15, 9, 10), SKEW * np.array([[1.0], [0.6], [0.7]]), 5.0, 3, 2),
    ("ortho", (72, 96, 128), synth.cubic_cell(), 162.0, 5, 8),
    ("radix5", (40, 30, 50), synth.cubic_cell(), 0.5 * 9.5 ** 2, 4, 4),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,grid,cell,ecut,nb,ng", CASES)
def test_gamma_apply_vs_oracle(precision, name, grid, cell, ecut, nb, ng):
    label(test="gamma", name=name, precision=precision, nb=nb)
    p = vloc.Plan(grid, cell, ecut, precision=precision, gamma=True)
    c = synth.coefficients(p.gvectors(), nb)
    V = synth.potential(grid, ng)
    got = run(p, c, V)
    if precision == "f64":
        ref, tol = oracle.apply_gamma(grid, cell, ecut, c, V), 1e-12
    else:
        ref = oracle.apply_gamma(grid, cell, ecut, c.astype(np.complex64).astype(np.complex128),
                                 V.astype(np.float32).astype(np.float64))
        tol = 2e-6
    err = relerr_per_band(got, ref)
    print(name, precision, "gamma max per-band err", err.max())
    assert err.max() <= tol
    # out(0) is real: exactly, since both halves of the pair are combined there
    z = np.nonzero((p.gvectors() == 0).all(axis=1))[0]
    assert np.all(got[:, z].imag == 0)


def test_gamma_c2_full_sampled_and_chunks():
    """96^3, R = 24, 256 bands in the real mode, in the default chunking and in
    odd chunks (pairs cut across launches); sampled bands against the oracle,
    and every band bitwise equal across chunkings."""
    w = synth.WORKLOADS["c2_96"]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    label(test="gamma_c2", grid=grid)
    p = vloc.Plan(grid, cell, ecut, gamma=True)
    assert p.npw == 28889
    c = synth.coefficients(p.gvectors(), w["nbands"])
    V = synth.potential(grid, w["ngauss"])
    got = run(p, c, V)
    sample = [0, 1, 100, 255]
    ref = oracle.apply_gamma(grid, cell, ecut, c[sample], V)
    err = relerr_per_band(got[sample], ref)
    print("gamma c2 sampled err", err)
    assert err.max() <= 1e-12
    p7 = vloc.Plan(grid, cell, ecut, gamma=True, band_chunk=7)
    assert np.array_equal(run(p7, c, V), got)
    # Im c(0) does not enter
    c2 = c.copy()
    z = np.nonzero((p.gvectors() == 0).all(axis=1))[0]
    c2[:, z] += 0.3j
    assert np.array_equal(run(p, c2, V), got)
