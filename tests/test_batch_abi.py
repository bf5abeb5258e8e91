"""Host-side checks of batches (several k-points in one launch per kernel):
members' spheres, stick tables and deals against the oracle's independent
enumeration, the shared plane layout, and argument validation before any
device work.  CPU only."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

vloc = pytest.importorskip("paper_1601_07378_amd.vloc")

C4 = synth.BATCH_WORKLOADS["c4_kpts"]


def c4_batch(**kw):
    return vloc.Batch(C4["grid"], synth.cubic_cell(), synth.ecut_for_radius(C4["R"]), C4["kpts"],
                      **kw)


def test_members_match_oracle_and_share_layout():
    b = c4_batch()
    cell, ecut = synth.cubic_cell(), synth.ecut_for_radius(C4["R"])
    counts = []
    for p, k in zip(b.plans, C4["kpts"]):
        ref = oracle.sphere_py(cell, ecut, k)
        assert np.array_equal(p.gvectors(), ref)
        st_ref = oracle.sticks(ref)
        assert np.array_equal(p.sticks().astype(np.int64), st_ref)
        g_ref, _ = oracle.greedy_deal(st_ref[:, 3], p.balance().size, "cyclic")
        assert np.array_equal(p.stick_groups(), g_ref)
        counts.append((p.npw, st_ref.shape[0]))
    # plane-wave and stick counts of the four shifted spheres
    assert counts == [(24405, 1009), (24408, 1012), (24371, 1015), (24420, 1015)]
    # whole-plane layout: every member keeps its own occupied x-planes and is
    # laid out as a stand-alone plan of its k
    lays = [p.layout() for p in b.plans]
    assert [l["nxo"] for l in lays] == [37, 36, 36, 36]
    assert all(l["plane_xmode"] == 3 for l in lays)
    for l, k in zip(lays, C4["kpts"]):
        assert l == vloc.Plan(C4["grid"], cell, ecut, k).layout()
    assert b.info() == dict(nk=4, band_chunk=0, graphs_captured=0, graph_launches=0)
    # row buffers size LDS by the occupied range: members cover the union
    br = c4_batch(plane_xmode=1)
    lays = [p.layout() for p in br.plans]
    assert all(l == lays[0] for l in lays) and lays[0]["nxo"] == 37
    assert vloc.Plan(C4["grid"], cell, ecut, C4["kpts"][1], plane_xmode=1).layout()["nxo"] == 36


def test_batch_create_validation():
    L = vloc.lib()
    h = ctypes.c_void_p()
    g = np.array(C4["grid"], dtype=np.int32)
    cell = np.ascontiguousarray(synth.cubic_cell().reshape(9))
    k = np.zeros((9, 3))
    for nk in (0, 9, -1):
        s = L.vloc_batch_create(ctypes.byref(h), vloc._i32(g), vloc._f64(cell), 162.0, nk,
                                vloc._f64(k), None)
        assert s == vloc.VLOC_E_INVALID and h.value is None
    assert L.vloc_batch_create(ctypes.byref(h), vloc._i32(g), vloc._f64(cell), 162.0, 2, None,
                               None) == vloc.VLOC_E_INVALID
    # a member whose sphere aliases fails the whole batch
    s = L.vloc_batch_create(ctypes.byref(h), vloc._i32(g), vloc._f64(cell), 0.5 * 40 ** 2, 1,
                            vloc._f64(k), None)
    assert s == vloc.VLOC_E_SPHERE and h.value is None
    assert L.vloc_batch_destroy(None) == vloc.VLOC_OK
    b = c4_batch()
    # members are borrowed: destroying one directly is refused
    assert L.vloc_plan_destroy(b.plans[0]._h) == vloc.VLOC_E_INVALID
    p = ctypes.c_void_p()
    assert L.vloc_batch_plan(b._h, 4, ctypes.byref(p)) == vloc.VLOC_E_INVALID


def test_batch_apply_validation_before_device():
    """Checks that return before any HIP call; pointers are never dereferenced."""
    L = vloc.lib()
    b = c4_batch()
    npw = [p.npw for p in b.plans]
    V = ctypes.c_void_p(0x70000000)
    base = [0x10000000 * (i + 1) for i in range(4)]
    outb = [0x08000000 + 0x10000000 * (i + 1) for i in range(4)]

    def call(nb, c=None, o=None, v=V):
        ca = (ctypes.c_void_p * 4)(*(base if c is None else c))
        oa = (ctypes.c_void_p * 4)(*(outb if o is None else o))
        na = (ctypes.c_int64 * 4)(*nb)
        return L.vloc_batch_apply(b._h, ca, na, v, oa)

    assert call([0, 0, 0, 0]) == vloc.VLOC_OK                       # no-op
    assert call([1, -1, 0, 0]) == vloc.VLOC_E_INVALID
    assert call([1, 0, 0, 0], v=None) == vloc.VLOC_E_INVALID
    assert call([1, 0, 0, 0], c=[0] + base[1:]) == vloc.VLOC_E_INVALID  # NULL c with bands
    # out of k-point 0 inside c of k-point 2
    o = list(outb)
    o[0] = base[2] + 16 * npw[2]
    assert call([1, 0, 3, 0], o=o) == vloc.VLOC_E_ALIAS
    # two outputs overlapping
    o = list(outb)
    o[1] = outb[0] + 16
    assert call([2, 2, 0, 0], o=o) == vloc.VLOC_E_ALIAS
    # out overlapping V
    o = list(outb)
    o[3] = 0x70000000 - 16
    assert call([0, 0, 0, 1], o=o) == vloc.VLOC_E_ALIAS
    # misaligned c
    c = list(base)
    c[1] += 8
    assert call([0, 1, 0, 0], c=c) == vloc.VLOC_E_INVALID
    assert L.vloc_batch_apply(None, None, None, None, None) == vloc.VLOC_E_INVALID


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_batch_apply_without_device_reports_device_error():
    L = vloc.lib()
    b = c4_batch()
    ca = (ctypes.c_void_p * 4)(0x10000000, 0, 0, 0)
    oa = (ctypes.c_void_p * 4)(0x20000000, 0, 0, 0)
    na = (ctypes.c_int64 * 4)(1, 0, 0, 0)
    assert L.vloc_batch_apply(b._h, ca, na, ctypes.c_void_p(0x40000000), oa) == vloc.VLOC_E_DEVICE
