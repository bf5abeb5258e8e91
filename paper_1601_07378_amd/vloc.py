"""Python binding of libvloc (ctypes).  Argument marshalling only: every step of
the transform runs in the HIP kernels of libvloc.so; torch is used for device
memory and the current stream.

Names follow the C ABI in include/vloc.h.  If the shared library is missing the
import fails loudly: there is no CPU fallback."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvloc.so")

VLOC_OK = 0
VLOC_E_INVALID = -1
VLOC_E_GRID = -2
VLOC_E_CELL = -3
VLOC_E_SPHERE = -4
VLOC_E_ALIAS = -5
VLOC_E_NOMEM = -6
VLOC_E_DEVICE = -7
VLOC_F64 = 0
VLOC_F32 = 1
DEALS = {"greedy": 0, "snake": 1, "contiguous": 2, "unsorted": 3}

# Every function the header declares; tests check each is exported.
EXPORTS = [
    "vloc_plan_create", "vloc_plan_create_ex", "vloc_plan_destroy", "vloc_set_stream",
    "vloc_apply", "vloc_plan_npw", "vloc_plan_gvectors", "vloc_plan_sticks",
    "vloc_plan_balance", "vloc_plan_stick_groups", "vloc_plan_layout", "vloc_g2r", "vloc_r2g",
    "vloc_status_string", "vloc_last_error", "vloc_plan_enable_timing", "vloc_plan_read_timing",
    "vloc_band_dot", "vloc_weighted_sum", "vloc_density", "vloc_scale_bands",
    "vloc_batch_create", "vloc_batch_destroy", "vloc_batch_plan", "vloc_batch_set_stream",
    "vloc_batch_apply", "vloc_batch_use_graph", "vloc_batch_enable_timing",
    "vloc_batch_read_timing", "vloc_batch_info", "vloc_apply_noalloc", "vloc_apply_density",
    "vloc_scale_real",
]


class VlocError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"vloc status {status}: {message}")
        self.status = status
        self.message = message


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("deal", ctypes.c_int32),
                ("sticks_per_group", ctypes.c_int32), ("band_chunk", ctypes.c_int32),
                ("plane_rows", ctypes.c_int32), ("plane_threads", ctypes.c_int32),
                ("plane_xwaves", ctypes.c_int32), ("plane_xmode", ctypes.c_int32),
                ("split", ctypes.c_int32 * 3), ("gamma", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -m paper_1601_07378_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "vloc_plan_create": [ctypes.POINTER(vp), i32p, dp, ctypes.c_double, dp],
        "vloc_plan_create_ex": [ctypes.POINTER(vp), i32p, dp, ctypes.c_double, dp,
                                ctypes.POINTER(Options)],
        "vloc_plan_destroy": [vp],
        "vloc_set_stream": [vp, vp],
        "vloc_apply": [vp, vp, i64, vp, vp],
        "vloc_apply_noalloc": [vp, vp, i64, vp, vp],
        "vloc_plan_npw": [vp, i64p],
        "vloc_plan_gvectors": [vp, i32p],
        "vloc_plan_sticks": [vp, i64p, i32p],
        "vloc_plan_balance": [vp, i64p, i64p],
        "vloc_plan_stick_groups": [vp, i32p],
        "vloc_plan_layout": [vp, i32p],
        "vloc_g2r": [vp, vp, i64, vp],
        "vloc_r2g": [vp, vp, i64, vp],
        "vloc_plan_enable_timing": [vp, ctypes.c_int32],
        "vloc_plan_read_timing": [vp, ctypes.POINTER(ctypes.c_double), i64p],
        "vloc_band_dot": [vp, vp, vp, i64, vp],
        "vloc_weighted_sum": [vp, vp, vp, i64, vp],
        "vloc_density": [vp, vp, i64, vp, vp, vp],
        "vloc_scale_bands": [vp, vp, i64, vp, vp, ctypes.c_double, vp],
        "vloc_apply_density": [vp, vp, i64, vp, vp, vp, vp],
        "vloc_scale_real": [vp, vp, i64, vp, ctypes.c_double, vp],
        "vloc_batch_create": [ctypes.POINTER(vp), i32p, dp, ctypes.c_double, ctypes.c_int32, dp,
                              ctypes.POINTER(Options)],
        "vloc_batch_destroy": [vp],
        "vloc_batch_plan": [vp, ctypes.c_int32, ctypes.POINTER(vp)],
        "vloc_batch_set_stream": [vp, vp],
        "vloc_batch_apply": [vp, ctypes.POINTER(vp), i64p, vp, ctypes.POINTER(vp)],
        "vloc_batch_use_graph": [vp, ctypes.c_int32],
        "vloc_batch_enable_timing": [vp, ctypes.c_int32],
        "vloc_batch_read_timing": [vp, ctypes.POINTER(ctypes.c_double), i64p],
        "vloc_batch_info": [vp, i64p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.vloc_status_string.argtypes = [ctypes.c_int]
    L.vloc_status_string.restype = ctypes.c_char_p
    L.vloc_last_error.argtypes = []
    L.vloc_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int):
    if status != VLOC_OK:
        msg = lib().vloc_last_error().decode()
        raise VlocError(status, msg or lib().vloc_status_string(status).decode())


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_options(precision: str = "f64", deal: str = "greedy", sticks_per_group: int = 0,
                 band_chunk: int = 0, plane_rows: int = 0, plane_threads: int = 0,
                 plane_xwaves: int = 0, plane_xmode: int = 0, split=(0, 0, 0),
                 gamma: bool = False) -> Options:
    """Plan options (zeros = automatic); `split` gives the first codelet length
    L1 of each axis' L = L1 * L2 split; `gamma` selects the real mode (k = 0,
    half-sphere coefficients, two bands per complex transform)."""
    if precision not in ("f64", "f32"):
        raise ValueError("precision must be 'f64' or 'f32'")
    return Options(VLOC_F64 if precision == "f64" else VLOC_F32, DEALS[deal], sticks_per_group,
                   band_chunk, plane_rows, plane_threads, plane_xwaves, plane_xmode,
                   (ctypes.c_int32 * 3)(*[int(s) for s in split]), 1 if gamma else 0)


class Plan:
    """A V_loc plan: grid (N1, N2, N3), cell rows a1..a3, E_cut (Hartree), k in
    reduced coordinates; precision 'f64' or 'f32'."""

    def __init__(self, grid, cell, ecut: float, k=(0.0, 0.0, 0.0), precision: str = "f64",
                 **options):
        self._h = ctypes.c_void_p()
        self._owner = None
        g = np.ascontiguousarray(np.asarray(grid, dtype=np.int32).reshape(3))
        c = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
        kk = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(3))
        opt = make_options(precision, **options)
        check(lib().vloc_plan_create_ex(ctypes.byref(self._h), _i32(g), _f64(c), float(ecut),
                                        _f64(kk), ctypes.byref(opt)))
        self._init_sizes(g, precision)

    def _init_sizes(self, g, precision):
        self.grid = tuple(int(x) for x in g)
        self.precision = precision
        n = ctypes.c_int64()
        check(lib().vloc_plan_npw(self._h, ctypes.byref(n)))
        self.npw = int(n.value)
        # layouts whose plane kernel runs the fused application + density
        # (whole plane: plane_xmode 3, 4, 5; parted plane: 6)
        self.whole_plane = self.layout()["plane_xmode"] >= 3

    @classmethod
    def _borrowed(cls, handle, grid, precision, owner):
        """Member plan of a batch: valid while the batch lives, never destroyed."""
        self = cls.__new__(cls)
        self._h = handle
        self._owner = owner
        self._init_sizes(grid, precision)
        return self

    def close(self):
        if self._h and self._owner is None:
            lib().vloc_plan_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- queries
    def gvectors(self) -> np.ndarray:
        out = np.empty((self.npw, 3), dtype=np.int32)
        check(lib().vloc_plan_gvectors(self._h, _i32(out)))
        return out

    def sticks(self) -> np.ndarray:
        n = ctypes.c_int64()
        check(lib().vloc_plan_sticks(self._h, ctypes.byref(n), None))
        out = np.empty((n.value, 5), dtype=np.int32)
        check(lib().vloc_plan_sticks(self._h, ctypes.byref(n), _i32(out)))
        return out

    def balance(self) -> np.ndarray:
        n = ctypes.c_int64()
        check(lib().vloc_plan_balance(self._h, ctypes.byref(n), None))
        out = np.empty(n.value, dtype=np.int64)
        check(lib().vloc_plan_balance(self._h, ctypes.byref(n),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return out

    def stick_groups(self) -> np.ndarray:
        out = np.empty(self.sticks().shape[0], dtype=np.int32)
        check(lib().vloc_plan_stick_groups(self._h, _i32(out)))
        return out

    def layout(self) -> dict:
        v = np.empty(14, dtype=np.int32)
        check(lib().vloc_plan_layout(self._h, _i32(v)))
        keys = ["L1x", "L2x", "L1y", "L2y", "L1z", "L2z", "sticks_per_group", "band_chunk",
                "plane_rows", "plane_threads", "plane_lds_bytes", "nxo", "plane_xwaves",
                "plane_xmode"]
        return dict(zip(keys, (int(x) for x in v)))

    # ---- per-kernel timing (HIP events around each launch on the plan stream)
    def enable_timing(self, on: bool = True):
        check(lib().vloc_plan_enable_timing(self._h, 1 if on else 0))

    def read_timing(self):
        """Summed ms and launch counts of (stick forward, plane, stick backward)."""
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        check(lib().vloc_plan_read_timing(self._h, ms, n))
        return list(ms), list(n)

    # ---- device work (torch tensors on the GPU)
    def _dtypes(self):
        import torch
        return (torch.complex128, torch.float64) if self.precision == "f64" else \
            (torch.complex64, torch.float32)

    def set_stream(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib().vloc_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)))

    def apply(self, c, V, out=None, stream=None):
        """out[n] = V_loc c[n]; c (nb, npw) complex, V (N3, N2, N1) real, on the GPU."""
        import torch
        ct, rt = self._dtypes()
        if c.dtype != ct or V.dtype != rt:
            raise TypeError(f"expected c {ct} and V {rt}")
        if not (c.is_cuda and V.is_cuda):
            raise ValueError("c and V must be device tensors")
        if c.dim() != 2 or c.shape[1] != self.npw or not c.is_contiguous():
            raise ValueError("c must be contiguous (nbands, npw)")
        if V.numel() != self.grid[0] * self.grid[1] * self.grid[2] or not V.is_contiguous():
            raise ValueError("V must be contiguous with N3*N2*N1 values")
        if out is None:
            out = torch.empty_like(c)
        self.set_stream(stream)
        check(lib().vloc_apply(self._h, ctypes.c_void_p(c.data_ptr()), c.shape[0],
                               ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    def apply_noalloc(self, c, V, out, stream=None):
        """As apply, through the allocation-free entry point (static device
        scratch; the plan must have run one apply first); `out` is required."""
        ct, rt = self._dtypes()
        for t, dt in ((c, ct), (out, ct), (V, rt)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"expected contiguous device tensors of {ct} / {rt}")
        if c.dim() != 2 or c.shape[1] != self.npw or out.shape != c.shape:
            raise ValueError("c and out must be (nbands, npw)")
        if V.numel() != self.grid[0] * self.grid[1] * self.grid[2]:
            raise ValueError("V must hold N3*N2*N1 values")
        self.set_stream(stream)
        check(lib().vloc_apply_noalloc(self._h, ctypes.c_void_p(c.data_ptr()), c.shape[0],
                                       ctypes.c_void_p(V.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr())))
        return out

    # ---- energy and gradient pieces (FP64 reductions)
    def _check_c(self, c, name="c"):
        ct, _ = self._dtypes()
        if c.dtype != ct or not c.is_cuda or not c.is_contiguous() or c.dim() != 2 \
                or c.shape[1] != self.npw:
            raise ValueError(f"{name} must be a contiguous device tensor (nbands, npw) of {ct}")

    @staticmethod
    def _f64(x, n, name):
        import torch
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != n:
            raise ValueError(f"{name} must be a contiguous float64 device tensor of {n} values")

    def band_dot(self, a, b, stream=None):
        """Re sum_g conj(a_n) b_n per band, float64 (nbands,)."""
        import torch
        self._check_c(a, "a")
        self._check_c(b, "b")
        e = torch.empty(a.shape[0], dtype=torch.float64, device=a.device)
        self.set_stream(stream)
        check(lib().vloc_band_dot(self._h, ctypes.c_void_p(a.data_ptr()),
                                  ctypes.c_void_p(b.data_ptr()), a.shape[0],
                                  ctypes.c_void_p(e.data_ptr())))
        return e

    def weighted_sum(self, x, w, stream=None):
        import torch
        self._f64(x, x.numel(), "x")
        self._f64(w, x.numel(), "w")
        E = torch.empty((), dtype=torch.float64, device=x.device)
        self.set_stream(stream)
        check(lib().vloc_weighted_sum(self._h, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(w.data_ptr()), x.numel(),
                                      ctypes.c_void_p(E.data_ptr())))
        return E

    def density(self, c, w, scale=None, rho=None, stream=None):
        """rho += scale (1/N) sum_n w_n |psi_n|^2 (float64 [N3, N2, N1])."""
        import torch
        self._check_c(c)
        self._f64(w, c.shape[0], "w")
        N1, N2, N3 = self.grid
        if rho is None:
            rho = torch.zeros((N3, N2, N1), dtype=torch.float64, device=c.device)
        self._f64(rho, N1 * N2 * N3, "rho")
        if scale is not None:
            self._f64(scale, 1, "scale")
        self.set_stream(stream)
        check(lib().vloc_density(self._h, ctypes.c_void_p(c.data_ptr()), c.shape[0],
                                 ctypes.c_void_p(w.data_ptr()),
                                 ctypes.c_void_p(scale.data_ptr() if scale is not None else 0),
                                 ctypes.c_void_p(rho.data_ptr())))
        return rho

    def apply_density(self, c, V, w, out=None, rho=None, stream=None):
        """out = V_loc c and rho += (1/N) sum_n w_n |psi_n|^2 in one pass;
        returns (out, rho)."""
        import torch
        ct, rt = self._dtypes()
        self._check_c(c)
        if V.dtype != rt or not V.is_cuda or not V.is_contiguous() or \
                V.numel() != self.grid[0] * self.grid[1] * self.grid[2]:
            raise ValueError("V must be a contiguous device tensor of N3*N2*N1 values")
        self._f64(w, c.shape[0], "w")
        if out is None:
            out = torch.empty_like(c)
        self._check_c(out, "out")
        N1, N2, N3 = self.grid
        if rho is None:
            rho = torch.zeros((N3, N2, N1), dtype=torch.float64, device=c.device)
        self._f64(rho, N1 * N2 * N3, "rho")
        self.set_stream(stream)
        check(lib().vloc_apply_density(self._h, ctypes.c_void_p(c.data_ptr()), c.shape[0],
                                       ctypes.c_void_p(V.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(w.data_ptr()),
                                       ctypes.c_void_p(rho.data_ptr())))
        return out, rho

    def scale_real(self, x, scale=None, factor=1.0, out=None, stream=None):
        """out = factor * scale * x for a float64 device tensor x."""
        import torch
        self._f64(x, x.numel(), "x")
        if scale is not None:
            self._f64(scale, 1, "scale")
        if out is None:
            out = torch.empty_like(x)
        self._f64(out, x.numel(), "out")
        self.set_stream(stream)
        check(lib().vloc_scale_real(self._h, ctypes.c_void_p(x.data_ptr()), x.numel(),
                                    ctypes.c_void_p(scale.data_ptr() if scale is not None else 0),
                                    float(factor), ctypes.c_void_p(out.data_ptr())))
        return out

    def scale_bands(self, x, w=None, scale=None, factor=1.0, out=None, stream=None):
        """out_n = factor * scale * w_n * x_n."""
        import torch
        self._check_c(x, "x")
        if w is not None:
            self._f64(w, x.shape[0], "w")
        if scale is not None:
            self._f64(scale, 1, "scale")
        if out is None:
            out = torch.empty_like(x)
        self.set_stream(stream)
        check(lib().vloc_scale_bands(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                     ctypes.c_void_p(w.data_ptr() if w is not None else 0),
                                     ctypes.c_void_p(scale.data_ptr() if scale is not None else 0),
                                     float(factor), ctypes.c_void_p(out.data_ptr())))
        return out

    def g2r(self, c, out=None, stream=None):
        import torch
        ct, _ = self._dtypes()
        if c.dtype != ct or not c.is_cuda or not c.is_contiguous() or c.shape[1] != self.npw:
            raise ValueError("c must be a contiguous device tensor (nbands, npw)")
        N1, N2, N3 = self.grid
        if out is None:
            out = torch.empty((c.shape[0], N3, N2, N1), dtype=ct, device=c.device)
        self.set_stream(stream)
        check(lib().vloc_g2r(self._h, ctypes.c_void_p(c.data_ptr()), c.shape[0],
                             ctypes.c_void_p(out.data_ptr())))
        return out

    def r2g(self, psi, out=None, stream=None):
        import torch
        ct, _ = self._dtypes()
        if psi.dtype != ct or not psi.is_cuda or not psi.is_contiguous():
            raise ValueError("psi must be a contiguous device tensor (nbands, N3, N2, N1)")
        if out is None:
            out = torch.empty((psi.shape[0], self.npw), dtype=ct, device=psi.device)
        self.set_stream(stream)
        check(lib().vloc_r2g(self._h, ctypes.c_void_p(psi.data_ptr()), psi.shape[0],
                             ctypes.c_void_p(out.data_ptr())))
        return out


class Batch:
    """Several k-points of one crystal (same grid, cell, E_cut and options)
    applied with one launch per kernel per band chunk; members share one
    plane layout.  `kpts` is a sequence of reduced k-vectors (at most 8)."""

    def __init__(self, grid, cell, ecut: float, kpts, precision: str = "f64", **options):
        self._h = ctypes.c_void_p()
        g = np.ascontiguousarray(np.asarray(grid, dtype=np.int32).reshape(3))
        c = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
        kk = np.ascontiguousarray(np.asarray(kpts, dtype=np.float64).reshape(-1, 3))
        opt = make_options(precision, **options)
        check(lib().vloc_batch_create(ctypes.byref(self._h), _i32(g), _f64(c), float(ecut),
                                      kk.shape[0], _f64(kk), ctypes.byref(opt)))
        self.grid = tuple(int(x) for x in g)
        self.precision = precision
        self.nk = kk.shape[0]
        self.plans = []
        for i in range(self.nk):
            h = ctypes.c_void_p()
            check(lib().vloc_batch_plan(self._h, i, ctypes.byref(h)))
            self.plans.append(Plan._borrowed(h, g, precision, self))

    def close(self):
        if self._h:
            for p in self.plans:
                p._h = ctypes.c_void_p()
            lib().vloc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        v = np.empty(4, dtype=np.int64)
        check(lib().vloc_batch_info(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return dict(nk=int(v[0]), band_chunk=int(v[1]), graphs_captured=int(v[2]),
                    graph_launches=int(v[3]))

    def set_stream(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib().vloc_batch_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)))

    def use_graph(self, on: bool = True):
        check(lib().vloc_batch_use_graph(self._h, 1 if on else 0))

    def enable_timing(self, on: bool = True):
        check(lib().vloc_batch_enable_timing(self._h, 1 if on else 0))

    def read_timing(self):
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        check(lib().vloc_batch_read_timing(self._h, ms, n))
        return list(ms), list(n)

    def apply(self, cs, V, outs=None, stream=None):
        """outs[i] = V_loc cs[i] for each k-point i; cs[i] (nb_i, npw_i) complex
        device tensors (nb_i may be 0), V (N3, N2, N1) real."""
        import torch
        if len(cs) != self.nk:
            raise ValueError(f"expected {self.nk} coefficient tensors")
        ct, rt = self.plans[0]._dtypes()
        if V.dtype != rt or not V.is_cuda or not V.is_contiguous() or \
                V.numel() != self.grid[0] * self.grid[1] * self.grid[2]:
            raise ValueError("V must be a contiguous device tensor of N3*N2*N1 values")
        if outs is None:
            outs = [torch.empty_like(c) for c in cs]
        for p, c, o in zip(self.plans, cs, outs):
            for t in (c, o):
                if t.dtype != ct or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 \
                        or t.shape[1] != p.npw:
                    raise ValueError("each c / out must be a contiguous device tensor (nb, npw)")
            if o.shape[0] != c.shape[0]:
                raise ValueError("out and c band counts differ")
        cp = (ctypes.c_void_p * self.nk)(*[c.data_ptr() for c in cs])
        op = (ctypes.c_void_p * self.nk)(*[o.data_ptr() for o in outs])
        nb = (ctypes.c_int64 * self.nk)(*[c.shape[0] for c in cs])
        self.set_stream(stream)
        check(lib().vloc_batch_apply(self._h, cp, nb, ctypes.c_void_p(V.data_ptr()), op))
        return outs
