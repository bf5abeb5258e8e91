"""Schedule autotuner for plans and batches.

The kernels have a handful of schedule knobs that the planner sets from a
cost model: the radix split L = L1 * L2 of each axis, the sticks per stick
workgroup, the plane workgroup's threads and x-pass waves, the x-pass mode,
the stick deal and the band chunk.  The tuner measures them on the device
instead: coordinate descent from the planner's choice, one knob at a time,
each candidate timed with HIP events over repeated applies (graph replays for
batches), keeping a candidate only when it beats the incumbent by a margin.
Every candidate is an ordinary plan option, so whatever the tuner picks runs
the same kernels that the tests check.

Results can be cached in a JSON file keyed by the workload and the device."""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import vloc

CODELETS = (1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32)
# Codelets of the plane kernels of more than 512 threads; the library compiles
# the whole-plane application kernel for every split of N1 and N2 into two of
# these for the plane sizes of TUNED_PLANES (with their zero masks), so the
# splits the tuner tries there run compiled code, not the run-time-sized kernel.
SMALL_CODELETS = (2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16)
TUNED_PLANES = ((96, 96), (72, 96), (128, 128))


def axis_splits(L: int) -> List[int]:
    """Every first codelet length L1 with L / L1 also a codelet length, L1 > 1 and
    L / L1 > 1 unless L itself is a codelet."""
    out = [a for a in CODELETS if L % a == 0 and (L // a) in CODELETS]
    if len(out) > 1:
        out = [a for a in out if a > 1 and L // a > 1] or out
    return out


def plane_splits(L: int) -> List[int]:
    """First factors L1 of the splits L = L1 * L2 into two codelets of at most
    16 points (those of the compiled tuner kernels)."""
    return [a for a in SMALL_CODELETS if L % a == 0 and (L // a) in SMALL_CODELETS]


def compiled_split(grid, sx: int, sy: int) -> bool:
    """True when the x and y splits of this plane size have compiled kernels
    (0 = the planner's split, which always has)."""
    if (sx == 0 and sy == 0) or tuple(grid[:2]) not in TUNED_PLANES:
        return sx == 0 and sy == 0
    return (sx == 0 or sx in plane_splits(grid[0])) and (sy == 0 or sy in plane_splits(grid[1]))


def knob_space(grid, precision: str, batch: bool, total_bands: int) -> Dict[str, list]:
    """Candidate values per knob (0 = the planner's automatic choice)."""
    chunks = [0]
    for c in (64, 128, 256, 512):
        if c < total_bands:
            chunks.append(c)
    space = {
        "split_x": [0] + plane_splits(grid[0]),
        "split_y": [0] + plane_splits(grid[1]),
        "split_z": [0] + axis_splits(grid[2]),
        "sticks_per_group": [0, 8, 16, 24, 32, 48],
        "plane_threads": [0, 256, 384, 512] + ([768, 1024] if precision == "f64" else []),
        "plane_xwaves": [0, 2, 4],
        "plane_xmode": [0, 1, 2, 3, 4] + ([5] if precision == "f64" else []) + [6],
        "deal": ["greedy", "contiguous"],
        "band_chunk": chunks,
    }
    return space


def thread_choices(precision: str) -> List[int]:
    """Plane workgroup sizes of the compiled tuner kernels."""
    return [1024, 768] if precision == "f64" else [512]


def to_options(cfg: dict) -> dict:
    """Knob dict -> keyword options of vloc.Plan / vloc.Batch."""
    opts = {k: v for k, v in cfg.items() if not k.startswith("split_")}
    opts["split"] = (cfg.get("split_x", 0), cfg.get("split_y", 0), cfg.get("split_z", 0))
    return opts


def device_tag() -> str:
    """Architecture and compute-unit count of device 0 (e.g. 'gfx950x256').

    The marketing name is not used: it is not reported the same way in every
    process (profilers that intercept the runtime change it)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.gcnArchName.split(':')[0]}x{p.multi_processor_count}"


def _cache_key(grid, cell, ecut, kpts, nbands, precision, device=None) -> str:
    h = hashlib.sha256()
    h.update(json.dumps([list(map(int, grid)), np.asarray(cell, float).round(12).tolist(),
                         float(ecut), np.asarray(kpts, float).round(12).tolist(),
                         list(map(int, nbands)), precision,
                         device or device_tag()]).encode())
    return h.hexdigest()[:24]


class Tuner:
    """Tunes one workload: `kpts` and `nbands` are sequences (one entry per
    k-point); a single k-point is tuned as a plan unless batch=True."""

    def __init__(self, grid, cell, ecut, kpts, nbands, precision="f32",
                 batch: Optional[bool] = None, graph: bool = True, reps: int = 10,
                 margin: float = 0.02, log=None):
        import torch

        self.grid = tuple(int(g) for g in grid)
        self.cell = np.asarray(cell, dtype=np.float64)
        self.ecut = float(ecut)
        self.kpts = [tuple(float(x) for x in k) for k in kpts]
        self.nbands = [int(n) for n in nbands]
        self.precision = precision
        self.batch = (len(self.kpts) > 1) if batch is None else batch
        self.graph = graph and self.batch
        self.reps = reps
        self.margin = margin
        self.log = log or (lambda *a: None)
        self.trials: List[dict] = []
        ct, rt = (torch.complex128, torch.float64) if precision == "f64" else \
            (torch.complex64, torch.float32)
        # timing inputs: seeded normal coefficients and a positive potential
        # (the kernels' time does not depend on the values)
        probe = vloc.Batch(self.grid, self.cell, self.ecut, self.kpts, precision=precision)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1234)
        self.cs = [torch.randn((nb, p.npw), dtype=ct, device="cuda", generator=gen)
                   for p, nb in zip(probe.plans, self.nbands)]
        self.outs = [torch.empty_like(c) for c in self.cs]
        N1, N2, N3 = self.grid
        self.V = 0.5 + torch.rand((N3, N2, N1), dtype=rt, device="cuda", generator=gen)
        probe.close()

    def measure(self, cfg: dict) -> float:
        """Median ms per apply of the whole workload, or inf if the options are
        rejected by the planner."""
        import torch
        try:
            if self.batch:
                obj = vloc.Batch(self.grid, self.cell, self.ecut, self.kpts,
                                 precision=self.precision, **to_options(cfg))
                if self.graph:
                    obj.use_graph(True)
                run = lambda: obj.apply(self.cs, self.V, outs=self.outs)  # noqa: E731
            else:
                obj = vloc.Plan(self.grid, self.cell, self.ecut, self.kpts[0],
                                precision=self.precision, **to_options(cfg))
                run = lambda: obj.apply(self.cs[0], self.V, out=self.outs[0])  # noqa: E731
        except vloc.VlocError:
            return float("inf")
        stream = torch.cuda.current_stream()
        for _ in range(2):
            run()
        torch.cuda.synchronize()
        times = []
        for _ in range(self.reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        obj.close()
        return float(np.median(times))

    def tune(self, rounds: int = 2) -> dict:
        """Coordinate descent over knob_space; returns the best knob dict."""
        space = knob_space(self.grid, self.precision, self.batch, sum(self.nbands))
        if not self.batch:
            space.pop("band_chunk")
        best = {k: v[0] for k, v in space.items()}
        self.measure(best)  # warm-up: clocks and caches, not a trial
        best_t = self.measure(best)
        self.trials.append(dict(cfg=dict(best), ms=best_t))
        self.log(f"# tune start {best_t:.4f} ms")
        for _ in range(rounds):
            improved = False
            for knob, values in space.items():
                for v in values:
                    if v == best[knob]:
                        continue
                    cand = dict(best)
                    cand[knob] = v
                    t = self.measure(cand)
                    self.trials.append(dict(cfg=cand, ms=t))
                    self.log(f"#   {knob}={v}: {t:.4f} ms")
                    if t < best_t * (1.0 - self.margin):
                        best, best_t, improved = cand, t, True
                        self.log(f"# best now {best} {best_t:.4f} ms")
            if not improved:
                break
        # coupled step: every compiled (x split, y split, plane threads) triple
        # from the incumbent, since one split can favour another thread count
        if "plane_threads" in space:
            for sx in [0] + plane_splits(self.grid[0]):
                for sy in [0] + plane_splits(self.grid[1]):
                    if not compiled_split(self.grid, sx, sy):
                        continue
                    for th in thread_choices(self.precision):
                        cand = dict(best, split_x=sx, split_y=sy, plane_threads=th,
                                    plane_xmode=0)
                        if cand == best:
                            continue
                        t = self.measure(cand)
                        self.trials.append(dict(cfg=cand, ms=t, coupled=True))
                        self.log(f"#   coupled split_x={sx} split_y={sy} threads={th}: {t:.4f} ms")
                        if t < best_t * (1.0 - self.margin):
                            best, best_t = cand, t
                            self.log(f"# best now {best} {best_t:.4f} ms")
        # the incumbent's final time, measured again beside the planner's default
        self.best, self.best_ms = best, self.measure(best)
        self.default_ms = self.measure({k: v[0] for k, v in space.items()})
        return best


def tune_cached(cache_path: Optional[str], grid, cell, ecut, kpts, nbands, precision="f32",
                **kw) -> dict:
    """Tuned knobs for the workload, from the JSON cache when present there."""
    key = _cache_key(grid, cell, ecut, kpts, nbands, precision)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"]
    t = Tuner(grid, cell, ecut, kpts, nbands, precision=precision, **kw)
    t0 = time.perf_counter()
    best = t.tune()
    entry = dict(best=best, best_ms=t.best_ms, default_ms=t.default_ms,
                 trials=len(t.trials), seconds=time.perf_counter() - t0,
                 workload=dict(grid=list(map(int, grid)), ecut=float(ecut),
                               kpts=np.asarray(kpts, float).round(6).tolist(),
                               nbands=list(map(int, nbands)), precision=precision),
                 device=device_tag(),
                 log=[dict(cfg=tr["cfg"], ms=round(tr["ms"], 4),
                           compiled=compiled_split(grid, tr["cfg"].get("split_x", 0),
                                                   tr["cfg"].get("split_y", 0)))
                      for tr in t.trials])
    if cache_path:
        cache[key] = entry
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return best


def main(argv=None):
    """Tune one workload on the current GPU and store the pick in a JSON cache:

        python -m paper_1601_07378_amd.autotune --grid 72 96 128 --radius 18 \
            --kpts 0 0 0 0.25 0 0 --nbands 64 128 --precision f32 --cache tune.json

    The cell is the cubic 2 pi I cell (grid-index units), so the sphere is
    |g + k| <= radius."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, nargs=3, required=True)
    ap.add_argument("--radius", type=float, required=True)
    ap.add_argument("--kpts", type=float, nargs="+", default=[0.0, 0.0, 0.0])
    ap.add_argument("--nbands", type=int, nargs="+", required=True)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f32")
    ap.add_argument("--cache", required=True)
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args(argv)
    kpts = np.asarray(a.kpts, dtype=np.float64).reshape(-1, 3)
    if len(a.nbands) != kpts.shape[0]:
        ap.error("one band count per k-point")
    cell = np.eye(3) * 2.0 * np.pi
    best = tune_cached(a.cache, a.grid, cell, 0.5 * a.radius ** 2, kpts, a.nbands,
                       precision=a.precision, reps=a.reps,
                       log=lambda *m: print(*m, flush=True))
    print(json.dumps(best))


if __name__ == "__main__":
    main()
